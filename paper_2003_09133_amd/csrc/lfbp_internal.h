// Internal definitions shared by the HIP kernels and the host runtime of
// liblfbp.so.  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "lfbp.h"

#if defined(__HIPCC__)
#define LFBP_HD __host__ __device__
#else
#define LFBP_HD
#endif

namespace lfbp {

// Unsigned 32-bit division by a run-time invariant divisor with one multiply-
// high, one subtract and two shifts (Granlund & Montgomery, "Division by
// invariant integers using multiplication", PLDI 1994, Fig. 4.1): exact for
// every 32-bit dividend n and every divisor d >= 1.
struct FastDiv {
    uint32_t d, m, s1, s2;
};

LFBP_HD inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;  // l = ceil(log2 d)
    FastDiv f;
    f.d = d;
    const uint64_t two32 = uint64_t(1) << 32;
    // m = floor(2^32 * (2^l - d) / d) + 1  (fits in 32 bits)
    f.m = uint32_t((two32 * ((uint64_t(1) << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
}

LFBP_HD inline uint32_t mulhi32(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return uint32_t((uint64_t(a) * b) >> 32);
#endif
}

LFBP_HD inline uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    const uint32_t t = mulhi32(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Everything a gather kernel needs about one H -> H' problem.
// Output x-row R (R = (s'*nt + t')*nx + x', W elements) is input x-row
//   ((ns-1-s')*nt + (nt-1-t'))*nx + ((x' + a(s')) mod nx)
// rotated left by rot(t') = b(t')*nz elements, with
//   a(s') = (s' - hs) mod nx,  b(t') = (t' - ht) mod ny.
struct GatherDesc {
    const void* H;
    void* Ht;
    uint64_t E;          // elements of H (and H')
    uint32_t ns, nt, nx, ny, nz;
    uint32_t W;          // ny*nz, elements per x-row
    uint32_t NB;         // ns*nt, number of blocks of nx x-rows
    uint32_t nrows;      // NB*nx
    uint32_t a_off;      // a(s') = (s' + a_off) mod nx
    uint32_t b_off;      // b(t') = (t' + b_off) mod ny
    FastDiv fnx, fny, fnt;
    // work decomposition: a work unit is rows_per_unit consecutive output x-rows
    uint32_t rows_per_unit;
    uint32_t nunits;
    uint32_t phase_in;   // (address of H  / element size) mod (16 / element size)
    uint32_t phase_out;  // (address of Ht / element size) mod (16 / element size)
    uint32_t vpr;        // WIDE: 16-byte vectors reserved per x-row
    FastDiv fvpr;
    uint32_t xcd_remap;  // 1: spread consecutive units over one XCD (one workgroup per unit)
    uint32_t pad;
};

// Kernel selection resolved by the host runtime.
struct LaunchPlan {
    int variant;        // LFBP_GATHER_DIRECT, _STAGED or _WIDE
    int threads;        // workgroup size
    int rows_in_flight; // DIRECT/STAGED: rows per wavefront step
    int vec_per_thread; // WIDE: 16-byte loads per thread per unit
    int lds_bytes;      // dynamic LDS per workgroup
    int nontemporal;    // 1 or 2
    int persistent;     // 1: workgroups loop over units; 2: one workgroup per unit
    int grid;           // workgroups launched
};

// Kernel arguments of a batched launch.  Up to kInlineProblems descriptors
// travel by value (table == nullptr); larger batches point at a device table
// of descriptors and per-XCD slot prefix sums.
constexpr uint32_t kInlineProblems = 16;

// Workgroups of a launch are dealt to the XCDs round-robin (workgroup b runs
// on XCD b mod kXcds).  A batched launch gives every XCD an even share of
// every problem: XCD x owns, of problem p's n units, the contiguous run
//   [x*(n/8) + min(x, n%8), ... + n/8 + (x < n%8)),
// and walks its runs problem after problem (problems sorted largest first).
// Slot (x, l) is the l-th unit of XCD x's walk.
constexpr uint32_t kXcds = 8;

LFBP_HD inline uint32_t xcd_share(uint32_t n, uint32_t x) { return n / kXcds + (x < n % kXcds ? 1u : 0u); }
LFBP_HD inline uint32_t xcd_first(uint32_t n, uint32_t x)
{
    return x * (n / kXcds) + (x < n % kXcds ? x : n % kXcds);
}

// LDS the in-place kernel can count on on every device (a pair of x-rows must
// fit; larger budgets give larger row groups).
constexpr int kInplaceMinLds = 65536;

struct BatchArgs {
    const GatherDesc* table;      // device descriptor table, or nullptr
    const uint32_t* table_xstart; // device [kXcds][count+1]: first slot of each problem in each XCD's walk
    uint32_t count;               // problems
    uint32_t nslots;              // slots b < nslots cover every unit
    uint32_t linear;              // 1: one walk over all units in launch order (row 0 of the prefix table)
    uint32_t max_rows;            // largest rows_per_unit (LDS table size)
    uint32_t nt;                  // 1: streaming stores
    uint32_t xtotal[kXcds];       // units in each XCD's walk
    GatherDesc d[kInlineProblems];
    uint32_t xstart[kXcds][kInlineProblems + 1];  // inline batches: first slot of each problem per XCD
};

// Bytes of a batched descriptor table for n problems: the descriptors, then
// the per-XCD prefix table [kXcds][n+1].
constexpr size_t batch_table_bytes(size_t n)
{
    return sizeof(GatherDesc) * n + sizeof(uint32_t) * size_t(kXcds) * (n + 1);
}

// Words written into device memory by one launch of the table-writer kernel
// (descriptor tables travel to the device as kernel arguments, so uploading
// them is stream-ordered and needs no host buffer to outlive the call).
constexpr uint32_t kPutWords = 512;

struct WordChunk {
    uint32_t* dst;
    uint32_t n;
    uint32_t pad;
    uint32_t w[kPutWords];
};

// 16-byte row-table entry of the WIDE kernels: where an input x-row starts
// (aligned down to a 16-byte vector) and by how much it rotates.
struct RowEnt {
    int64_t vbase;  // element index of the aligned vector holding the row's first element
    uint32_t lead;  // row start - vbase
    uint32_t rot;   // left rotation of the row, elements
};

}  // namespace lfbp
