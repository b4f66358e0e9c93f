// H -> H' re-arrangement kernels for gfx950 (Sec. 4, Eq. 3 with Eqs. 4-9).
//
// Index map.  With hs = (ns-1)/2, ht = (nt-1)/2 and non-negative mod,
//   H'[s'][t'][x'][y'][z] = H[ns-1-s'][nt-1-t'][(x'+a) mod nx][(y'+b) mod ny][z],
//   a = (s'-hs) mod nx,  b = (t'-ht) mod ny.
// This is Eqs. 4-9 (reflection of s and t, Eqs. 8-9; cyclic wrap of the
// extended slice index, Eq. 5; window position, Eqs. 6-7) with the periodic
// extension of Sec. 4 (Figs. 8-9) applied to every entry, so every entry of H'
// is written exactly once.  z is the contiguous axis (depth planes are
// independent, Sec. 4), so the map moves whole "x-rows" of W = ny*nz
// contiguous elements: output x-row (s',t',x') is input x-row
// (ns-1-s', nt-1-t', (x'+a) mod nx) rotated left by b*nz elements.  Row index
// work is per row (wave-uniform, or once per row in a small LDS table); per
// element only the rotation wraps.  No arithmetic touches the payloads:
// float32 and float16 both move as raw 32/16-bit words.
//
// Kernel families (all write every element of H' exactly once):
//   DIRECT  a wavefront copies whole x-rows, reading H at rotated addresses and
//           writing H' contiguously with 4/2-byte accesses.
//   STAGED  4/2-byte row loads, rotated into an LDS tile that is laid out like
//           the stretch of H' it covers, written out with aligned 16-byte
//           stores (full cache lines).
//   WIDE    as STAGED, with the rows also read as aligned 16-byte vectors (a
//           row's superset; the few elements of neighbouring rows are
//           dropped).  Its persistent form keeps the 16-byte loads of the next
//           unit in flight while the current tile is written (LDS-only
//           barriers do not drain outstanding global loads), and gives each
//           workgroup a contiguous range of units so that the cache lines two
//           consecutive units share stay in one XCD's L2.
// Each has a plain entry (descriptor by value, nothing allocated) and a
// batched entry (descriptor table in device memory, one launch for many
// problems).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <iterator>
#include <mutex>
#include <vector>

#include "lfbp.h"

#include "lfbp_internal.h"

namespace lfbp {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
union Pack16 {
    u32x4 v;
    T e[16 / sizeof(T)];
};

// Pointers into global memory.  The arrays are always addressed through
// these: a batched launch reads its descriptors with a runtime index, and a
// pointer loaded that way would otherwise be treated as generic, i.e. flat
// loads and stores, which also count against the LDS wait counter and so
// make every LDS wait wait for the outstanding stores too.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<const T> in_ptr(const GatherDesc& d)
{
    return (gptr<const T>)(d.H);
}

template <typename T>
__device__ __forceinline__ gptr<T> out_ptr(const GatherDesc& d)
{
    return (gptr<T>)(d.Ht);
}

template <typename T>
__device__ __forceinline__ void put(gptr<T> p, T v, bool nt)
{
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <typename T>
__device__ __forceinline__ void put16(gptr<T> p, u32x4 v, bool nt)
{
    gptr<u32x4> q = (gptr<u32x4>)p;
    if (nt)
        __builtin_nontemporal_store(v, q);
    else
        *q = v;
}

// Workgroup barrier ordering LDS accesses only: outstanding global loads and
// stores of the waves stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Source of output x-row R: element offset of the input x-row and its left
// rotation in elements.
__device__ __forceinline__ void row_source(const GatherDesc& d, uint32_t R, uint64_t& src, uint32_t& rot)
{
    const uint32_t O = fdiv(R, d.fnx);  // block index s'*nt + t'
    const uint32_t xo = R - O * d.nx;   // x'
    const uint32_t sp = fdiv(O, d.fnt);
    const uint32_t tp = O - sp * d.nt;
    const uint32_t ua = sp + d.a_off, ub = tp + d.b_off;
    const uint32_t a = ua - fdiv(ua, d.fnx) * d.nx;
    const uint32_t b = ub - fdiv(ub, d.fny) * d.ny;
    uint32_t xs = xo + a;
    if (xs >= d.nx) xs -= d.nx;
    src = (uint64_t(d.NB - 1 - O) * d.nx + xs) * d.W;  // block reversal (Eqs. 8-9)
    rot = b * d.nz;
}

// Unit index of workgroup b when one workgroup serves each unit: workgroups
// are dealt to the 8 XCDs round-robin, so hand each XCD a contiguous range of
// units (bijective on [0, n)).
__device__ __forceinline__ uint32_t unit_of_block(uint32_t b, uint32_t n, bool remap)
{
    if (!remap) return b;
    const uint32_t x = b & 7u, l = b >> 3, per = n >> 3, rem = n & 7u;
    return x * per + min(x, rem) + l;
}

// Emit a tile that holds H'[O0, O0+L) starting at LDS slot `lead`:
// 16-byte stores at 16-byte aligned addresses, partial vectors at the ends
// element by element.
template <typename T>
__device__ __forceinline__ void emit_tile(const GatherDesc& d, uint64_t O0, uint32_t L, uint32_t lead, const T* tile,
                                          bool nt)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const gptr<T> out = out_ptr<T>(d);
    const uint64_t g0 = O0 + d.phase_out;
    const uint64_t u0 = g0 / VE, u1 = (g0 + L + VE - 1) / VE;
    for (uint64_t u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
        const uint32_t li = uint32_t((u - u0) * VE);     // LDS index of the vector
        const int64_t rel = int64_t(li) - int64_t(lead);  // position in the unit
        if (rel >= 0 && rel + VE <= L) {
            put16<T>(out + (O0 + rel), *reinterpret_cast<const u32x4*>(tile + li), nt);
        } else {
#pragma unroll
            for (uint32_t e = 0; e < VE; ++e) {
                const int64_t p = rel + e;
                if (p >= 0 && p < int64_t(L)) put<T>(out + (O0 + p), tile[li + e], nt);
            }
        }
    }
}

// ---------------------------------------------------------------- DIRECT

// U consecutive output x-rows starting at R0, S 64-element segments per row
// per step, all U*S loads of a step in flight before the stores.
template <typename T, int S, int U>
__device__ __forceinline__ void direct_rows(const GatherDesc& d, uint32_t R0, uint32_t lane, bool nt)
{
    gptr<const T> src[U];
    gptr<T> dst[U];
    uint32_t rot[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t R = R0 + u;
        live[u] = R < d.nrows;
        const uint32_t Rc = live[u] ? R : R0;
        uint64_t so;
        row_source(d, Rc, so, rot[u]);
        src[u] = in_ptr<T>(d) + so;
        dst[u] = out_ptr<T>(d) + uint64_t(Rc) * d.W;
    }
    const uint32_t W = d.W;
    for (uint32_t base = 0; base < W; base += 64 * S) {
        T v[U][S];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const uint32_t j = base + 64 * k + lane;
                if (live[u] && j < W) {
                    uint32_t js = j + rot[u];
                    if (js >= W) js -= W;
                    v[u][k] = src[u][js];
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const uint32_t j = base + 64 * k + lane;
                if (live[u] && j < W) put<T>(dst[u] + j, v[u][k], nt);
            }
    }
}

template <typename T, int S, int U>
__device__ __forceinline__ void direct_unit(const GatherDesc& d, uint32_t unit, bool nt)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t R0 = unit * d.rows_per_unit;
    const uint32_t R1 = min(R0 + d.rows_per_unit, d.nrows);
    for (uint32_t R = R0 + wave * U; R < R1; R += nw * U) {
        if (R + U <= R1) {
            direct_rows<T, S, U>(d, R, lane, nt);
        } else {
            for (uint32_t r = R; r < R1; ++r) direct_rows<T, S, 1>(d, r, lane, nt);
        }
    }
}

// ---------------------------------------------------------------- STAGED

template <typename T, int S, int U>
__device__ __forceinline__ void staged_unit(const GatherDesc& d, uint32_t unit, T* lds, bool nt)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t W = d.W;
    const uint32_t R0 = unit * d.rows_per_unit;
    const uint32_t nr = min(d.rows_per_unit, d.nrows - R0);
    const uint64_t O0 = uint64_t(R0) * W;
    const uint32_t lead = uint32_t((O0 + d.phase_out) % VE);
    for (uint32_t r0 = wave * U; r0 < nr; r0 += nw * U) {
        gptr<const T> src[U];
        uint32_t rot[U];
        bool live[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            live[u] = r0 + u < nr;
            uint64_t so;
            row_source(d, R0 + (live[u] ? r0 + u : r0), so, rot[u]);
            src[u] = in_ptr<T>(d) + so;
        }
        for (uint32_t base = 0; base < W; base += 64 * S) {
            T v[U][S];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    const uint32_t j = base + 64 * k + lane;
                    if (live[u] && j < W) v[u][k] = src[u][j];
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    const uint32_t j = base + 64 * k + lane;
                    if (live[u] && j < W) {
                        // input element j of the row lands at output position (j - rot) mod W
                        const uint32_t jd = j >= rot[u] ? j - rot[u] : j + W - rot[u];
                        lds[lead + (r0 + u) * W + jd] = v[u][k];
                    }
                }
        }
    }
    __syncthreads();
    emit_tile<T>(d, O0, nr * W, lead, lds, nt);
    __syncthreads();
}

// ---------------------------------------------------------------- WIDE

// Row table of the unit starting at output row R0 (nr rows).
template <typename T>
__device__ __forceinline__ void wide_table(const GatherDesc& d, uint32_t R0, uint32_t nr, RowEnt* tab)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    for (uint32_t r = threadIdx.x; r < nr; r += blockDim.x) {
        uint64_t src;
        uint32_t rot;
        row_source(d, R0 + r, src, rot);
        RowEnt e;
        e.lead = uint32_t((src + d.phase_in) % VE);
        e.vbase = int64_t(src) - int64_t(e.lead);
        e.rot = rot;
        tab[r] = e;
    }
}

// Issue the 16-byte loads of a unit: slot m of thread t reads vector
// idx = t + m*blockDim of the flattened (row, vector-in-row) space.
template <typename T, int M>
__device__ __forceinline__ void wide_load(const GatherDesc& d, uint32_t nr, const RowEnt* tab, u32x4 (&v)[M])
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint32_t nvec = nr * d.vpr;
    const gptr<const T> H = in_ptr<T>(d);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const uint32_t idx = threadIdx.x + uint32_t(m) * blockDim.x;
        if (idx < nvec) {
            const uint32_t r = fdiv(idx, d.fvpr);
            const uint32_t k = idx - r * d.vpr;
            const RowEnt e = tab[r];
            if (k * VE < e.lead + d.W) {  // the vector holds part of the row
                const int64_t g = e.vbase + int64_t(k * VE);
                if (g >= 0 && uint64_t(g) + VE <= d.E) {
                    v[m] = *(gptr<const u32x4>)(H + g);
                } else {  // a vector sticking out of the array (its first or last)
                    Pack16<T> p;
#pragma unroll
                    for (uint32_t q = 0; q < VE; ++q) {
                        const int64_t gi = g + q;
                        p.e[q] = (gi >= 0 && uint64_t(gi) < d.E) ? H[gi] : T(0);
                    }
                    v[m] = p.v;
                }
            }
        }
    }
}

// Scatter the loaded vectors into the tile at their rotated output slots.
template <typename T, int M>
__device__ __forceinline__ void wide_scatter(const GatherDesc& d, uint32_t nr, const RowEnt* tab,
                                             const u32x4 (&v)[M], T* tile, uint32_t lead_out)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint32_t nvec = nr * d.vpr;
    const int32_t W = int32_t(d.W);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const uint32_t idx = threadIdx.x + uint32_t(m) * blockDim.x;
        if (idx < nvec) {
            const uint32_t r = fdiv(idx, d.fvpr);
            const uint32_t k = idx - r * d.vpr;
            const RowEnt e = tab[r];
            const int32_t j0 = int32_t(k * VE) - int32_t(e.lead);  // row position of element 0
            if (j0 < W) {
                Pack16<T> p;
                p.v = v[m];
                T* row = tile + lead_out + r * d.W;
                const int32_t rot = int32_t(e.rot);
#pragma unroll
                for (uint32_t q = 0; q < VE; ++q) {
                    const int32_t j = j0 + int32_t(q);
                    if (j >= 0 && j < W) row[j >= rot ? j - rot : j + W - rot] = p.e[q];
                }
            }
        }
    }
}

template <typename T, int M>
__device__ __forceinline__ void wide_unit(const GatherDesc& d, uint32_t unit, RowEnt* tab, T* tile, bool nt)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint32_t R0 = unit * d.rows_per_unit;
    const uint32_t nr = min(d.rows_per_unit, d.nrows - R0);
    const uint64_t O0 = uint64_t(R0) * d.W;
    const uint32_t lead = uint32_t((O0 + d.phase_out) % VE);
    wide_table<T>(d, R0, nr, tab);
    lds_barrier();
    u32x4 v[M];
    wide_load<T, M>(d, nr, tab, v);
    wide_scatter<T, M>(d, nr, tab, v, tile, lead);
    lds_barrier();
    emit_tile<T>(d, O0, nr * d.W, lead, tile, nt);
    lds_barrier();
}

// Persistent, software-pipelined walk over global units u_first,
// u_first + stride, ... below total.  get(u, desc, local) returns whether unit
// u exists, and then its descriptor and problem-local index; a unit that does
// not exist (a hole of a batched walk) is run with no rows: no load, no store.
template <typename T, int M, class Get>
__device__ __forceinline__ void wide_pipeline(uint32_t u_first, uint32_t stride, uint32_t total, Get get,
                                              RowEnt* tab0, RowEnt* tab1, T* tile, bool nt)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    if (u_first >= total) return;
    GatherDesc dc;
    uint32_t lc;
    const bool ok = get(u_first, dc, lc);
    uint32_t R0 = ok ? lc * dc.rows_per_unit : 0;
    uint32_t nr = ok ? min(dc.rows_per_unit, dc.nrows - R0) : 0;
    wide_table<T>(dc, R0, nr, tab0);
    lds_barrier();
    u32x4 v[M];
    wide_load<T, M>(dc, nr, tab0, v);
    bool flip = false;
    for (uint32_t u = u_first; u < total; u += stride) {
        RowEnt* tc = flip ? tab1 : tab0;
        RowEnt* tn = flip ? tab0 : tab1;
        flip = !flip;
        const uint64_t O0 = uint64_t(R0) * dc.W;
        const uint32_t lead = uint32_t((O0 + dc.phase_out) % VE);
        wide_scatter<T, M>(dc, nr, tc, v, tile, lead);
        GatherDesc dn;
        uint32_t ln = 0, Rn = 0, nn = 0;
        const bool more = uint64_t(u) + stride < total;
        if (more) {
            if (get(u + stride, dn, ln)) {
                Rn = ln * dn.rows_per_unit;
                nn = min(dn.rows_per_unit, dn.nrows - Rn);
            }
            wide_table<T>(dn, Rn, nn, tn);
        }
        lds_barrier();                                    // tile and next table complete
        if (more) wide_load<T, M>(dn, nn, tn, v);         // next unit's loads in flight ...
        emit_tile<T>(dc, O0, nr * dc.W, lead, tile, nt);  // ... while this tile is written
        lds_barrier();                                    // tile free again
        if (more) {
            dc = dn;
            R0 = Rn;
            nr = nn;
        }
    }
}

// First unit of workgroup b in a persistent grid of g workgroups: at every
// step the grid covers a window of g consecutive units, and each XCD
// (workgroups b = x mod 8) takes a contiguous eighth of the window.
__device__ __forceinline__ uint32_t persistent_first(uint32_t b, uint32_t g)
{
    if (g & 7u) return b;
    return (b & 7u) * (g >> 3) + (b >> 3);
}

// ---------------------------------------------------------------- entries

template <typename T, int S, int U>
__global__ void __launch_bounds__(512) k_direct(GatherDesc d, int nt)
{
    for (uint32_t unit = blockIdx.x; unit < d.nunits; unit += gridDim.x) direct_unit<T, S, U>(d, unit, nt != 0);
}

template <typename T, int S, int U>
__global__ void __launch_bounds__(512) k_staged(GatherDesc d, int nt)
{
    extern __shared__ u32x4 smem[];
    T* lds = reinterpret_cast<T*>(smem);
    for (uint32_t unit = blockIdx.x; unit < d.nunits; unit += gridDim.x) staged_unit<T, S, U>(d, unit, lds, nt != 0);
}

template <typename T, int M>
__global__ void __launch_bounds__(512) k_wide(GatherDesc d, int nt)
{
    extern __shared__ u32x4 smem[];
    RowEnt* tab = reinterpret_cast<RowEnt*>(smem);
    T* tile = reinterpret_cast<T*>(smem + d.rows_per_unit);
    for (uint32_t b = blockIdx.x; b < d.nunits; b += gridDim.x)
        wide_unit<T, M>(d, unit_of_block(b, d.nunits, d.xcd_remap && gridDim.x == d.nunits), tab, tile, nt != 0);
}

template <typename T, int M>
__global__ void __launch_bounds__(512) k_wide_persist(GatherDesc d, int nt)
{
    extern __shared__ u32x4 smem[];
    RowEnt* tab0 = reinterpret_cast<RowEnt*>(smem);
    RowEnt* tab1 = tab0 + d.rows_per_unit;
    T* tile = reinterpret_cast<T*>(smem + 2 * d.rows_per_unit);
    auto get = [&](uint32_t u, GatherDesc& dd, uint32_t& lu) {
        dd = d;
        lu = u;
        return true;
    };
    wide_pipeline<T, M>(d.xcd_remap ? persistent_first(blockIdx.x, gridDim.x) : blockIdx.x, gridDim.x, d.nunits,
                        get, tab0, tab1, tile, nt != 0);
}

// A descriptor read from a device table (word by word, through a global
// pointer).
__device__ __forceinline__ GatherDesc load_desc(gptr<const GatherDesc> p)
{
    static_assert(sizeof(GatherDesc) % 4 == 0, "descriptor is whole words");
    GatherDesc d;
    const gptr<const uint32_t> w = (gptr<const uint32_t>)p;
    uint32_t* o = reinterpret_cast<uint32_t*>(&d);
#pragma unroll
    for (uint32_t i = 0; i < sizeof(GatherDesc) / 4; ++i) o[i] = w[i];
    return d;
}

// Problem and problem-local unit of slot b of a batched launch.  In the
// XCD schedule, slot b is unit l = b / kXcds of the walk of XCD
// x = b mod kXcds (the XCD that workgroup b runs on), which takes an even
// share of every problem in turn; in the linear schedule slot b is unit b of
// one walk over all problems (row 0 of the prefix table).  The prefix table
// (first slot of each problem in each walk) travels in the kernel arguments
// with the descriptors for up to kInlineProblems problems (a branch-free
// scalar count over one row of it); larger batches use a device table
// searched by bisection.  Returns false for the slots past the end of a walk
// (d is then a valid descriptor of the batch and local 0, so that callers may
// run it with no rows).
__device__ __forceinline__ bool batch_slot(const BatchArgs& a, uint32_t b, GatherDesc& d, uint32_t& local)
{
    const uint32_t x = a.linear ? 0u : b & (kXcds - 1), l = a.linear ? b : b / kXcds;
    const gptr<const GatherDesc> table = (gptr<const GatherDesc>)a.table;
    if (l >= a.xtotal[x]) {
        d = a.table == nullptr ? a.d[0] : load_desc(table);
        local = 0;
        return false;
    }
    if (a.table == nullptr) {
        const uint32_t* xs = a.xstart[x];
        uint32_t p = 0;
#pragma unroll
        for (uint32_t i = 1; i < kInlineProblems; ++i) p += (i < a.count && xs[i] <= l) ? 1u : 0u;
        d = a.d[p];
        local = (a.linear ? 0u : xcd_first(d.nunits, x)) + (l - xs[p]);
    } else {
        const gptr<const uint32_t> xs = (gptr<const uint32_t>)a.table_xstart + size_t(x) * (a.count + 1);
        uint32_t lo = 0, hi = a.count;  // xs[lo] <= l < xs[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (xs[mid] <= l)
                lo = mid;
            else
                hi = mid;
        }
        d = load_desc(table + lo);
        local = (a.linear ? 0u : xcd_first(d.nunits, x)) + (l - xs[lo]);
    }
    return true;
}

template <typename T, int S, int U>
__global__ void __launch_bounds__(512) k_direct_batched(BatchArgs a)
{
    for (uint32_t b = blockIdx.x; b < a.nslots; b += gridDim.x) {
        GatherDesc d;
        uint32_t lu;
        if (batch_slot(a, b, d, lu)) direct_unit<T, S, U>(d, lu, a.nt != 0);
    }
}

template <typename T, int S, int U>
__global__ void __launch_bounds__(512) k_staged_batched(BatchArgs a)
{
    extern __shared__ u32x4 smem[];
    T* lds = reinterpret_cast<T*>(smem);
    for (uint32_t b = blockIdx.x; b < a.nslots; b += gridDim.x) {
        GatherDesc d;
        uint32_t lu;
        if (batch_slot(a, b, d, lu)) staged_unit<T, S, U>(d, lu, lds, a.nt != 0);
    }
}

// One workgroup per unit over all problems.
template <typename T, int M>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(M >= 8 ? 5 : 8))) k_wide_batched(BatchArgs a)
{
    extern __shared__ u32x4 smem[];
    RowEnt* tab = reinterpret_cast<RowEnt*>(smem);
    T* tile = reinterpret_cast<T*>(smem + a.max_rows);
    for (uint32_t b = blockIdx.x; b < a.nslots; b += gridDim.x) {
        GatherDesc d;
        uint32_t lu;
        if (batch_slot(a, b, d, lu)) wide_unit<T, M>(d, lu, tab, tile, a.nt != 0);
    }
}

// Persistent and pipelined over all problems (the grid is a multiple of
// kXcds, so each workgroup stays on one XCD's walk).
template <typename T, int M>
__global__ void __launch_bounds__(512) k_wide_batched_persist(BatchArgs a)
{
    extern __shared__ u32x4 smem[];
    RowEnt* tab0 = reinterpret_cast<RowEnt*>(smem);
    RowEnt* tab1 = tab0 + a.max_rows;
    T* tile = reinterpret_cast<T*>(smem + 2 * a.max_rows);
    // The arguments are read in place from the kernel-argument segment (the
    // only argument, at offset 0): a reference to the by-value parameter
    // kept across the pipelined loop would make the compiler copy all of it
    // into per-lane scratch memory.
    const BatchArgs& ka = *reinterpret_cast<const BatchArgs*>(
        reinterpret_cast<uintptr_t>(__builtin_amdgcn_kernarg_segment_ptr()));
    auto get = [&](uint32_t u, GatherDesc& dd, uint32_t& lu) { return batch_slot(ka, u, dd, lu); };
    wide_pipeline<T, M>(blockIdx.x, gridDim.x, a.nslots, get, tab0, tab1, tile, a.nt != 0);
}

// Device-side copy of up to kPutWords words carried in the kernel arguments.
__global__ void __launch_bounds__(256) k_put_words(WordChunk c)
{
    const gptr<uint32_t> dst = (gptr<uint32_t>)c.dst;
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

// ---------------------------------------------------------------- host side

namespace {

typedef void (*PlainFn)(GatherDesc, int);
typedef void (*BatchFn)(BatchArgs);

// S = 64-element segments per row loaded per step: enough to cover a row of
// W elements in one step up to W = 1024, in batches of 16 beyond that.
int segments_for(uint32_t W)
{
    const uint32_t need = (W + 63) / 64;
    return need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
}

template <typename T>
PlainFn pick_plain(const LaunchPlan& p, uint32_t W)
{
    const bool U2 = p.rows_in_flight >= 2;
    if (p.variant == LFBP_GATHER_WIDE) {
        const bool pers = p.persistent == 1;
        switch (p.vec_per_thread) {
            case 2: return pers ? k_wide_persist<T, 2> : k_wide<T, 2>;
            case 4: return pers ? k_wide_persist<T, 4> : k_wide<T, 4>;
            default: return pers ? k_wide_persist<T, 8> : k_wide<T, 8>;
        }
    }
    const bool direct = p.variant == LFBP_GATHER_DIRECT;
    switch (segments_for(W)) {
        case 2: return direct ? (U2 ? k_direct<T, 2, 2> : k_direct<T, 2, 1>) : (U2 ? k_staged<T, 2, 2> : k_staged<T, 2, 1>);
        case 4: return direct ? (U2 ? k_direct<T, 4, 2> : k_direct<T, 4, 1>) : (U2 ? k_staged<T, 4, 2> : k_staged<T, 4, 1>);
        case 8: return direct ? (U2 ? k_direct<T, 8, 2> : k_direct<T, 8, 1>) : (U2 ? k_staged<T, 8, 2> : k_staged<T, 8, 1>);
        default:
            return direct ? (U2 ? k_direct<T, 16, 2> : k_direct<T, 16, 1>) : (U2 ? k_staged<T, 16, 2> : k_staged<T, 16, 1>);
    }
}

template <typename T>
BatchFn pick_batch(const LaunchPlan& p, uint32_t W)
{
    const bool U2 = p.rows_in_flight >= 2;
    if (p.variant == LFBP_GATHER_WIDE) {
        const bool pers = p.persistent == 1;
        switch (p.vec_per_thread) {
            case 2: return pers ? k_wide_batched_persist<T, 2> : k_wide_batched<T, 2>;
            case 4: return pers ? k_wide_batched_persist<T, 4> : k_wide_batched<T, 4>;
            default: return pers ? k_wide_batched_persist<T, 8> : k_wide_batched<T, 8>;
        }
    }
    const bool direct = p.variant == LFBP_GATHER_DIRECT;
    switch (segments_for(W)) {
        case 2:
            return direct ? (U2 ? k_direct_batched<T, 2, 2> : k_direct_batched<T, 2, 1>)
                          : (U2 ? k_staged_batched<T, 2, 2> : k_staged_batched<T, 2, 1>);
        case 4:
            return direct ? (U2 ? k_direct_batched<T, 4, 2> : k_direct_batched<T, 4, 1>)
                          : (U2 ? k_staged_batched<T, 4, 2> : k_staged_batched<T, 4, 1>);
        case 8:
            return direct ? (U2 ? k_direct_batched<T, 8, 2> : k_direct_batched<T, 8, 1>)
                          : (U2 ? k_staged_batched<T, 8, 2> : k_staged_batched<T, 8, 1>);
        default:
            return direct ? (U2 ? k_direct_batched<T, 16, 2> : k_direct_batched<T, 16, 1>)
                          : (U2 ? k_staged_batched<T, 16, 2> : k_staged_batched<T, 16, 1>);
    }
}

PlainFn pick_plain_any(const LaunchPlan& p, uint32_t W, int esize)
{
    return esize == 4 ? pick_plain<uint32_t>(p, W) : pick_plain<uint16_t>(p, W);
}

BatchFn pick_batch_any(const LaunchPlan& p, uint32_t W, int esize)
{
    return esize == 4 ? pick_batch<uint32_t>(p, W) : pick_batch<uint16_t>(p, W);
}

template <typename T>
void all_lds_kernels(std::vector<const void*>& out)
{
    const void* k[] = {
        (const void*)k_staged<T, 2, 1>,       (const void*)k_staged<T, 2, 2>,       (const void*)k_staged<T, 4, 1>,
        (const void*)k_staged<T, 4, 2>,       (const void*)k_staged<T, 8, 1>,       (const void*)k_staged<T, 8, 2>,
        (const void*)k_staged<T, 16, 1>,      (const void*)k_staged<T, 16, 2>,      (const void*)k_staged_batched<T, 2, 1>,
        (const void*)k_staged_batched<T, 2, 2>,  (const void*)k_staged_batched<T, 4, 1>,
        (const void*)k_staged_batched<T, 4, 2>,  (const void*)k_staged_batched<T, 8, 1>,
        (const void*)k_staged_batched<T, 8, 2>,  (const void*)k_staged_batched<T, 16, 1>,
        (const void*)k_staged_batched<T, 16, 2>, (const void*)k_wide<T, 2>,
        (const void*)k_wide<T, 4>,            (const void*)k_wide<T, 8>,            (const void*)k_wide_persist<T, 2>,
        (const void*)k_wide_persist<T, 4>,    (const void*)k_wide_persist<T, 8>,    (const void*)k_wide_batched<T, 2>,
        (const void*)k_wide_batched<T, 4>,    (const void*)k_wide_batched<T, 8>,
        (const void*)k_wide_batched_persist<T, 2>, (const void*)k_wide_batched_persist<T, 4>,
        (const void*)k_wide_batched_persist<T, 8>,
    };
    out.insert(out.end(), std::begin(k), std::end(k));
}

}  // namespace

hipError_t launch_gather(const GatherDesc& d, int esize, const LaunchPlan& p, hipStream_t stream)
{
    PlainFn fn = pick_plain_any(p, d.W, esize);
    hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.threads), size_t(p.lds_bytes), stream, d, p.nontemporal == 1 ? 1 : 0);
    return hipGetLastError();
}

// Device scratch of lfbp_compute_Ht_batched_noalloc: the descriptor table of
// one batch of up to LFBP_NOALLOC_MAX_PROBLEMS problems, compiled into the
// library (each GPU holds its own copy until the process ends).  In host code
// `scratch` names a host-side stand-in, not device memory: kernels receive the
// device address that noalloc_scratch() looks up per device.
constexpr size_t kScratchBytes = batch_table_bytes(LFBP_NOALLOC_MAX_PROBLEMS);
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Device address of this GPU's `scratch` (the current device's), looked up
// once per device with that device current.
hipError_t noalloc_scratch(void** ptr, size_t* bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

// Write n words from host memory to device memory dst, ordered on stream:
// the words travel in the arguments of small copy kernels, so src may be
// reused as soon as this returns and the writes may be captured into a graph.
hipError_t put_words(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t stream)
{
    for (size_t i = 0; i < n; i += kPutWords) {
        WordChunk c;
        c.dst = dst + i;
        c.n = uint32_t(std::min<size_t>(kPutWords, n - i));
        c.pad = 0;
        std::memcpy(c.w, src + i, sizeof(uint32_t) * c.n);
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, stream, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_gather_batched(const BatchArgs& a, uint32_t maxW, int esize, const LaunchPlan& p,
                                 hipStream_t stream)
{
    BatchFn fn = pick_batch_any(p, maxW, esize);
    hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.threads), size_t(p.lds_bytes), stream, a);
    return hipGetLastError();
}

// Workgroups of a kernel that fit one CU at once.
int gather_occupancy(const LaunchPlan& p, uint32_t W, int esize, bool batched)
{
    const void* fn = batched ? reinterpret_cast<const void*>(pick_batch_any(p, W, esize))
                             : reinterpret_cast<const void*>(pick_plain_any(p, W, esize));
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, p.threads, size_t(p.lds_bytes)) != hipSuccess) return 1;
    return n < 1 ? 1 : n;
}

hipError_t set_gather_smem_limits(int max_bytes)
{
    std::vector<const void*> fns;
    all_lds_kernels<uint32_t>(fns);
    all_lds_kernels<uint16_t>(fns);
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lfbp
