// In-place H -> H' (the re-arrangement of Sec. 4 applied to one array).
//
// The map is an involution (applying it twice gives H back, Sec. 4): output
// block O = (s', t') is filled from input block O' = (ns-1-s', nt-1-t') and
// block O' from block O, with the x-rows paired as x <-> (x + a) mod nx and
// the rotations b*nz and -b*nz (a = (s'-hs) mod nx, b = (t'-ht) mod ny).  The
// centre block (s', t') = (hs, ht) has a = b = 0 and maps onto itself
// unchanged.  So the array is rewritten in disjoint pairs of row groups: a
// workgroup reads nr x-rows of block O and their nr partner rows of block O'
// into LDS, already rotated into output order, waits until every read of the
// pair is done, and writes both groups back.  Every element is read once and
// written once (the same HBM traffic as the out-of-place copy) and no second
// array is needed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lfbp_internal.h"

namespace lfbp {

struct InplaceDesc {
    void* H;
    uint32_t nt, nx, ny, nz, W, NB;
    uint32_t a_off, b_off;  // (s' - hs) mod nx = (s' + a_off) mod nx; likewise t'
    uint32_t nr;            // x-rows per group
    uint32_t groups;        // groups per block pair, ceil(nx / nr)
    FastDiv fnx, fny, fnt, fW, fgroups;
};

namespace {

constexpr int kTileBudget = 40 * 1024;   // LDS per workgroup when a row pair allows: four workgroups per CU

template <typename T>
__global__ void __launch_bounds__(256) k_inplace(InplaceDesc d)
{
    extern __shared__ unsigned char smem_raw[];
    T* tileA = reinterpret_cast<T*>(smem_raw);   // output rows of block O, in output order
    T* tileB = tileA + size_t(d.nr) * d.W;      // output rows of block O'
    const uint32_t unit = blockIdx.x;
    const uint32_t O = fdiv(unit, d.fgroups), grp = unit - O * d.groups;
    const uint32_t Op = d.NB - 1 - O;
    const uint32_t sp = fdiv(O, d.fnt), tp = O - sp * d.nt;
    const uint32_t ua = sp + d.a_off, ub = tp + d.b_off;
    const uint32_t a = ua - fdiv(ua, d.fnx) * d.nx;
    const uint32_t b = ub - fdiv(ub, d.fny) * d.ny;
    const uint32_t rotA = b * d.nz;                              // rotation of block O's output rows
    const uint32_t rotB = (b == 0 ? 0u : d.ny - b) * d.nz;      // and of block O''s
    const uint32_t x0 = grp * d.nr;
    if (x0 >= d.nx) return;  // never taken: the host balances groups so that every group has rows
    const uint32_t nr = min(d.nr, d.nx - x0);
    const uint32_t W = d.W, n = nr * W;
    T* H = static_cast<T*>(d.H);
    const uint64_t baseO = uint64_t(O) * d.nx * W, baseOp = uint64_t(Op) * d.nx * W;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t r = fdiv(i, d.fW), j = i - r * W;
        const uint32_t xa = x0 + r;
        uint32_t xb = xa + a;
        if (xb >= d.nx) xb -= d.nx;
        // output row (O, xa) is input row (O', xb) rotated left by rotA;
        // output row (O', xb) is input row (O, xa) rotated left by rotB
        const T vA = H[baseOp + uint64_t(xb) * W + j];
        const T vB = H[baseO + uint64_t(xa) * W + j];
        tileA[r * W + (j >= rotA ? j - rotA : j + W - rotA)] = vA;
        tileB[r * W + (j >= rotB ? j - rotB : j + W - rotB)] = vB;
    }
    __syncthreads();  // every read of the pair precedes every write
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t r = fdiv(i, d.fW), j = i - r * W;
        const uint32_t xa = x0 + r;
        uint32_t xb = xa + a;
        if (xb >= d.nx) xb -= d.nx;
        H[baseO + uint64_t(xa) * W + j] = tileA[i];
        H[baseOp + uint64_t(xb) * W + j] = tileB[i];
    }
}

}  // namespace

hipError_t set_inplace_smem_limits(int max_bytes)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_inplace<uint32_t>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_inplace<uint16_t>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
}

// H <- H' in place; max_lds: dynamic LDS one workgroup may use.
hipError_t launch_inplace(void* H, const lfbp_shape& s, int esize, int max_lds, hipStream_t stream)
{
    InplaceDesc d;
    d.H = H;
    d.nt = uint32_t(s.nt);
    d.nx = uint32_t(s.nx);
    d.ny = uint32_t(s.ny);
    d.nz = uint32_t(s.nz);
    d.W = uint32_t(s.ny * s.nz);
    d.NB = uint32_t(s.ns * s.nt);
    const uint32_t hs = uint32_t((s.ns - 1) / 2), ht = uint32_t((s.nt - 1) / 2);
    d.a_off = (d.nx - hs % d.nx) % d.nx;
    d.b_off = (d.ny - ht % d.ny) % d.ny;
    const uint32_t pairs = (d.NB - 1) / 2;  // the centre block stays as it is
    if (pairs == 0) return hipSuccess;
    // rows per group: two tiles of nr rows within kTileBudget bytes (several
    // workgroups per CU), or within the whole LDS when a row pair is larger
    const uint64_t row_bytes = uint64_t(d.W) * uint32_t(esize);
    const uint64_t budget = 2 * row_bytes <= uint64_t(kTileBudget) ? uint64_t(kTileBudget) : uint64_t(max_lds);
    uint32_t nr = uint32_t(std::min<uint64_t>(d.nx, budget / (2 * row_bytes)));
    if (nr == 0) return hipErrorInvalidValue;  // one x-row pair exceeds the LDS (refused on the host first)
    d.groups = (d.nx + nr - 1) / nr;
    d.nr = (d.nx + d.groups - 1) / d.groups;  // balance the groups
    d.fnx = make_fastdiv(d.nx);
    d.fny = make_fastdiv(d.ny);
    d.fnt = make_fastdiv(d.nt);
    d.fW = make_fastdiv(d.W);
    d.fgroups = make_fastdiv(d.groups);
    const size_t lds = 2 * size_t(d.nr) * row_bytes;
    const uint64_t units = uint64_t(pairs) * d.groups;
    if (units >= (uint64_t(1) << 31)) return hipErrorInvalidValue;
    if (esize == 4)
        hipLaunchKernelGGL(k_inplace<uint32_t>, dim3(unsigned(units)), dim3(256), lds, stream, d);
    else
        hipLaunchKernelGGL(k_inplace<uint16_t>, dim3(unsigned(units)), dim3(256), lds, stream, d);
    return hipGetLastError();
}

}  // namespace lfbp
