// H -> H' for arrays stored column-major (s fastest, then t, x, y, z: the
// order of Matlab arrays, in which the paper's implementation works, Sec. 5).
//
// The map is the one of Sec. 4 (Eqs. 4-9):
//   H'(s',t',x',y',z) = H(ns-1-s', nt-1-t', (x'+a(s')) mod nx, (y'+b(t')) mod ny, z),
//   a(s') = (s'-hs) mod nx,  b(t') = (t'-ht) mod ny.
// With s contiguous, one output s-row (t',x',y',z) draws on nx different
// input s-rows, because x cycles with s': the (s, x) plane is a sheared
// transpose.  For fixed (t',y',z) all nx output rows read the same input plane
// (t, y, z) = (nt-1-t', (y'+b(t')) mod ny, z), so a workgroup loads a chunk of
// S positions of that plane's nx input rows into LDS (contiguous row pieces)
// and writes the matching chunk of the nx output rows (contiguous too), each
// element taken from the tile at (x, s) = ((x'+a(s')) mod nx, ns-1-s').
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lfbp_internal.h"

namespace lfbp {

struct ColDesc {
    const void* H;
    void* Ht;
    uint32_t ns, nt, nx, ny, nz;
    uint32_t a_off, b_off;   // a(s') = (s' + a_off) mod nx; b(t') = (t' + b_off) mod ny
    uint32_t S;              // s positions per chunk
    uint32_t chunks;         // ceil(ns / S)
    FastDiv fnt, fny, fnx, fchunks, fS;
};

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_colmajor(ColDesc d)
{
    extern __shared__ unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);   // [nx][Sn]: input rows x, positions s_lo .. s_lo+Sn-1
    const uint32_t unit = blockIdx.x;
    const uint32_t plane = fdiv(unit, d.fchunks), c = unit - plane * d.chunks;
    // plane = (z * ny + y') * nt + t'
    const uint32_t q1 = fdiv(plane, d.fnt), tp = plane - q1 * d.nt;
    const uint32_t z = fdiv(q1, d.fny), yp = q1 - z * d.ny;
    const uint32_t ub = tp + d.b_off;
    const uint32_t b = ub - fdiv(ub, d.fny) * d.ny;
    uint32_t y = yp + b;
    if (y >= d.ny) y -= d.ny;
    const uint32_t t = d.nt - 1 - tp;
    const uint32_t s0 = c * d.S;
    if (s0 >= d.ns) return;  // never taken: the host balances the chunks
    const uint32_t Sn = min(d.S, d.ns - s0);
    const uint32_t s_lo = d.ns - s0 - Sn;   // input positions ns-1-s' for s' in [s0, s0+Sn)
    const uint64_t row = d.ns, xstride = uint64_t(d.ns) * d.nt;
    const uint64_t in0 = (uint64_t(t) + uint64_t(d.nt) * uint64_t(d.nx) * (uint64_t(y) + uint64_t(d.ny) * z)) * row;
    const uint64_t out0 = (uint64_t(tp) + uint64_t(d.nt) * uint64_t(d.nx) * (uint64_t(yp) + uint64_t(d.ny) * z)) * row;
    const T* H = static_cast<const T*>(d.H);
    T* Ht = static_cast<T*>(d.Ht);
    const uint32_t n = d.nx * Sn;
    const bool full = Sn == d.S;   // every chunk but a shorter last one
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t x = full ? fdiv(i, d.fS) : i / Sn, k = i - x * Sn;
        tile[i] = H[in0 + x * xstride + s_lo + k];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t xp = full ? fdiv(i, d.fS) : i / Sn, k = i - xp * Sn;
        const uint32_t sp = s0 + k;
        const uint32_t ua = sp + d.a_off;
        uint32_t x = xp + (ua - fdiv(ua, d.fnx) * d.nx);
        if (x >= d.nx) x -= d.nx;
        Ht[out0 + xp * xstride + sp] = tile[x * Sn + (Sn - 1 - k)];
    }
}

constexpr int kColTileBudget = 32 * 1024;   // LDS per workgroup when the plane allows

}  // namespace

hipError_t set_colmajor_smem_limits(int max_bytes)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colmajor<uint32_t>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_colmajor<uint16_t>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
}

hipError_t launch_colmajor(const void* H, void* Ht, const lfbp_shape& s, int esize, int max_lds, hipStream_t stream)
{
    ColDesc d;
    d.H = H;
    d.Ht = Ht;
    d.ns = uint32_t(s.ns);
    d.nt = uint32_t(s.nt);
    d.nx = uint32_t(s.nx);
    d.ny = uint32_t(s.ny);
    d.nz = uint32_t(s.nz);
    const uint32_t hs = (d.ns - 1) / 2, ht = (d.nt - 1) / 2;
    d.a_off = (d.nx - hs % d.nx) % d.nx;
    d.b_off = (d.ny - ht % d.ny) % d.ny;
    // s positions per chunk: the whole row when nx rows of it fit the tile budget
    const uint64_t col_bytes = uint64_t(d.nx) * uint32_t(esize);
    const uint64_t budget = col_bytes <= uint64_t(kColTileBudget) ? uint64_t(kColTileBudget) : uint64_t(max_lds);
    const uint32_t S0 = uint32_t(std::min<uint64_t>(d.ns, budget / col_bytes));
    if (S0 == 0) return hipErrorInvalidValue;   // refused on the host first
    d.chunks = (d.ns + S0 - 1) / S0;
    d.S = (d.ns + d.chunks - 1) / d.chunks;
    d.fnt = make_fastdiv(d.nt);
    d.fny = make_fastdiv(d.ny);
    d.fnx = make_fastdiv(d.nx);
    d.fchunks = make_fastdiv(d.chunks);
    d.fS = make_fastdiv(d.S);
    const uint64_t units = uint64_t(d.nt) * d.ny * d.nz * d.chunks;
    if (units >= (uint64_t(1) << 31)) return hipErrorInvalidValue;
    const size_t lds = size_t(d.nx) * d.S * uint32_t(esize);
    if (esize == 4)
        hipLaunchKernelGGL(k_colmajor<uint32_t>, dim3(unsigned(units)), dim3(256), lds, stream, d);
    else
        hipLaunchKernelGGL(k_colmajor<uint16_t>, dim3(unsigned(units)), dim3(256), lds, stream, d);
    return hipGetLastError();
}

}  // namespace lfbp
