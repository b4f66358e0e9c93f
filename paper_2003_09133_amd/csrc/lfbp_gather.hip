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
// (ns-1-s', nt-1-t', (x'+a) mod nx) rotated left by b*nz elements.  All index
// work is per row and wave-uniform (scalar unit); per element only the
// rotation wraps.  No arithmetic touches the payloads: float32 and float16
// both move as raw 32/16-bit words.
//
// Two kernels:
//   direct  -- a wavefront copies U whole x-rows, reading H at rotated
//              addresses and writing H' contiguously (dword/short accesses,
//              each wave instruction covers 64 consecutive elements).
//   staged  -- a workgroup rotates a run of consecutive output x-rows into an
//              LDS tile laid out exactly like that stretch of H', then writes
//              the tile to HBM with aligned 16-byte stores (full cache lines).
// Each has a plain entry (descriptor passed by value, nothing allocated) and a
// batched entry (descriptor table in device memory, one persistent launch for
// many problems).
#include <hip/hip_runtime.h>

#include "lfbp_internal.h"

namespace lfbp {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void put(T* p, T v, bool nt)
{
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

__device__ __forceinline__ void put16(void* p, u32x4 v, bool nt)
{
    if (nt)
        __builtin_nontemporal_store(v, static_cast<u32x4*>(p));
    else
        *static_cast<u32x4*>(p) = v;
}

// Source of output x-row R: pointer to the start of the input x-row and the
// left rotation in elements.
template <typename T>
__device__ __forceinline__ void row_source(const GatherDesc& d, uint32_t R, const T*& src, uint32_t& rot)
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
    const uint64_t in_row = uint64_t(d.NB - 1 - O) * d.nx + xs;  // block reversal (Eqs. 8-9)
    src = static_cast<const T*>(d.H) + in_row * d.W;
    rot = b * d.nz;
}

// ---------------------------------------------------------------- direct

// U consecutive output x-rows starting at R0, S 64-element segments per row
// per step, all U*S loads of a step in flight before the stores.
template <typename T, int S, int U>
__device__ __forceinline__ void direct_rows(const GatherDesc& d, uint32_t R0, uint32_t lane, bool nt)
{
    const T* src[U];
    T* dst[U];
    uint32_t rot[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t R = R0 + u;
        live[u] = R < d.nrows;
        const uint32_t Rc = live[u] ? R : R0;
        row_source<T>(d, Rc, src[u], rot[u]);
        dst[u] = static_cast<T*>(d.Ht) + uint64_t(Rc) * d.W;
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

// Work unit of the direct kernel = rows_per_unit consecutive output rows,
// split over the wavefronts of the workgroup in steps of U rows.
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

// ---------------------------------------------------------------- staged

template <typename T, int S, int U>
__device__ __forceinline__ void staged_unit(const GatherDesc& d, uint32_t unit, T* lds, bool nt)
{
    constexpr uint32_t VE = 16 / sizeof(T);  // elements per 16-byte vector
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t W = d.W;
    const uint32_t R0 = unit * d.rows_per_unit;
    const uint32_t nr = min(d.rows_per_unit, d.nrows - R0);
    const uint64_t O0 = uint64_t(R0) * W;                       // first output element
    const uint32_t lead = uint32_t((O0 + d.phase_out) % VE);    // LDS slot of O0
    const uint32_t L = nr * W;

    // 1. Load: input rows in, rotated into their output slots.
    for (uint32_t r0 = wave * U; r0 < nr; r0 += nw * U) {
        const T* src[U];
        uint32_t rot[U];
        bool live[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            live[u] = r0 + u < nr;
            row_source<T>(d, R0 + (live[u] ? r0 + u : r0), src[u], rot[u]);
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

    // 2. Emit: the tile is H'[O0, O0+L) shifted by `lead`; write it with
    //    16-byte stores at 16-byte aligned addresses, partial vectors at the
    //    two ends element by element.
    T* out = static_cast<T*>(d.Ht);
    const uint64_t g0 = O0 + d.phase_out;
    const uint64_t u0 = g0 / VE, u1 = (g0 + L + VE - 1) / VE;
    for (uint64_t u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
        const uint32_t li = uint32_t((u - u0) * VE);            // LDS index of the vector
        const int64_t rel = int64_t(li) - int64_t(lead);         // position in the unit
        if (rel >= 0 && rel + VE <= L) {
            put16(out + (O0 + rel), *reinterpret_cast<const u32x4*>(lds + li), nt);
        } else {
#pragma unroll
            for (uint32_t e = 0; e < VE; ++e) {
                const int64_t p = rel + e;
                if (p >= 0 && p < int64_t(L)) put<T>(out + (O0 + p), lds[li + e], nt);
            }
        }
    }
    __syncthreads();
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

// Batched entries: unit_start[p] = first global unit of problem p,
// unit_start[count] = total.  The grid strides over all units of all problems.
__device__ __forceinline__ uint32_t find_problem(const uint32_t* unit_start, uint32_t count, uint32_t g)
{
    uint32_t lo = 0, hi = count;  // unit_start[lo] <= g < unit_start[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (unit_start[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename T, int S, int U>
__global__ void __launch_bounds__(512)
    k_direct_batched(const GatherDesc* descs, const uint32_t* unit_start, uint32_t count, int nt)
{
    const uint32_t total = unit_start[count];
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
        const uint32_t p = find_problem(unit_start, count, g);
        const GatherDesc d = descs[p];
        direct_unit<T, S, U>(d, g - unit_start[p], nt != 0);
    }
}

template <typename T, int S, int U>
__global__ void __launch_bounds__(512)
    k_staged_batched(const GatherDesc* descs, const uint32_t* unit_start, uint32_t count, int nt)
{
    extern __shared__ u32x4 smem[];
    T* lds = reinterpret_cast<T*>(smem);
    const uint32_t total = unit_start[count];
    for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
        const uint32_t p = find_problem(unit_start, count, g);
        const GatherDesc d = descs[p];
        staged_unit<T, S, U>(d, g - unit_start[p], lds, nt != 0);
    }
}

// ---------------------------------------------------------------- host side

namespace {

typedef void (*PlainFn)(GatherDesc, int);
typedef void (*BatchFn)(const GatherDesc*, const uint32_t*, uint32_t, int);

template <typename T, int S>
PlainFn pick_plain_s(int variant, int U)
{
    if (variant == LFBP_GATHER_DIRECT) return U >= 2 ? k_direct<T, S, 2> : k_direct<T, S, 1>;
    return U >= 2 ? k_staged<T, S, 2> : k_staged<T, S, 1>;
}

template <typename T, int S>
BatchFn pick_batch_s(int variant, int U)
{
    if (variant == LFBP_GATHER_DIRECT) return U >= 2 ? k_direct_batched<T, S, 2> : k_direct_batched<T, S, 1>;
    return U >= 2 ? k_staged_batched<T, S, 2> : k_staged_batched<T, S, 1>;
}

// S = 64-element segments per row loaded per step: enough to cover a row of
// W elements in one step up to W = 1024, in batches of 16 beyond that.
int segments_for(uint32_t W)
{
    const uint32_t need = (W + 63) / 64;
    return need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 16;
}

template <typename T>
PlainFn pick_plain(int variant, uint32_t W, int U)
{
    switch (segments_for(W)) {
        case 2: return pick_plain_s<T, 2>(variant, U);
        case 4: return pick_plain_s<T, 4>(variant, U);
        case 8: return pick_plain_s<T, 8>(variant, U);
        default: return pick_plain_s<T, 16>(variant, U);
    }
}

template <typename T>
BatchFn pick_batch(int variant, uint32_t W, int U)
{
    switch (segments_for(W)) {
        case 2: return pick_batch_s<T, 2>(variant, U);
        case 4: return pick_batch_s<T, 4>(variant, U);
        case 8: return pick_batch_s<T, 8>(variant, U);
        default: return pick_batch_s<T, 16>(variant, U);
    }
}

}  // namespace

// Launch one problem.  The plan is fully resolved; d.rows_per_unit/nunits set.
hipError_t launch_gather(const GatherDesc& d, int esize, const LaunchPlan& p, hipStream_t stream)
{
    PlainFn fn = esize == 4 ? pick_plain<uint32_t>(p.variant, d.W, p.rows_in_flight)
                            : pick_plain<uint16_t>(p.variant, d.W, p.rows_in_flight);
    const size_t shmem = p.variant == LFBP_GATHER_STAGED ? size_t(p.tile_bytes) : 0;
    hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.threads), shmem, stream, d, p.nontemporal == 1 ? 1 : 0);
    return hipGetLastError();
}

// Launch a batch.  All problems share variant, threads, U and S (the largest W
// of the batch picks S); descs and unit_start live in device memory.
hipError_t launch_gather_batched(const GatherDesc* descs_dev, const uint32_t* unit_start_dev, uint32_t count,
                                 uint32_t maxW, int esize, const LaunchPlan& p, hipStream_t stream)
{
    BatchFn fn = esize == 4 ? pick_batch<uint32_t>(p.variant, maxW, p.rows_in_flight)
                            : pick_batch<uint16_t>(p.variant, maxW, p.rows_in_flight);
    const size_t shmem = p.variant == LFBP_GATHER_STAGED ? size_t(p.tile_bytes) : 0;
    hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.threads), shmem, stream, descs_dev, unit_start_dev, count,
                       p.nontemporal == 1 ? 1 : 0);
    return hipGetLastError();
}

// Workgroups of the batched kernel that fit one CU at once.
int batched_occupancy(int variant, uint32_t maxW, int esize, int U, int threads, int smem)
{
    BatchFn fn = esize == 4 ? pick_batch<uint32_t>(variant, maxW, U) : pick_batch<uint16_t>(variant, maxW, U);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(fn), threads, size_t(smem)) !=
        hipSuccess)
        return 1;
    return n;
}

hipError_t set_gather_smem_limits(int max_bytes)
{
    // Allow the staged kernels to use up to max_bytes of dynamic LDS.
    const void* fns[] = {
        (const void*)k_staged<uint32_t, 2, 1>,  (const void*)k_staged<uint32_t, 2, 2>,
        (const void*)k_staged<uint32_t, 4, 1>,  (const void*)k_staged<uint32_t, 4, 2>,
        (const void*)k_staged<uint32_t, 8, 1>,  (const void*)k_staged<uint32_t, 8, 2>,
        (const void*)k_staged<uint32_t, 16, 1>, (const void*)k_staged<uint32_t, 16, 2>,
        (const void*)k_staged<uint16_t, 2, 1>,  (const void*)k_staged<uint16_t, 2, 2>,
        (const void*)k_staged<uint16_t, 4, 1>,  (const void*)k_staged<uint16_t, 4, 2>,
        (const void*)k_staged<uint16_t, 8, 1>,  (const void*)k_staged<uint16_t, 8, 2>,
        (const void*)k_staged<uint16_t, 16, 1>, (const void*)k_staged<uint16_t, 16, 2>,
        (const void*)k_staged_batched<uint32_t, 2, 1>,  (const void*)k_staged_batched<uint32_t, 2, 2>,
        (const void*)k_staged_batched<uint32_t, 4, 1>,  (const void*)k_staged_batched<uint32_t, 4, 2>,
        (const void*)k_staged_batched<uint32_t, 8, 1>,  (const void*)k_staged_batched<uint32_t, 8, 2>,
        (const void*)k_staged_batched<uint32_t, 16, 1>, (const void*)k_staged_batched<uint32_t, 16, 2>,
        (const void*)k_staged_batched<uint16_t, 2, 1>,  (const void*)k_staged_batched<uint16_t, 2, 2>,
        (const void*)k_staged_batched<uint16_t, 4, 1>,  (const void*)k_staged_batched<uint16_t, 4, 2>,
        (const void*)k_staged_batched<uint16_t, 8, 1>,  (const void*)k_staged_batched<uint16_t, 8, 2>,
        (const void*)k_staged_batched<uint16_t, 16, 1>, (const void*)k_staged_batched<uint16_t, 16, 2>,
    };
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lfbp
