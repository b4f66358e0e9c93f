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
    uint64_t E;             // elements of H
    uint32_t phase;         // (address of H / element size) mod (16 / element size)
    uint32_t nt, nx, ny, nz, W, NB;
    uint32_t a_off, b_off;  // (s' - hs) mod nx = (s' + a_off) mod nx; likewise t'
    uint32_t nr;            // x-rows per group
    uint32_t groups;        // groups per block pair, ceil(nx / nr)
    uint32_t units;         // workgroups: pairs * groups
    FastDiv fnx, fny, fnt, fW, fgroups;
};

namespace {

constexpr int kTileBudget = 40 * 1024;   // LDS per workgroup when a row pair allows: four workgroups per CU
constexpr int kGroupRows = 5;            // x-rows per group

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
union Vec16 {
    u32x4 v;
    T e[16 / sizeof(T)];
};

// Read the L contiguous elements H[g, g+L) (whole x-rows) into a tile, each
// row rotated left by rot: aligned 16-byte loads, kBatch of them issued by
// each thread before any is used; element loads only for a vector that
// sticks out of the array (a segment at either end of H).  Elements of the
// vectors outside the segment belong to other rows and are dropped.
template <int kBatch, typename T>
__device__ __forceinline__ void load_segment(const T* H, uint64_t E, uint32_t phase, uint64_t g, uint32_t L,
                                             uint32_t W, const FastDiv& fW, uint32_t rot, T* tile)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint64_t u0 = (g + phase) / VE, u1 = (g + L + phase + VE - 1) / VE;
    const uint32_t nvec = uint32_t(u1 - u0);
    auto put = [&](const Vec16<T>& p, int64_t vg) {
#pragma unroll
        for (uint32_t q = 0; q < VE; ++q) {
            const int64_t e = vg + int64_t(q) - int64_t(g);
            if (e >= 0 && e < int64_t(L)) {
                const uint32_t r = fdiv(uint32_t(e), fW), j = uint32_t(e) - r * W;
                tile[r * W + (j >= rot ? j - rot : j + W - rot)] = p.e[q];
            }
        }
    };
    if (u0 * VE >= phase && u1 * VE - phase <= E) {
        // every vector lies inside H; lanes past the end reload the first
        for (uint32_t i0 = threadIdx.x; i0 < nvec; i0 += kBatch * blockDim.x) {
            Vec16<T> p[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const uint32_t i = i0 + k * blockDim.x;
                const int64_t vg = int64_t((u0 + (i < nvec ? i : 0)) * VE) - int64_t(phase);
                p[k].v = *reinterpret_cast<const u32x4*>(H + vg);
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const uint32_t i = i0 + k * blockDim.x;
                if (i < nvec) put(p[k], int64_t((u0 + i) * VE) - int64_t(phase));
            }
        }
        return;
    }
    for (uint32_t i = threadIdx.x; i < nvec; i += blockDim.x) {
        const int64_t vg = int64_t((u0 + i) * VE) - int64_t(phase);   // array index of the vector's first element
        Vec16<T> p;
        if (vg >= 0 && uint64_t(vg) + VE <= E) {
            p.v = *reinterpret_cast<const u32x4*>(H + vg);
        } else {
#pragma unroll
            for (uint32_t q = 0; q < VE; ++q) {
                const int64_t j = vg + q;
                p.e[q] = (j >= 0 && uint64_t(j) < E) ? H[j] : T(0);
            }
        }
        put(p, vg);
    }
}

// Write a tile (already in output order) to H[g, g+L): aligned 16-byte stores
// where a vector lies inside the segment, element stores at its ends; nothing
// outside the segment is written.
template <typename T>
__device__ __forceinline__ void store_segment(T* H, uint32_t phase, uint64_t g, uint32_t L, const T* tile)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint64_t u0 = (g + phase) / VE, u1 = (g + L + phase + VE - 1) / VE;
    for (uint64_t u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
        const int64_t vg = int64_t(u * VE) - int64_t(phase);
        const int64_t e0 = vg - int64_t(g);
        if (e0 >= 0 && e0 + VE <= L) {
            Vec16<T> p;
#pragma unroll
            for (uint32_t q = 0; q < VE; ++q) p.e[q] = tile[e0 + q];
            *reinterpret_cast<u32x4*>(H + vg) = p.v;
        } else {
#pragma unroll
            for (uint32_t q = 0; q < VE; ++q) {
                const int64_t e = e0 + q;
                if (e >= 0 && e < int64_t(L)) H[vg + q] = tile[e];
            }
        }
    }
}

template <typename T, int kBatch>
__global__ void __launch_bounds__(256) k_inplace(InplaceDesc d)
{
    extern __shared__ unsigned char smem_raw[];
    T* tileA = reinterpret_cast<T*>(smem_raw);   // output rows of block O, in output order
    T* tileB = tileA + size_t(d.nr) * d.W;      // output rows of block O' (partner order)
    const uint32_t unit = blockIdx.x + blockIdx.y * gridDim.x;   // dispatch order
    if (unit >= d.units) return;                                  // the last row of a two-dimensional grid
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
    const uint32_t W = d.W;
    T* H = static_cast<T*>(d.H);
    // rows x0.. of block O pair with rows (x0 + a) mod nx.. of block O': one
    // segment there, or two when the partner rows wrap past row nx-1
    uint32_t xb0 = x0 + a;
    if (xb0 >= d.nx) xb0 -= d.nx;
    const uint32_t k1 = min(nr, d.nx - xb0);
    const uint64_t gO = (uint64_t(O) * d.nx + x0) * W;
    const uint64_t gP1 = (uint64_t(Op) * d.nx + xb0) * W, gP2 = uint64_t(Op) * d.nx * W;
    load_segment<kBatch>(H, d.E, d.phase, gO, nr * W, W, d.fW, rotB, tileB);
    load_segment<kBatch>(H, d.E, d.phase, gP1, k1 * W, W, d.fW, rotA, tileA);
    if (nr > k1) load_segment<kBatch>(H, d.E, d.phase, gP2, (nr - k1) * W, W, d.fW, rotA, tileA + size_t(k1) * W);
    __syncthreads();  // every read of the pair precedes every write
    store_segment(H, d.phase, gO, nr * W, tileA);
    store_segment(H, d.phase, gP1, k1 * W, tileB);
    if (nr > k1) store_segment(H, d.phase, gP2, (nr - k1) * W, tileB + size_t(k1) * W);
}

}  // namespace

hipError_t set_inplace_smem_limits(int max_bytes)
{
    const void* kernels[] = {reinterpret_cast<const void*>(&k_inplace<uint32_t, 1>),
                             reinterpret_cast<const void*>(&k_inplace<uint32_t, 4>),
                             reinterpret_cast<const void*>(&k_inplace<uint16_t, 1>),
                             reinterpret_cast<const void*>(&k_inplace<uint16_t, 4>)};
    for (const void* k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// H <- H' in place; max_lds: dynamic LDS one workgroup may use.
hipError_t launch_inplace(void* H, const lfbp_shape& s, int esize, int max_lds, hipStream_t stream)
{
    InplaceDesc d;
    d.H = H;
    d.E = uint64_t(s.ns) * uint64_t(s.nt) * uint64_t(s.nx) * uint64_t(s.ny) * uint64_t(s.nz);
    d.phase = uint32_t((reinterpret_cast<uintptr_t>(H) / uint32_t(esize)) % (16 / uint32_t(esize)));
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
    // rows per group: about kGroupRows (measured best on the microscope and
    // camera PSFs, f32 and f16), fewer when two tiles of that many rows would
    // exceed kTileBudget, and at least one row pair (up to the whole LDS)
    const uint64_t row_bytes = uint64_t(d.W) * uint32_t(esize);
    const uint64_t budget = 2 * row_bytes <= uint64_t(kTileBudget) ? uint64_t(kTileBudget) : uint64_t(max_lds);
    uint32_t nr = uint32_t(std::min<uint64_t>(std::min<uint64_t>(d.nx, kGroupRows), budget / (2 * row_bytes)));
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
    d.units = uint32_t(units);
    // loads in flight per thread: four for rows under 2 KB, one for longer
    // rows (measured best on the microscope, camera and camera-f16 PSFs)
    const bool batch = row_bytes < 2048;
    // one workgroup per unit; beyond 2^24 units (work-items past 32 bits) the
    // grid takes a second dimension of 2^16-wide rows
    const dim3 grid = units < (uint64_t(1) << 24) ? dim3(static_cast<unsigned>(units))
                                                  : dim3(1u << 16, static_cast<unsigned>((units + 0xFFFF) >> 16));
    const dim3 block = dim3(256);
    if (esize == 4) {
        if (batch)
            hipLaunchKernelGGL((k_inplace<uint32_t, 4>), grid, block, lds, stream, d);
        else
            hipLaunchKernelGGL((k_inplace<uint32_t, 1>), grid, block, lds, stream, d);
    } else {
        if (batch)
            hipLaunchKernelGGL((k_inplace<uint16_t, 4>), grid, block, lds, stream, d);
        else
            hipLaunchKernelGGL((k_inplace<uint16_t, 1>), grid, block, lds, stream, d);
    }
    return hipGetLastError();
}

}  // namespace lfbp
