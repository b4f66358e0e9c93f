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
    uint64_t E;              // elements of H (and of Ht)
    uint32_t ns, nt, nx, ny, nz;
    uint32_t a_off;          // a(s') = (s' + a_off) mod nx
    uint32_t b_off;          // b(t') = (t' + b_off) mod ny
    uint32_t phase_in;       // (address of H / element size) mod (16 / element size)
    uint32_t phase_out;      // the same for Ht
    uint32_t S;              // s positions per chunk
    uint32_t chunks;         // ceil(ns / S)
    uint32_t P;              // tile row pitch in elements: a multiple of the vector width, >= S + width - 1
    uint32_t VR;             // 16-byte vectors per tile row, P / width
    uint32_t units;          // workgroups: nt * ny * nz * chunks
    uint32_t xstride;        // ns * nt: distance between x-rows
    uint32_t dq_load, dr_load;   // kThreads = dq_load * VR + dr_load
    uint32_t dq_off;         // dq_load * xstride
    // per chunk kind [full chunk, last chunk]:
    uint32_t NF[2];          // whole output vectors every row holds
    uint32_t dq_st[2], dr_st[2];   // kThreads = dq_st * max(NF, 1) + dr_st
    uint32_t du_st[2];       // (dr_st * width) mod nx
    uint32_t dnf_st[2];      // (NF * width) mod nx
    FastDiv fnt, fny, fnx, fchunks, fVR;
    FastDiv fNF[2];          // of max(NF, 1)
    FastDiv fL[2];           // of the elements left over per row, Sn - NF * width
};

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
union Vec16 {
    u32x4 v;
    T e[16 / sizeof(T)];
};

constexpr uint32_t kThreads = 256;
constexpr int kLoadBatch = 4;   // 16-byte loads each thread keeps in flight
constexpr bool kXcdOrder = true;
constexpr uint32_t kColXcds = 8;   // XCDs of the device

// Unit of this workgroup.  Workgroups are dealt to the XCDs round-robin;
// with kXcdOrder each XCD takes a contiguous run of units instead, so that the
// chunks of one plane, whose pieces share cache lines at their ends, meet in
// one L2.
__device__ __forceinline__ uint32_t unit_of_block(uint32_t units)
{
    const uint32_t bid = blockIdx.x + blockIdx.y * gridDim.x;   // dispatch order; < units
    if (!kXcdOrder) return bid;
    const uint32_t x = bid % kColXcds, q = units / kColXcds, r = units % kColXcds;
    return x * q + min(x, r) + bid / kColXcds;
}

// A barrier that orders LDS accesses only: pending global stores and loads
// stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Where one unit reads and writes.  A unit is the chunk [s0, s0+Sn) of the
// nx output rows (t', x', y', z), x' = 0..nx-1, made from the matching pieces
// [s_lo, s_lo+Sn) of the nx input rows (t, x, y, z) of one plane,
// t = nt-1-t', y = (y' + b(t')) mod ny.
struct UnitGeom {
    uint64_t in0, out0;   // element index of input row (t, 0, y, z), output row (t', 0, y', z)
    uint32_t s0, Sn, s_lo;
    uint32_t cin;         // misalignment of input row x's piece: (cin + x * xsm) mod VE
    uint32_t cout;        // the same for output row x' at s' = s0
    int last;             // 1 for a shorter last chunk
    bool safe;            // every 16-byte vector the unit reads lies inside H
};

template <uint32_t VE>
__device__ __forceinline__ UnitGeom unit_geom(const ColDesc& d, uint32_t unit)
{
    UnitGeom g;
    const uint32_t plane = fdiv(unit, d.fchunks), c = unit - plane * d.chunks;
    // plane = (z * ny + y') * nt + t'
    const uint32_t q1 = fdiv(plane, d.fnt), tp = plane - q1 * d.nt;
    const uint32_t z = fdiv(q1, d.fny), yp = q1 - z * d.ny;
    const uint32_t ub = tp + d.b_off;
    const uint32_t b = ub - fdiv(ub, d.fny) * d.ny;
    uint32_t y = yp + b;
    if (y >= d.ny) y -= d.ny;
    const uint32_t t = d.nt - 1 - tp;
    g.s0 = c * d.S;                     // < ns: the host balances the chunks
    g.Sn = min(d.S, d.ns - g.s0);
    g.s_lo = d.ns - g.s0 - g.Sn;        // input positions ns-1-s' for s' in [s0, s0+Sn)
    g.last = g.Sn != d.S;
    g.in0 = (uint64_t(t) + uint64_t(d.nt) * uint64_t(d.nx) * (uint64_t(y) + uint64_t(d.ny) * z)) * d.ns;
    g.out0 = (uint64_t(tp) + uint64_t(d.nt) * uint64_t(d.nx) * (uint64_t(yp) + uint64_t(d.ny) * z)) * d.ns;
    g.cin = uint32_t((g.in0 + g.s_lo + d.phase_in) % VE);
    g.cout = uint32_t((g.out0 + g.s0 + d.phase_out) % VE);
    const uint64_t g_first = g.in0 + g.s_lo, g_last = g.in0 + uint64_t(d.nx - 1) * d.xstride + g.s_lo;
    g.safe = g_first >= VE && g_last + d.P <= d.E;
    return g;
}

// Read a unit's tile for a unit at either end of H: vectors that stick out
// of the array are read element by element.
template <typename T>
__device__ __forceinline__ void load_tile_edge(const ColDesc& d, const UnitGeom& g, T* tile)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const T* H = static_cast<const T*>(d.H);
    const uint32_t xsm = d.xstride % VE;
    for (uint32_t j = threadIdx.x; j < d.nx * d.VR; j += kThreads) {
        const uint32_t x = fdiv(j, d.fVR), v = j - x * d.VR;
        const uint32_t m = (g.cin + x * xsm) & (VE - 1);
        if (v * VE >= m + g.Sn) continue;
        const int64_t vg = int64_t(g.in0 + x * d.xstride + g.s_lo) - m + int64_t(v * VE);   // aligned
        Vec16<T> p;
        if (vg >= 0 && uint64_t(vg) + VE <= d.E) {
            p.v = *reinterpret_cast<const u32x4*>(H + vg);
        } else {
#pragma unroll
            for (uint32_t q = 0; q < VE; ++q) {
                const int64_t i = vg + q;
                p.e[q] = (i >= 0 && uint64_t(i) < d.E) ? H[i] : T(0);
            }
        }
        *reinterpret_cast<u32x4*>(tile + x * d.P + v * VE) = p.v;
    }
}

// Issue the loads of kN of this thread's tile vectors, j = j0 + k * kThreads
// for k < kN, starting from (row x, vector v, x * xstride) = (x, v, xoff) of
// j0 and stepping without divisions; slot[k] is the vector's tile index or
// ~0 for none (such lanes read the aligned vector at the start of the first
// piece again).  For units with g.safe.
template <typename T, int kN>
__device__ __forceinline__ void issue_loads(const ColDesc& d, const UnitGeom& g, uint32_t j0, uint32_t& x,
                                            uint32_t& v, uint32_t& xoff, u32x4 (&p)[kN], uint32_t (&slot)[kN])
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const T* Hb = static_cast<const T*>(d.H) + (g.in0 + g.s_lo - VE);   // VE before the first piece
    const uint32_t xsm = d.xstride % VE, total = d.nx * d.VR;
    uint32_t off[kN];
#pragma unroll
    for (int k = 0; k < kN; ++k) {
        const uint32_t m = (g.cin + x * xsm) & (VE - 1);
        const bool live = j0 + k * kThreads < total && v * VE < m + g.Sn;
        off[k] = live ? xoff + VE - m + v * VE : VE - g.cin;
        slot[k] = live ? x * d.P + v * VE : ~0u;
        v += d.dr_load;
        x += d.dq_load;
        xoff += d.dq_off;
        if (v >= d.VR) {
            v -= d.VR;
            ++x;
            xoff += d.xstride;
        }
    }
#pragma unroll
    for (int k = 0; k < kN; ++k) p[k] = *reinterpret_cast<const u32x4*>(Hb + off[k]);
}

template <typename T, int kN>
__device__ __forceinline__ void commit_loads(T* tile, const u32x4 (&p)[kN], const uint32_t (&slot)[kN])
{
#pragma unroll
    for (int k = 0; k < kN; ++k)
        if (slot[k] != ~0u) *reinterpret_cast<u32x4*>(tile + slot[k]) = p[k];
}

// Row table after the tile: for i = 0 .. nx+VE-2, rt[i] = R(i mod nx) - i
// with R(x) = x * P + m_x + Sn - 1, the tile index of input row x at
// s' = s0.  Element kk of output row x' comes from input row
// x = (x' + a(s0 + kk)) mod nx at tile index R(x) - kk, and for the VE
// elements kk = k0 + q of one output vector, with x_q = x_0 + q (unreduced),
// that is rt[x_0 + q] + x_0 - k0.
template <uint32_t VE>
__device__ __forceinline__ void build_row_table(const ColDesc& d, const UnitGeom& g, int32_t* rt)
{
    const uint32_t xsm = d.xstride % VE;
    for (uint32_t i = threadIdx.x; i < d.nx + VE - 1; i += kThreads) {
        const uint32_t x = i - fdiv(i, d.fnx) * d.nx;
        rt[i] = int32_t(x * d.P + ((g.cin + x * xsm) & (VE - 1)) + g.Sn - 1) - int32_t(i);
    }
}

// Write a unit's nx output rows from its tile.  Output row x' holds
// s' = s0 + kk at out0 + x' * xstride + s0 + kk; its whole aligned 16-byte
// vectors start at kk = kA, the first kk whose address is aligned, and the
// L = Sn - NF * VE elements outside them (kk < kA, kk >= kA + NF * VE) are
// written one by one.
template <typename T>
__device__ __forceinline__ void store_tile(const ColDesc& d, const UnitGeom& g, const T* tile, const int32_t* rt)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    const uint32_t xsm = d.xstride % VE;
    const uint32_t NF = d.NF[g.last];
    T* Ob = static_cast<T*>(d.Ht) + (g.out0 + g.s0);
    const uint32_t nvec = d.nx * NF;
    if (threadIdx.x < nvec) {
        // this thread's vectors j = threadIdx.x + i * kThreads, as (row x',
        // vector f), and u = (s0 + a_off + f * VE) mod nx, stepped without
        // divisions
        uint32_t xp = fdiv(threadIdx.x, d.fNF[g.last]), f = threadIdx.x - xp * NF;
        uint32_t xoff = xp * d.xstride;
        uint32_t u = g.s0 + d.a_off + f * VE;
        u -= fdiv(u, d.fnx) * d.nx;
        const uint32_t dq = d.dq_st[g.last], dr = d.dr_st[g.last], du = d.du_st[g.last], dnf = d.dnf_st[g.last];
        const uint32_t dq_off = dq * d.xstride;
        for (uint32_t j = threadIdx.x; j < nvec; j += kThreads) {
            const uint32_t mo = (g.cout + xp * xsm) & (VE - 1);
            const uint32_t kA = (VE - mo) & (VE - 1);
            const uint32_t k0 = kA + f * VE;
            // x_0 = (x' + a(s0 + k0)) mod nx = (x' + u + kA) mod nx
            uint32_t x0 = xp + u;
            if (x0 >= d.nx) x0 -= d.nx;
            x0 += kA;
            if (d.nx >= VE) {
                if (x0 >= d.nx) x0 -= d.nx;
            } else {
                while (x0 >= d.nx) x0 -= d.nx;
            }
            const int32_t C = int32_t(x0) - int32_t(k0);
            Vec16<T> p;
#pragma unroll
            for (uint32_t q = 0; q < VE; ++q) p.e[q] = tile[rt[x0 + q] + C];
            *reinterpret_cast<u32x4*>(Ob + (xoff + k0)) = p.v;
            f += dr;
            xp += dq;
            xoff += dq_off;
            u += du;
            if (u >= d.nx) u -= d.nx;
            if (f >= NF) {
                f -= NF;
                ++xp;
                xoff += d.xstride;
                u = u >= dnf ? u - dnf : u + d.nx - dnf;
            }
        }
    }
    const uint32_t L = g.Sn - NF * VE;
    for (uint32_t j = threadIdx.x; j < d.nx * L; j += kThreads) {
        const uint32_t xp = fdiv(j, d.fL[g.last]), i = j - xp * L;
        const uint32_t mo = (g.cout + xp * xsm) & (VE - 1);
        const uint32_t kA = (VE - mo) & (VE - 1);
        const uint32_t kk = i < kA ? i : i + NF * VE;
        const uint32_t ua = g.s0 + kk + d.a_off;
        uint32_t x = xp + (ua - fdiv(ua, d.fnx) * d.nx);
        if (x >= d.nx) x -= d.nx;
        Ob[xp * d.xstride + kk] = tile[rt[x] + int32_t(x) - int32_t(kk)];
    }
}

// One workgroup per unit.  Tile row x holds input row x's piece starting at
// tile column m_x, the misalignment of the piece's first element in memory,
// so that every aligned 16-byte vector of H that overlaps the piece lands on
// an aligned 16-byte slot of the tile (elements of it outside the piece land
// in the row's slack and are never read).  Serves every tile size.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_colmajor(ColDesc d)
{
    constexpr uint32_t VE = 16 / sizeof(T);
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    int32_t* rt = reinterpret_cast<int32_t*>(tile + d.nx * d.P);
    if (blockIdx.x + blockIdx.y * gridDim.x >= d.units) return;   // the last row of a two-dimensional grid
    const UnitGeom g = unit_geom<VE>(d, unit_of_block(d.units));
    if (g.safe) {
        uint32_t x = fdiv(threadIdx.x, d.fVR), v = threadIdx.x - x * d.VR;
        uint32_t xoff = x * d.xstride;
        for (uint32_t j0 = threadIdx.x; j0 < d.nx * d.VR; j0 += kLoadBatch * kThreads) {
            u32x4 p[kLoadBatch];
            uint32_t slot[kLoadBatch];
            issue_loads<T, kLoadBatch>(d, g, j0, x, v, xoff, p, slot);
            commit_loads<T, kLoadBatch>(tile, p, slot);
        }
    } else {
        load_tile_edge(d, g, tile);
    }
    build_row_table<VE>(d, g, rt);
    lds_barrier();
    store_tile(d, g, tile, rt);
}

constexpr int kColTileBudget = 96 * 1024;   // LDS per workgroup when the plane allows

// Bytes of the row table that follows the tile (nx + VE - 1 entries, padded).
inline uint64_t row_table_bytes(uint32_t nx, uint32_t VE)
{
    return (uint64_t(nx + VE - 1) * 4 + 15) / 16 * 16;
}

}  // namespace

hipError_t set_colmajor_smem_limits(int max_bytes)
{
    const void* kernels[] = {reinterpret_cast<const void*>(&k_colmajor<uint32_t>),
                             reinterpret_cast<const void*>(&k_colmajor<uint16_t>)};
    for (const void* k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// H' of a column-major H; max_lds: dynamic LDS one workgroup may use.
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
    d.E = uint64_t(s.ns) * uint64_t(s.nt) * uint64_t(s.nx) * uint64_t(s.ny) * uint64_t(s.nz);
    const uint32_t VE = 16 / uint32_t(esize);
    d.phase_in = uint32_t((reinterpret_cast<uintptr_t>(H) / uint32_t(esize)) % VE);
    d.phase_out = uint32_t((reinterpret_cast<uintptr_t>(Ht) / uint32_t(esize)) % VE);
    const uint32_t hs = (d.ns - 1) / 2, ht = (d.nt - 1) / 2;
    d.a_off = (d.nx - hs % d.nx) % d.nx;
    d.b_off = (d.ny - ht % d.ny) % d.ny;
    // s positions per chunk: as many as nx tile rows of them (padded to whole
    // 16-byte vectors, plus one vector of slack) and the row table fit
    // kColTileBudget, the whole row where it fits (long contiguous pieces in
    // both arrays, measured fastest); wide cells, which would leave fewer
    // than four vectors per tile row, take up to the device's whole LDS
    const uint64_t vec_col = uint64_t(d.nx) * 16;   // bytes of one 16-byte column of the tile
    const uint64_t table = row_table_bytes(d.nx, VE);
    const uint64_t small = uint64_t(std::min(kColTileBudget, max_lds));
    const uint64_t budget = vec_col * 4 + table <= small ? small : uint64_t(max_lds);
    if (budget < table + vec_col) return hipErrorInvalidValue;   // refused on the host first
    const uint64_t pmax = ((budget - table) / vec_col) * VE;   // widest row pitch that fits
    if (pmax < VE) return hipErrorInvalidValue;      // refused on the host first
    const uint32_t S0 = uint32_t(std::min<uint64_t>(d.ns, pmax - (VE - 1)));
    d.chunks = (d.ns + S0 - 1) / S0;
    d.S = (d.ns + d.chunks - 1) / d.chunks;
    d.P = (d.S + 2 * VE - 2) / VE * VE;
    d.VR = d.P / VE;
    d.fnt = make_fastdiv(d.nt);
    d.fny = make_fastdiv(d.ny);
    d.fnx = make_fastdiv(d.nx);
    d.fchunks = make_fastdiv(d.chunks);
    d.fVR = make_fastdiv(d.VR);
    d.xstride = d.ns * d.nt;
    d.dq_load = kThreads / d.VR;
    d.dr_load = kThreads % d.VR;
    d.dq_off = d.dq_load * d.xstride;
    // whole output vectors per row: at least floor((Sn - VE + 1) / VE) in
    // every row, whatever its alignment
    const uint32_t Sl = d.ns - (d.chunks - 1) * d.S;
    for (int i = 0; i < 2; ++i) {
        const uint32_t Sn = i == 0 ? d.S : Sl;
        d.NF[i] = Sn >= VE - 1 ? (Sn - (VE - 1)) / VE : 0;
        const uint32_t nf1 = std::max(d.NF[i], 1u);
        d.dq_st[i] = kThreads / nf1;
        d.dr_st[i] = kThreads % nf1;
        d.du_st[i] = uint32_t((uint64_t(d.dr_st[i]) * VE) % d.nx);
        d.dnf_st[i] = uint32_t((uint64_t(d.NF[i]) * VE) % d.nx);
        d.fNF[i] = make_fastdiv(nf1);
        d.fL[i] = make_fastdiv(Sn - d.NF[i] * VE);
    }
    const uint64_t units = uint64_t(d.nt) * d.ny * d.nz * d.chunks;
    if (units >= (uint64_t(1) << 31)) return hipErrorInvalidValue;
    d.units = uint32_t(units);
    const size_t lds = size_t(d.nx) * d.P * uint32_t(esize) + row_table_bytes(d.nx, VE);
    if (lds > size_t(max_lds)) return hipErrorInvalidValue;
    // one workgroup per unit; beyond 2^24 units (work-items past 32 bits) the
    // grid takes a second dimension of 2^16-wide rows
    const dim3 grid = units < (uint64_t(1) << 24) ? dim3(unsigned(units))
                                                  : dim3(1u << 16, unsigned((units + 0xFFFF) >> 16));
    if (esize == 4) {
        hipLaunchKernelGGL(k_colmajor<uint32_t>, grid, dim3(kThreads), lds, stream, d);
    } else {
        hipLaunchKernelGGL(k_colmajor<uint16_t>, grid, dim3(kThreads), lds, stream, d);
    }
    return hipGetLastError();
}

}  // namespace lfbp
