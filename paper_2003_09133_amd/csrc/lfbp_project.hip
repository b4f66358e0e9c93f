// Light-field forward projection f = H g (Sec. 2.1, Eq. 1) and backprojection
// g = H' f (the bracketed operator of Eq. 2) as implicit GEMMs on the fp32
// matrix cores of gfx950 (v_mfma_f32_32x32x2_f32).
//
// Forward.  f[p][q] = sum_z sum_{s,t} H[s][t][P mod nx][Q mod ny][z] g[z][P][Q],
// P = p - s + hs, Q = q - t + ht.  Split pixels into lenslet position and class,
// p = nx*Lp + u, q = ny*Lq + v, and substitute s' = s - u, t' = t - v:
//   F[(Lp,Lq)][(u,v)] = sum_{(s',t',z)} A[(Lp,Lq)][(s',t',z)] * B[(s',t',z)][(u,v)]
//   A = g[z][nx*Lp + hs - s'][ny*Lq + ht - t']                       (0 outside the image)
//   B = H[s'+u][t'+v][(hs - s') mod nx][(ht - t') mod ny][z]        (0 outside the patch)
// with s' in [-(nx-1), ns-1] and t' in [-(ny-1), nt-1]: A no longer depends on
// the output class and B is a permutation of H (plus zeros), so this is a
// dense contraction with K = (ns+nx-1)(nt+ny-1)nz.
//
// Backward.  g[z][P][Q] = sum_{p,q} f[p][q] Ht[P-p+hs][Q-q+ht][p mod nx][q mod ny][z].
// With P = nx*LP + cx, Q = ny*LQ + cy and r = P - p + hs - cx, r2 likewise:
//   G[(LP,LQ)][(cx,cy,z)] = sum_{(r,r2)} A[(LP,LQ)][(r,r2)] * B[(r,r2)][(cx,cy,z)]
//   A = f[nx*LP + hs - r][ny*LQ + ht - r2]
//   B = Ht[r+cx][r2+cy][(hs - r) mod nx][(ht - r2) mod ny][z]
//
// Kernel.  A workgroup of 4 wavefronts owns a 64 x 256 output tile (wave w owns
// columns 64w..64w+63 as 2 x 2 MFMA tiles of 32 x 32).  The reduction runs in
// stages staged through double-buffered LDS: the next stage's operands are
// loaded from global memory into registers while the matrix cores work on the
// current one.  Accumulation is two-level: the MFMA accumulators are folded into
// a second float32 register set every few stages, so rounding grows with the
// chunk length, not with the ~10^5-10^6 terms of a full sum.  The forward
// splits K over workgroups (partials reduced in a fixed order by a second
// kernel, so results are deterministic); the backward needs no split.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lfbp_internal.h"

namespace lfbp {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int kThreads = 256;
constexpr int kMT = 64;       // output rows (lenslet positions) per workgroup
constexpr int kNT = 256;      // output columns per workgroup (4 waves x 64)
constexpr int kAStride = kMT + 1;   // LDS row strides, padded against bank conflicts
constexpr int kBStride = kNT + 1;
constexpr int kFwdZC = 22;    // forward: depth planes per stage (even)
constexpr int kBwdKC = 16;    // backward: (r, r2) pairs per stage
constexpr int kFold = 16;     // stages between folds of the MFMA accumulators

struct ProjGeom {
    int ns, nt, nx, ny, nz, hs, ht, R, C;
    int Lr, Lc;   // lenslets per image side (ceil(R/nx), ceil(C/ny))
    int M;        // Lr*Lc
    int Kr, Kc;   // ns+nx-1, nt+ny-1
    FastDiv fKc, fny, fnz, fzc;
};

ProjGeom make_geom(const lfbp_shape& s, int64_t R, int64_t C)
{
    ProjGeom g;
    g.ns = int(s.ns);
    g.nt = int(s.nt);
    g.nx = int(s.nx);
    g.ny = int(s.ny);
    g.nz = int(s.nz);
    g.hs = (g.ns - 1) / 2;
    g.ht = (g.nt - 1) / 2;
    g.R = int(R);
    g.C = int(C);
    g.Lr = int((R + s.nx - 1) / s.nx);
    g.Lc = int((C + s.ny - 1) / s.ny);
    g.M = g.Lr * g.Lc;
    g.Kr = g.ns + g.nx - 1;
    g.Kc = g.nt + g.ny - 1;
    g.fKc = make_fastdiv(uint32_t(g.Kc));
    g.fny = make_fastdiv(uint32_t(g.ny));
    g.fnz = make_fastdiv(uint32_t(g.nz));
    g.fzc = make_fastdiv(uint32_t(kFwdZC));
    return g;
}

__device__ __forceinline__ int imod(int a, int n)
{
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// MFMA work of one stage from LDS buffers As[kc][kAStride], Bs[kc][kBStride].
__device__ __forceinline__ void mma_stage(const float* As, const float* Bs, int kc, int wave, int lane,
                                          f32x16 (&acc)[2][2])
{
    const int li = lane & 31, lk = lane >> 5;
    const int nb = wave * 64;
    for (int s = 0; s < kc; s += 2) {
        const int k = s + lk;
        const float a0 = As[k * kAStride + li];
        const float a1 = As[k * kAStride + 32 + li];
        const float b0 = Bs[k * kBStride + nb + li];
        const float b1 = Bs[k * kBStride + nb + 32 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
}

__device__ __forceinline__ void fold(f32x16 (&acc)[2][2], f32x16 (&tot)[2][2])
{
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            tot[i][j] += acc[i][j];
            acc[i][j] = f32x16{};
        }
}

// ------------------------------------------------------------------ forward

// Operand registers of one forward stage (stage = one (s', t') pair and one
// chunk of kFwdZC depth planes).  Thread t owns B column n0 + t (all depths of
// the chunk: one contiguous run of H) and A row m0 + (t mod 64) at depths
// t/64, t/64 + 4, ... (contiguous runs of the depth-last copy of g), so a
// stage's addresses are a uniform base plus per-thread constants.
constexpr int kFwdAPer = (kFwdZC + 3) / 4;  // depths per thread in the A tile
constexpr int kFwdBPer = kFwdZC;           // depths per thread in the B tile

struct FwdArgs {
    const float* H;    // [ns][nt][nx][ny][nz]
    const float* gT;   // [R][C][nz]  (g with depth innermost)
    float* partial;    // [splits][Mpad][Npad]
    ProjGeom g;
    int N, Npad, Mpad;
    int stages;        // Kr*Kc*nzc
    int nzc;           // depth chunks
    int splits;
};

struct FwdThread {
    int64_t hoff;  // (u*nt + v)*cell of this thread's B column; -1: padding column
    int u, v;
    int P0, Q0;    // nx*Lp + hs, ny*Lq + ht of this thread's A row; P0 < 0: padding row
    int zg;        // first depth of this thread in the A tile
};

__device__ __forceinline__ FwdThread fwd_thread(const FwdArgs& a, int m0, int n0)
{
    const ProjGeom& g = a.g;
    FwdThread t;
    const int tid = threadIdx.x;
    const int n = n0 + tid;
    t.u = 0;
    t.v = 0;
    t.hoff = -1;
    if (n < a.N) {
        t.u = int(fdiv(uint32_t(n), g.fny));
        t.v = n - t.u * g.ny;
        t.hoff = (int64_t(t.u) * g.nt + t.v) * (int64_t(g.nx) * g.ny * g.nz);
    }
    const int m = m0 + (tid & 63);
    t.zg = __builtin_amdgcn_readfirstlane(tid >> 6);
    t.P0 = -1 << 30;
    t.Q0 = 0;
    if (m < g.M) {
        const int Lp = m / g.Lc, Lq = m - Lp * g.Lc;
        t.P0 = g.nx * Lp + g.hs;
        t.Q0 = g.ny * Lq + g.ht;
    }
    return t;
}

// Raw operand values of a stage plus what decides which of them are real:
// the zero mask is applied when the values are written to LDS, after the
// stage's MFMA work, so the loads stay in flight during that work.
struct FwdMask {
    bool va, vb;  // this lane's A row / B column has data at this stage
    int zn;       // depth planes present in the stage (uniform)
};

__device__ __forceinline__ FwdMask fwd_load(const FwdArgs& a, const FwdThread& th, int stage,
                                            float (&ra)[kFwdAPer], float (&rb)[kFwdBPer])
{
    const ProjGeom& g = a.g;
    const int st = stage / a.nzc, zc = stage - st * a.nzc;
    const int sr = int(fdiv(uint32_t(st), g.fKc)), tc = st - sr * g.Kc;
    const int sp = sr - (g.nx - 1), tp = tc - (g.ny - 1);  // s', t'
    const int z0 = zc * kFwdZC, zn = min(kFwdZC, g.nz - z0);
    const int x = imod(g.hs - sp, g.nx), y = imod(g.ht - tp, g.ny);
    // B column: H[s'+u][t'+v][x][y][z0 .. z0+zn)
    // Loads are unconditional: lanes without data read element 0 of the array
    // and keep zero, so no load sits behind a branch.
    const bool vb = (th.hoff >= 0) & (unsigned(sp + th.u) < unsigned(g.ns)) & (unsigned(tp + th.v) < unsigned(g.nt));
    const float* pb = vb ? a.H + ((int64_t(sp) * g.nt + tp) * (int64_t(g.nx) * g.ny * g.nz) + th.hoff +
                                  (int64_t(x) * g.ny + y) * g.nz + z0)
                         : a.H;
#pragma unroll
    for (int z = 0; z < kFwdBPer; ++z) rb[z] = pb[z < zn ? z : zn - 1];  // uniform clamp, no branch
    // A row: gT[P][Q][z0 + zg + 4j]
    const int P = th.P0 - sp, Q = th.Q0 - tp;
    const bool va = (P >= 0) & (P < g.R) & (Q >= 0) & (Q < g.C);
    // pa points at depth z0 of the pixel (or at gT[0] for lanes without data);
    // the clamped depth min(zl, zn-1) lies in [0, zn), so every read stays
    // inside the pixel's run (or inside gT[0, zn)).
    const float* pa = va ? a.gT + ((int64_t(P) * g.C + Q) * g.nz + z0) : a.gT;
#pragma unroll
    for (int j = 0; j < kFwdAPer; ++j) {
        const int zl = th.zg + 4 * j;  // zg is the wave index: uniform
        ra[j] = pa[zl < zn ? zl : zn - 1];
    }
    FwdMask mk;
    mk.va = va;
    mk.vb = vb;
    mk.zn = zn;
    return mk;
}

__device__ __forceinline__ void fwd_store(float* As, float* Bs, const FwdThread& th, const FwdMask& mk,
                                          const float (&ra)[kFwdAPer], const float (&rb)[kFwdBPer])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int z = 0; z < kFwdBPer; ++z) Bs[z * kBStride + tid] = (mk.vb & (z < mk.zn)) ? rb[z] : 0.0f;
#pragma unroll
    for (int j = 0; j < kFwdAPer; ++j) {
        const int zl = th.zg + 4 * j;
        if (zl < kFwdZC) As[zl * kAStride + (tid & 63)] = (mk.va & (zl < mk.zn)) ? ra[j] : 0.0f;
    }
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) k_fwd_gemm(FwdArgs a)
{
    __shared__ float As[2][kFwdZC * kAStride];
    __shared__ float Bs[2][kFwdZC * kBStride];
    const int m0 = blockIdx.x * kMT, n0 = blockIdx.y * kNT, split = blockIdx.z;
    const int s_begin = int(int64_t(a.stages) * split / a.splits);
    const int s_end = int(int64_t(a.stages) * (split + 1) / a.splits);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool active = n0 + wave * 64 < a.Npad;
    f32x16 acc[2][2] = {}, tot[2][2] = {};
    float ra[kFwdAPer], rb[kFwdBPer];
    const FwdThread th = fwd_thread(a, m0, n0);
    FwdMask mk{};
    if (s_begin < s_end) {
        mk = fwd_load(a, th, s_begin, ra, rb);
        fwd_store(As[0], Bs[0], th, mk, ra, rb);
        __syncthreads();
    }
    int buf = 0, since = 0;
    for (int s = s_begin; s < s_end; ++s) {
        const bool more = s + 1 < s_end;
        if (more) mk = fwd_load(a, th, s + 1, ra, rb);
        if (active) mma_stage(As[buf], Bs[buf], kFwdZC, wave, lane, acc);
        if (++since == kFold) {
            fold(acc, tot);
            since = 0;
        }
        if (more) fwd_store(As[buf ^ 1], Bs[buf ^ 1], th, mk, ra, rb);
        __syncthreads();
        buf ^= 1;
    }
    fold(acc, tot);
    if (!active) return;
    float* out = a.partial + size_t(split) * a.Mpad * a.Npad;
    const int li = lane & 31, lk = lane >> 5;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + 32 * i + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int n = n0 + wave * 64 + 32 * j + li;
                out[size_t(m) * a.Npad + n] = tot[i][j][r];
            }
}

// f[p][q] = sum over splits of the partial tile entry of (lenslet, class).
__global__ void __launch_bounds__(256) k_fwd_reduce(const float* partial, int splits, int Mpad, int Npad,
                                                     ProjGeom g, float* f)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(g.R) * g.C) return;
    const int p = int(i / g.C), q = int(i - int64_t(p) * g.C);
    const int m = (p / g.nx) * g.Lc + q / g.ny;
    const int n = (p % g.nx) * g.ny + q % g.ny;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += double(partial[(size_t(s) * Mpad + m) * Npad + n]);
    f[i] = float(acc);
}

// gT[P][Q][z] = g[z][P][Q] through an LDS tile.
__global__ void __launch_bounds__(256) k_depth_last(const float* g, int nz, int plane, float* gT)
{
    __shared__ float tile[32][33];
    const int z0 = blockIdx.y * 32, p0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int z = z0 + r, p = p0 + tx;
        tile[r][tx] = (z < nz && p < plane) ? g[size_t(z) * plane + p] : 0.0f;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int p = p0 + r, z = z0 + tx;
        if (p < plane && z < nz) gT[size_t(p) * nz + z] = tile[tx][r];
    }
}

// ------------------------------------------------------------------ backward

constexpr int kBwdAPer = (kMT * kBwdKC + kThreads - 1) / kThreads;  // 4 pairs per thread
constexpr int kBwdBPer = kBwdKC;                                    // one column per thread, all rows

struct BwdArgs {
    const float* Ht;   // [ns][nt][nx][ny][nz]
    const float* f;    // [R][C]
    float* g;          // [nz][R][C]
    ProjGeom geo;
    int N;             // nx*ny*nz
    int K;             // Kr*Kc
};

// Thread t owns B column n0 + t = (cx, cy, z) and, in the A tile, row
// m0 + t/4 at the 4 consecutive pairs 4(t mod 4) .. 4(t mod 4)+3 of the stage.
// Per-element zero masks of a backward stage, bit j (A) and bit kk (B).
struct BwdMask {
    uint32_t a, b;
};

__device__ __forceinline__ BwdMask bwd_load(const BwdArgs& a, int k0, int m, int P0, int Q0, int64_t hoff, int cx,
                                            int cy, float (&ra)[kBwdAPer], float (&rb)[kBwdBPer])
{
    BwdMask mk{0u, 0u};
    const ProjGeom& g = a.geo;
    const int tid = threadIdx.x;
    // A: f[P0 - r][Q0 - r2] for this thread's 4 pairs
#pragma unroll
    for (int j = 0; j < kBwdAPer; ++j) {
        const int k = k0 + 4 * (tid & 3) + j;
        const int ri = int(fdiv(uint32_t(k), g.fKc)), r2i = k - ri * g.Kc;
        const int p = P0 - (ri - (g.nx - 1)), q = Q0 - (r2i - (g.ny - 1));
        const bool ok = (m < g.M) & (k < a.K) & (p >= 0) & (p < g.R) & (q >= 0) & (q < g.C);
        ra[j] = a.f[ok ? int64_t(p) * g.C + q : 0];
        mk.a |= uint32_t(ok) << j;
    }
    // B: Ht[r+cx][r2+cy][x][y][z]; (r, r2, x, y) are uniform over the workgroup
    const int64_t cell = int64_t(g.nx) * g.ny * g.nz;
#pragma unroll
    for (int kk = 0; kk < kBwdKC; ++kk) {
        const int k = k0 + kk;
        const int ri = int(fdiv(uint32_t(k), g.fKc)), r2i = k - ri * g.Kc;
        const int r = ri - (g.nx - 1), r2 = r2i - (g.ny - 1);
        const int x = imod(g.hs - r, g.nx), y = imod(g.ht - r2, g.ny);
        const bool valid = (hoff >= 0) & (k < a.K) & (unsigned(r + cx) < unsigned(g.ns)) &
                           (unsigned(r2 + cy) < unsigned(g.nt));
        const int64_t base = (int64_t(r) * g.nt + r2) * cell + (int64_t(x) * g.ny + y) * g.nz;
        rb[kk] = a.Ht[valid ? base + hoff : 0];
        mk.b |= uint32_t(valid) << kk;
    }
    return mk;
}

__device__ __forceinline__ void bwd_store(float* As, float* Bs, const BwdMask& mk, const float (&ra)[kBwdAPer],
                                          const float (&rb)[kBwdBPer])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kBwdAPer; ++j)
        As[(4 * (tid & 3) + j) * kAStride + (tid >> 2)] = ((mk.a >> j) & 1u) ? ra[j] : 0.0f;
#pragma unroll
    for (int kk = 0; kk < kBwdKC; ++kk) Bs[kk * kBStride + tid] = ((mk.b >> kk) & 1u) ? rb[kk] : 0.0f;
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) k_bwd_gemm(BwdArgs a)
{
    __shared__ float As[2][kBwdKC * kAStride];
    __shared__ float Bs[2][kBwdKC * kBStride];
    const ProjGeom& g = a.geo;
    const int m0 = blockIdx.x * kMT, n0 = blockIdx.y * kNT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool active = n0 + wave * 64 < a.N;
    // this thread's B column (cx, cy, z) and A row
    const int n = n0 + int(threadIdx.x);
    int cx = 0, cy = 0;
    int64_t hoff = -1;
    if (n < a.N) {
        const int c = int(fdiv(uint32_t(n), g.fnz));
        const int z = n - c * g.nz;
        cx = int(fdiv(uint32_t(c), g.fny));
        cy = c - cx * g.ny;
        hoff = (int64_t(cx) * g.nt + cy) * (int64_t(g.nx) * g.ny * g.nz) + z;
    }
    const int m = m0 + int(threadIdx.x >> 2);
    int P0 = 0, Q0 = 0;
    if (m < g.M) {
        const int Lp = m / g.Lc, Lq = m - Lp * g.Lc;
        P0 = g.nx * Lp + g.hs;
        Q0 = g.ny * Lq + g.ht;
    }
    f32x16 acc[2][2] = {}, tot[2][2] = {};
    float ra[kBwdAPer], rb[kBwdBPer];
    const int stages = (a.K + kBwdKC - 1) / kBwdKC;
    BwdMask mk = bwd_load(a, 0, m, P0, Q0, hoff, cx, cy, ra, rb);
    bwd_store(As[0], Bs[0], mk, ra, rb);
    __syncthreads();
    int buf = 0, since = 0;
    for (int s = 0; s < stages; ++s) {
        const bool more = s + 1 < stages;
        if (more) mk = bwd_load(a, (s + 1) * kBwdKC, m, P0, Q0, hoff, cx, cy, ra, rb);
        if (active) mma_stage(As[buf], Bs[buf], kBwdKC, wave, lane, acc);
        if (++since == kFold) {
            fold(acc, tot);
            since = 0;
        }
        if (more) bwd_store(As[buf ^ 1], Bs[buf ^ 1], mk, ra, rb);
        __syncthreads();
        buf ^= 1;
    }
    fold(acc, tot);
    if (!active) return;
    const int li = lane & 31, lk = lane >> 5;
    const size_t plane = size_t(g.R) * g.C;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int nn = n0 + wave * 64 + 32 * j + li;
        if (nn >= a.N) continue;
        const int c = int(fdiv(uint32_t(nn), g.fnz));
        const int zz = nn - c * g.nz;
        const int ccx = int(fdiv(uint32_t(c), g.fny)), ccy = c - ccx * g.ny;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + 32 * i + 8 * (r >> 2) + 4 * lk + (r & 3);
                if (m >= g.M) continue;
                const int Lp = m / g.Lc, Lq = m - Lp * g.Lc;
                const int P = g.nx * Lp + ccx, Q = g.ny * Lq + ccy;
                if (P < g.R && Q < g.C) a.g[zz * plane + size_t(P) * g.C + Q] = tot[i][j][r];
            }
    }
}

int g_cus_proj = 256;

int fwd_splits(const ProjGeom& g, int mtiles, int ntiles, int stages)
{
    const int want = (2 * g_cus_proj) / (mtiles * ntiles);  // one round at two workgroups per CU
    return std::max(1, std::min({want, 64, std::max(1, stages / 8)}));
}

}  // namespace

hipError_t project_init(int max_lds)
{
    (void)max_lds;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        g_cus_proj = cus;
    return hipSuccess;
}

// Workspace of the forward projection: g with depth innermost, then the
// split-K partial tiles.
size_t forward_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const ProjGeom g = make_geom(s, R, C);
    const int N = g.nx * g.ny, Npad = (N + 63) / 64 * 64;
    const int mtiles = (g.M + kMT - 1) / kMT, ntiles = (N + kNT - 1) / kNT;
    const int nzc = (g.nz + kFwdZC - 1) / kFwdZC;
    const int stages = g.Kr * g.Kc * nzc;
    const int splits = fwd_splits(g, mtiles, ntiles, stages);
    const size_t gT = size_t(g.nz) * g.R * g.C * sizeof(float);
    const size_t part = size_t(splits) * size_t(mtiles * kMT) * size_t(ntiles * kNT) * sizeof(float);
    return (gT + 255) / 256 * 256 + part;
}

hipError_t launch_forward_ws(const float* H, const lfbp_shape& s, const float* gin, int64_t R, int64_t C, float* f,
                             void* ws, hipStream_t stream)
{
    const ProjGeom g = make_geom(s, R, C);
    FwdArgs a;
    a.H = H;
    a.g = g;
    a.N = g.nx * g.ny;
    const int mtiles = (g.M + kMT - 1) / kMT, ntiles = (a.N + kNT - 1) / kNT;
    a.Mpad = mtiles * kMT;
    a.Npad = ntiles * kNT;
    a.nzc = (g.nz + kFwdZC - 1) / kFwdZC;
    a.stages = g.Kr * g.Kc * a.nzc;
    a.splits = fwd_splits(g, mtiles, ntiles, a.stages);
    const size_t gT_bytes = (size_t(g.nz) * g.R * g.C * sizeof(float) + 255) / 256 * 256;
    float* gT = static_cast<float*>(ws);
    a.gT = gT;
    a.partial = reinterpret_cast<float*>(static_cast<char*>(ws) + gT_bytes);
    const int plane = g.R * g.C;
    hipLaunchKernelGGL(k_depth_last, dim3(unsigned((plane + 31) / 32), unsigned((g.nz + 31) / 32)), dim3(256), 0,
                       stream, gin, g.nz, plane, gT);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fwd_gemm, dim3(unsigned(mtiles), unsigned(ntiles), unsigned(a.splits)), dim3(kThreads), 0,
                       stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t npix = int64_t(g.R) * g.C;
    hipLaunchKernelGGL(k_fwd_reduce, dim3(unsigned((npix + 255) / 256)), dim3(256), 0, stream, a.partial, a.splits,
                       a.Mpad, a.Npad, g, f);
    return hipGetLastError();
}

hipError_t launch_forward(const float* H, const lfbp_shape& s, const float* g, int64_t R, int64_t C, float* f,
                          hipStream_t stream)
{
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, forward_workspace_bytes(s, R, C), stream);
    if (e != hipSuccess) return e;
    e = launch_forward_ws(H, s, g, R, C, f, ws, stream);
    const hipError_t e2 = hipFreeAsync(ws, stream);
    return e != hipSuccess ? e : e2;
}

hipError_t launch_backward(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                           hipStream_t stream)
{
    BwdArgs a;
    a.Ht = Ht;
    a.f = f;
    a.g = g;
    a.geo = make_geom(s, R, C);
    a.N = a.geo.nx * a.geo.ny * a.geo.nz;
    a.K = a.geo.Kr * a.geo.Kc;
    const int mtiles = (a.geo.M + kMT - 1) / kMT, ntiles = (a.N + kNT - 1) / kNT;
    hipLaunchKernelGGL(k_bwd_gemm, dim3(unsigned(mtiles), unsigned(ntiles)), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace lfbp
