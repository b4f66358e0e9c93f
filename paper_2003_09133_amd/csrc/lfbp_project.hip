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

// Operand fetch of one forward stage (stage = one (s', t') pair and one chunk
// of up to kFwdZC depth planes).  Every B column (pixel class (u,v)) and every
// A row (lenslet) needs one contiguous run of <= kFwdZC floats: H[s'+u][t'+v]
// [x][y][z0..] and gT[P][Q][z0..].  Each run is read as the kFwdVPR aligned
// 16-byte vectors that cover it (consecutive lanes take consecutive vectors of
// a run), and the vectors are scattered into the LDS tile when it is written,
// after the stage's MFMA work.  A 16-byte aligned vector that holds at least
// one element of the run never leaves the run's page, so the reads need no
// bounds branch; elements outside the run are written to LDS as zeros.
constexpr int kFwdVPR = (kFwdZC + 3 + 3) / 4;                           // vectors per run: 7
constexpr int kFwdBSlots = kNT * kFwdVPR / kThreads;                     // 7 per thread
constexpr int kFwdASlots = (kMT * kFwdVPR + kThreads - 1) / kThreads;    // 2 per thread
static_assert(kNT * kFwdVPR % kThreads == 0, "B slots must tile the workgroup");

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct FwdArgs {
    const float* H;    // [ns][nt][nx][ny][nz]
    const float* gT;   // [R][C][nz]  (g with depth innermost)
    float* partial;    // [splits][Mpad][Npad]
    ProjGeom g;
    int N, Npad, Mpad;
    int stages;        // Kr*Kc*nzc
    int nzc;           // depth chunks
    int splits;
    int phaseH;        // (address of H / 4) mod 4
    int phaseG;        // (address of gT / 4) mod 4
};

// Loaded vectors of one stage and, per slot, the run's offset inside its first
// vector (bits 0-1) and whether the run exists (bit 2).
struct FwdRegs {
    u32x4 b[kFwdBSlots];
    u32x4 a[kFwdASlots];
    uint32_t bmeta[kFwdBSlots];
    uint32_t ameta[kFwdASlots];
    int zn;  // depth planes present in the stage (uniform)
};

__device__ __forceinline__ void fwd_load(const FwdArgs& a, int m0, int n0, int stage, FwdRegs& R)
{
    const ProjGeom& g = a.g;
    const int st = stage / a.nzc, zc = stage - st * a.nzc;
    const int sr = int(fdiv(uint32_t(st), g.fKc)), tc = st - sr * g.Kc;
    const int sp = sr - (g.nx - 1), tp = tc - (g.ny - 1);  // s', t'
    const int z0 = zc * kFwdZC, zn = min(kFwdZC, g.nz - z0);
    const int x = imod(g.hs - sp, g.nx), y = imod(g.ht - tp, g.ny);
    const int64_t cell = int64_t(g.nx) * g.ny * g.nz;
    const int64_t sbase = (int64_t(sp) * g.nt + tp) * cell + (int64_t(x) * g.ny + y) * g.nz + z0;
    const int tid = threadIdx.x;
    R.zn = zn;
#pragma unroll
    for (int j = 0; j < kFwdBSlots; ++j) {
        const int e = tid + j * kThreads;
        const int nl = e / kFwdVPR, k = e - nl * kFwdVPR;
        const int n = n0 + nl;
        const int u = int(fdiv(uint32_t(n), g.fny)), v = n - u * g.ny;
        const bool valid = (n < a.N) & (unsigned(sp + u) < unsigned(g.ns)) & (unsigned(tp + v) < unsigned(g.nt));
        const int64_t rs = sbase + (int64_t(u) * g.nt + v) * cell;
        const int lead = valid ? int((rs + a.phaseH) & 3) : 0;
        const int64_t vb = valid ? rs - lead : -int64_t(a.phaseH);
        const int kmax = (lead + zn - 1) >> 2;
        const int kk = k < kmax ? k : kmax;                 // always a vector that overlaps the run
        R.b[j] = *reinterpret_cast<const u32x4*>(a.H + vb + 4 * kk);
        R.bmeta[j] = uint32_t(lead) | (uint32_t(valid) << 2);
    }
#pragma unroll
    for (int j = 0; j < kFwdASlots; ++j) {
        const int e = tid + j * kThreads;
        const int ml = e / kFwdVPR, k = e - ml * kFwdVPR;
        const int m = m0 + ml;
        const int Lp = m / g.Lc, Lq = m - Lp * g.Lc;
        const int P = g.nx * Lp + g.hs - sp, Q = g.ny * Lq + g.ht - tp;
        const bool valid = (ml < kMT) & (m < g.M) & (P >= 0) & (P < g.R) & (Q >= 0) & (Q < g.C);
        const int64_t rs = (int64_t(P) * g.C + Q) * g.nz + z0;
        const int lead = valid ? int((rs + a.phaseG) & 3) : 0;
        const int64_t vb = valid ? rs - lead : -int64_t(a.phaseG);
        const int kmax = (lead + zn - 1) >> 2;
        const int kk = k < kmax ? k : kmax;
        R.a[j] = *reinterpret_cast<const u32x4*>(a.gT + vb + 4 * kk);
        R.ameta[j] = uint32_t(lead) | (uint32_t(valid) << 2);
    }
}

// Scatter the stage's vectors into As[z][m] and Bs[z][n]: vector k of a run
// holds depths 4k - lead .. 4k - lead + 3, so the kFwdVPR vectors of a run
// write every depth 0..kFwdZC-1 of its row or column exactly once.
__device__ __forceinline__ void fwd_store(float* As, float* Bs, const FwdRegs& R)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kFwdBSlots; ++j) {
        const int e = tid + j * kThreads;
        const int nl = e / kFwdVPR, k = e - nl * kFwdVPR;
        const int lead = int(R.bmeta[j] & 3u);
        const bool valid = (R.bmeta[j] >> 2) & 1u;
        const float v4[4] = {__uint_as_float(R.b[j].x), __uint_as_float(R.b[j].y), __uint_as_float(R.b[j].z),
                             __uint_as_float(R.b[j].w)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int z = 4 * k + q - lead;
            if (z >= 0 && z < kFwdZC) Bs[z * kBStride + nl] = (valid & (z < R.zn)) ? v4[q] : 0.0f;
        }
    }
#pragma unroll
    for (int j = 0; j < kFwdASlots; ++j) {
        const int e = tid + j * kThreads;
        const int ml = e / kFwdVPR, k = e - ml * kFwdVPR;
        if (ml >= kMT) continue;
        const int lead = int(R.ameta[j] & 3u);
        const bool valid = (R.ameta[j] >> 2) & 1u;
        const float v4[4] = {__uint_as_float(R.a[j].x), __uint_as_float(R.a[j].y), __uint_as_float(R.a[j].z),
                             __uint_as_float(R.a[j].w)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int z = 4 * k + q - lead;
            if (z >= 0 && z < kFwdZC) As[z * kAStride + ml] = (valid & (z < R.zn)) ? v4[q] : 0.0f;
        }
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
    FwdRegs regs;
    if (s_begin < s_end) {
        fwd_load(a, m0, n0, s_begin, regs);
        fwd_store(As[0], Bs[0], regs);
        __syncthreads();
    }
    int buf = 0, since = 0;
    for (int s = s_begin; s < s_end; ++s) {
        const bool more = s + 1 < s_end;
        if (more) fwd_load(a, m0, n0, s + 1, regs);
        if (active) mma_stage(As[buf], Bs[buf], kFwdZC, wave, lane, acc);
        if (++since == kFold) {
            fold(acc, tot);
            since = 0;
        }
        if (more) fwd_store(As[buf ^ 1], Bs[buf ^ 1], regs);
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
    // and advance by one pair per row of the stage: one division per stage,
    // then scalar increments (r2 up by one, x and y down by one, cyclically).
    const int64_t cell = int64_t(g.nx) * g.ny * g.nz;
    int ri = int(fdiv(uint32_t(k0), g.fKc));
    int r2i = k0 - ri * g.Kc;
    int x = imod(g.hs - (ri - (g.nx - 1)), g.nx);
    int y = imod(g.ht - (r2i - (g.ny - 1)), g.ny);
    const int y_first = imod(g.ht + g.ny - 1, g.ny);  // y at r2 = -(ny-1)
#pragma unroll
    for (int kk = 0; kk < kBwdKC; ++kk) {
        const int r = ri - (g.nx - 1), r2 = r2i - (g.ny - 1);
        const bool valid = (hoff >= 0) & (k0 + kk < a.K) & (unsigned(r + cx) < unsigned(g.ns)) &
                           (unsigned(r2 + cy) < unsigned(g.nt));
        const int64_t base = (int64_t(r) * g.nt + r2) * cell + (int64_t(x) * g.ny + y) * g.nz;
        rb[kk] = a.Ht[valid ? base + hoff : 0];
        mk.b |= uint32_t(valid) << kk;
        if (++r2i == g.Kc) {
            r2i = 0;
            ++ri;
            x = x == 0 ? g.nx - 1 : x - 1;
            y = y_first;
        } else {
            y = y == 0 ? g.ny - 1 : y - 1;
        }
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
    a.phaseH = int((reinterpret_cast<uintptr_t>(H) / 4) % 4);
    a.phaseG = int((reinterpret_cast<uintptr_t>(gT) / 4) % 4);
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
