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
// Operand records.  Each product runs as one GEMM kernel over "records": the
// reduction runs in stages of 22 indices, split into two halves of 11 (lanes
// 0-31 of a wavefront feed the matrix cores from the first half, lanes 32-63
// from the second, which is a fixed permutation of the reduction order), and
// one stage of one operand row or column is a record of 24 floats: the halves
// at offsets 0 and 12, each padded with one zero.  Before the GEMM the
// operands are copied into records, with explicit zeros wherever the
// formulation above has zeros:
//   forward  B[stage][class][24] from H; A from g split by pixel phase,
//            one block per (px, py, depth chunk) holding a record per lenslet
//            of the phase plane, with zero lenslets around the image, so the
//            record of lenslet (Lp,Lq) at stage (s',t',chunk) is the record at
//            lenslet offset (floor((hs-s')/nx), floor((ht-t')/ny)) in phase
//            plane ((hs-s') mod nx, (ht-t') mod ny);
//   backward A[stage][lenslet][24] from f and B[stage][column][24] from H'.
// A lane reads its half of a record as three 16-byte vectors and hands the
// values to the matrix cores straight from registers.  The records of one
// block (one stage of one operand, or one phase plane and depth chunk of g)
// are stored vector-major, [vector v][record][half][4 floats], so that each
// 16-byte load instruction of a wavefront reads 1 KB of consecutive memory.
//
// GEMM kernel.  A workgroup of 4 wavefronts owns a 64 x 256 output tile; wave
// w owns columns 64w..64w+63 as 2 x 2 MFMA tiles of 32 x 32 and works on its
// own: each lane loads the next stage's records (its two rows and two columns)
// into registers while the matrix cores consume the current stage, so there
// is neither LDS staging nor a workgroup barrier in the loop.  Accumulation is
// two-level: the MFMA accumulators are folded into float32 sums held in LDS
// (one region per wavefront) every few stages, so rounding grows with the
// chunk length, not with the ~10^5-10^6 terms of a full sum.  The forward
// splits the reduction over workgroups (partials added in a fixed order, in
// float64, by a second kernel, so results are deterministic); the backward
// needs no split.  Workgroups that read the same operand slab are placed on
// the same XCD (L2).  Stages whose A records are zero for a whole row tile
// (source pixels outside the image) are not run: the forward drops such patch
// rows and gives each row tile splits in proportion to what is left (a work
// table maps workgroups to row tiles, column tiles and splits); the gradient
// with respect to H drops such lenslet rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lfbp_internal.h"

namespace lfbp {

hipError_t put_words(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t stream);

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x3 __attribute__((ext_vector_type(3)));

namespace {

constexpr int kThreads = 256;
constexpr int kMT = 64;              // output rows per workgroup (shared by its 4 waves)
constexpr int kNT = 256;             // output columns per workgroup (64 per wave)
constexpr int kHalf = 11;            // MFMA steps per stage (two reduction indices each)
constexpr int kStageK = 2 * kHalf;   // reduction indices per stage
constexpr int kRec = 24;             // floats per record (halves at 0 and 12)
constexpr int kRecVec = kRec / 4;    // 16-byte vectors per record (3 per half)
constexpr int kFoldGroups = 11;      // groups of three stages between folds of the MFMA accumulators
constexpr int kXcds = 8;
constexpr int kTargetBlocks = 512;

struct ProjGeom {
    int ns, nt, nx, ny, nz, hs, ht, R, C;
    int Lr, Lc;   // lenslets per image side (ceil(R/nx), ceil(C/ny))
    int M;        // Lr*Lc
    int Kr, Kc;   // ns+nx-1, nt+ny-1
    FastDiv fKc, fnx, fny, fnz, fLc;
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
    g.fnx = make_fastdiv(uint32_t(g.nx));
    g.fny = make_fastdiv(uint32_t(g.ny));
    g.fnz = make_fastdiv(uint32_t(g.nz));
    g.fLc = make_fastdiv(uint32_t(g.Lc));
    return g;
}

__device__ __forceinline__ int imod(int a, int n)
{
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// Reduction index inside a stage of record slot q (0..23); -1 for the pads.
__device__ __forceinline__ int slot_k(int q)
{
    const int h = q >= 12 ? 1 : 0, j = q - 12 * h;
    return j < kHalf ? kHalf * h + j : -1;
}


// Forward output columns are classes (u, v) arranged in boxes of bu x bv
// classes, one box per wavefront (64 columns): the B records of a box are
// zero outside a window of (ns + bu - 1) x (nt + bv - 1) patch shifts, so a
// wavefront runs only the stages of its window.  Box b = (bi, bj), bj fastest
// (nbv boxes along v); column 64 b + du * bv + dv is class
// (bi * bu + du, bj * bv + dv).
struct ClassBoxes {
    int bu, bv, nbv, boxes;
};

__device__ __forceinline__ bool class_of_col(const ClassBoxes& c, int nx, int ny, int n, int& u, int& v)
{
    const int b = n >> 6, k = n & 63;
    if (b >= c.boxes || k >= c.bu * c.bv) return false;
    const int bi = b / c.nbv, bj = b - bi * c.nbv;
    const int du = k / c.bv, dv = k - du * c.bv;
    u = bi * c.bu + du;
    v = bj * c.bv + dv;
    return u < nx && v < ny;
}

__device__ __forceinline__ int col_of_class(const ClassBoxes& c, int u, int v)
{
    const int bi = u / c.bu, bj = v / c.bv;
    return (bi * c.nbv + bj) * 64 + (u - bi * c.bu) * c.bv + (v - bj * c.bv);
}

// Forward walk of a box's window, Rw patch-row shifts by Cw patch-column
// shifts (times the depth chunks, fastest): the column shifts are taken by
// residue b modulo ny, and within a residue class all Rw row shifts, each with
// the class's column shifts b, b + ny, b + 2 ny, ... innermost.  Consecutive
// stages then read the same phase plane of g one lenslet apart, so they share
// all but one of their A records.  The first r0 residues hold q1 = q0 + 1
// column shifts, the others q0 (Cw = ny q0 + r0); n1 = r0 Rw q1 window
// positions belong to the first group (n1 and the divisors by Rw q1, Rw q0
// are taken per wavefront, whose Rw is the count of rows its row tile needs).
struct WindowWalk {
    int r0, q0, q1;
    FastDiv fq1, fq0;   // by q1, q0 (a divisor of 0 stored as 1)
};

struct GemmArgs {
    const float* A;   // left operand records
    const float* B;   // right operand records [stage][Npad][kRec]
    float* out;       // forward: partial tiles [splits][Mpad][Npad]; backward: g [nz][R][C]
    // backward, Richardson-Lucy update (Eq. 2): when set, the result v of a
    // voxel is written as gprev * v / norm (0 where norm is 0)
    const float* gprev;
    const float* norm;
    ProjGeom g;
    int M, N, Mpad, Npad;
    int mtiles, ntiles;
    int stages, splits;
    // forward: A blocks are (px, py, depth chunk), LRp x LCp records each
    int nzc, LRp, LCp, padP, padQ;
    FastDiv fnzc;
    ClassBoxes cb;    // forward column layout
    WindowWalk walk;  // forward order of a box's window
    // forward work table: tab[mt] (mt <= mtiles) is the first partial-sum slot
    // of row tile mt (its splits: tab[mt+1] - tab[mt]), and
    // tab[mtiles + 1 + L] = ((mt * ntiles + nt) << 6) | split for workgroup L
    const uint32_t* tab;
    int nwg;
};

// Geometry of the forward depth chunking and of the phase-split copy of g.
struct FwdLayout {
    int nzc;            // depth chunks of kStageK planes
    int stages;         // Kr*Kc*nzc
    int padP, padQ;     // zero lenslets before the image (rows, columns)
    int LRp, LCp;       // padded lenslet grid
};

FwdLayout fwd_layout(const ProjGeom& g)
{
    FwdLayout L;
    L.nzc = (g.nz + kStageK - 1) / kStageK;
    L.stages = g.Kr * g.Kc * L.nzc;
    // lenslet offsets floor((hs - s')/nx) over s' in [-(nx-1), ns-1] span
    // [-ceil(hs/nx), floor((hs+nx-1)/nx)] = [-pad, pad]
    L.padP = (g.hs + g.nx - 1) / g.nx;
    L.padQ = (g.ht + g.ny - 1) / g.ny;
    L.LRp = g.Lr + 2 * L.padP;
    L.LCp = g.Lc + 2 * L.padQ;
    return L;
}

// Forward stage (s', t', chunk) of stage index s: Kr*Kc*nzc stages, chunk fastest.
struct FwdStage {
    int sp, tp, zc, px, py, dP, dQ;
};

__device__ __forceinline__ FwdStage fwd_stage(const ProjGeom& g, const FastDiv& fnzc, int nzc, int s)
{
    FwdStage t;
    const int st = int(fdiv(uint32_t(s), fnzc));
    t.zc = s - st * nzc;
    const int sr = int(fdiv(uint32_t(st), g.fKc)), tc = st - sr * g.Kc;
    t.sp = sr - (g.nx - 1);
    t.tp = tc - (g.ny - 1);
    const int e = g.hs - t.sp, f = g.ht - t.tp;
    t.px = imod(e, g.nx);
    t.py = imod(f, g.ny);
    t.dP = (e - t.px) / g.nx;   // exact: floor(e / nx)
    t.dQ = (f - t.py) / g.ny;
    return t;
}

// The window rows of forward box `box` that row tile mt needs: a window row
// ir is the patch-row shift s' = ir - u1 (u1 the box's last class row), and
// its A records are all zero (every lenslet row of the tile sees a source
// row P = nx Lp + hs - s' outside the image) unless s' lies in
// [nx Lp_lo + hs - (R - 1), nx Lp_hi + hs].  Returns the count, and the first
// row in ir_lo.  The host sizes the splits of each row tile with it, the
// GEMM walks only these rows.
__host__ __device__ inline int fwd_tile_rows(const ProjGeom& g, const ClassBoxes& cb, int mt, int box, int& ir_lo)
{
    const int bi = box / cb.nbv;
    const int u1 = min(g.nx, (bi + 1) * cb.bu) - 1, Rw = g.ns + cb.bu - 1;
    const int m_lo = mt * kMT, m_hi = min(g.M - 1, mt * kMT + kMT - 1);
    const int lp_lo = m_lo / g.Lc, lp_hi = m_hi / g.Lc;
    ir_lo = max(0, g.nx * lp_lo + g.hs - (g.R - 1) + u1);
    const int ir_hi = min(Rw - 1, g.nx * lp_hi + g.hs + u1);
    return max(0, ir_hi - ir_lo + 1);
}

// --------------------------------------------------------------- GEMM kernel

struct Frag {
    f32x4 a[2][3];   // rows 32i + (lane mod 32), this lane's half of the stage
    f32x4 b[2][3];   // columns 32j + (lane mod 32)
};

// Record blocks are read through buffer resources: a wavefront-uniform base
// and size in scalar registers, this lane's 32-bit byte offset in a vector
// register, the vector plane's offset in a scalar register.  No per-load
// address arithmetic or address registers in the vector file, and a read
// outside the block returns zeros instead of touching other memory.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format

__device__ __forceinline__ Rsrc make_rsrc(const char* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), short(0), int(bytes), kRsrcWord3);
}

__device__ __forceinline__ f32x4 load_vec(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), int(soff), 0));
}

// ra, rb: the stage's A and B record blocks; oa, ob: this lane's (record,
// half) byte offsets; sa, sb: bytes between the vector planes of a block.
__device__ __forceinline__ void load_frag(Rsrc ra, Rsrc rb, const uint32_t (&oa)[2], const uint32_t (&ob)[2],
                                          uint32_t sa, uint32_t sb, Frag& f)
{
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 3; ++v) f.a[i][v] = load_vec(ra, oa[i], v * sa);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 3; ++v) f.b[j][v] = load_vec(rb, ob[j], v * sb);
}

__device__ __forceinline__ void mma_stage(const Frag& f, f32x16 (&acc)[2][2])
{
#pragma unroll
    for (int s = 0; s < kHalf; ++s) {
        const float a0 = f.a[0][s >> 2][s & 3], a1 = f.a[1][s >> 2][s & 3];
        const float b0 = f.b[0][s >> 2][s & 3], b1 = f.b[1][s >> 2][s & 3];
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    // The last float of each half (a zero pad) is never read by the MFMAs.  Keep
    // the whole loaded vector live until here anyway: otherwise its register is
    // handed out while the load that fills it is still in flight, and the
    // reuse forces a wait for the prefetch of later stages.
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        asm volatile("" ::"v"(f.a[i][2]));
        asm volatile("" ::"v"(f.b[i][2]));
    }
    // Spread the scalar work of the region (the next stage's record
    // addresses) between the MFMAs: a wavefront issues it while its own MFMAs
    // run, instead of in one block during which neither of the two wavefronts
    // sharing the SIMD, which the shared matrix core keeps in step, has an
    // MFMA ready.
#pragma unroll
    for (int s = 0; s < 4 * kHalf; ++s) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x004, 3, 0);   // up to three scalar ALU instructions
    }
}

// T[tile][quad][lane] += accumulator registers 4*quad .. 4*quad+3; acc = 0.
__device__ __forceinline__ void fold(f32x16 (&acc)[2][2], f32x4 (*T)[4][64], int lane)
{
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                f32x4 v = T[2 * i + j][q][lane];
                v.x += acc[i][j][4 * q];
                v.y += acc[i][j][4 * q + 1];
                v.z += acc[i][j][4 * q + 2];
                v.w += acc[i][j][4 * q + 3];
                T[2 * i + j][q][lane] = v;
            }
            acc[i][j] = f32x16{};
        }
}

// Workgroup -> (m tile, n tile, split), with consecutive logical indices (same
// n tile / split, all m tiles) on the same XCD: dispatch deals workgroups to
// the XCDs round-robin.
__device__ __forceinline__ void tile_of_block(const GemmArgs& a, int& mt, int& nt, int& split)
{
    const int nb = a.mtiles * a.ntiles * a.splits;
    const int b = int(blockIdx.x);
    const int x = b % kXcds, q = nb / kXcds, r = nb % kXcds;
    const int L = x * q + min(x, r) + b / kXcds;
    mt = L % a.mtiles;
    const int rest = L / a.mtiles;
    nt = rest % a.ntiles;
    split = rest / a.ntiles;
}

// What a GEMM launch computes (operand records and epilogue).
enum GemmMode { kModeFwd = 0, kModeBwd = 1, kModeGradH = 2 };

template <int kMode>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) k_gemm(GemmArgs a)
{
    constexpr bool kFwd = kMode == kModeFwd;
    __shared__ f32x4 tot[kThreads / 64][4][4][64];   // per wave: 4 tiles x 16 sums x 64 lanes
    int mt, ntile, split, splits = a.splits, slot = 0;
    if (kFwd) {
        // logical workgroup L (consecutive L on one XCD, as in tile_of_block)
        // -> its row tile, column tile and split, from the work table
        const int b = int(blockIdx.x), x = b % kXcds, q = a.nwg / kXcds, r = a.nwg % kXcds;
        const int L = x * q + min(x, r) + b / kXcds;
        const uint32_t e = a.tab[a.mtiles + 1 + L];
        const int tile = int(e >> 6);
        split = int(e & 63u);
        mt = tile / a.ntiles;
        ntile = tile - mt * a.ntiles;
        slot = int(a.tab[mt]) + split;
        splits = int(a.tab[mt + 1] - a.tab[mt]);
    } else {
        tile_of_block(a, mt, ntile, split);
    }
    const ProjGeom& g = a.g;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = int(threadIdx.x) & 63;
    // This wavefront's 64 x 64 output block at rows m0, columns nb: a
    // workgroup is one 64-row tile of 256 columns, 64 per wavefront (forward:
    // one class box per wavefront).
    const int m0 = mt * kMT;
    const int nb = ntile * kNT + 64 * wave;

    // This wavefront's window: the stages whose B records can be nonzero in
    // its columns, w_cnt of them (window index i: forward position fwd_pos(i),
    // otherwise stage w_base + i).
    // Forward: the box's patch shifts, s' + u inside [0, ns) and t' + v
    // inside [0, nt) for some class (u, v) of the box, in a window of the
    // full box size for every box (a box cut short by the cell edge pads it
    // at the far end), less the patch rows whose A records are zero for the
    // whole row tile (fwd_tile_rows), walked in the order WindowWalk
    // describes (consecutive stages share their A records).  Backward: the
    // reduction pairs with r + cx inside [0, ns) for some column of the
    // workgroup, a contiguous run of stages (columns are (cx, cy, z) with z
    // fastest, so a workgroup spans few cx).  Gradient with respect to H:
    // the run of stages (22 lenslets each) over the lenslet rows whose image
    // rows the tile's r reach, or none for a tile none of whose entries is
    // kept.
    int w_cnt = a.stages, w_base = 0, sr0 = 0, tc0 = 0, Rw = 1;
    if (kFwd) {
        const int b = ntile * (kNT / 64) + wave;
        if (b >= a.cb.boxes) {
            w_cnt = 0;
        } else {
            const int bi = b / a.cb.nbv, bj = b - bi * a.cb.nbv;
            const int u1 = min(g.nx, (bi + 1) * a.cb.bu) - 1, v1 = min(g.ny, (bj + 1) * a.cb.bv) - 1;
            int ir_lo;
            Rw = fwd_tile_rows(g, a.cb, mt, b, ir_lo);   // the rows with nonzero A records
            sr0 = g.nx - 1 - u1 + ir_lo;   // s' from -u1 + ir_lo (shifted by nx - 1)
            tc0 = g.ny - 1 - v1;
            w_cnt = Rw * (g.nt + a.cb.bv - 1) * a.nzc;
        }
    } else if (kMode == kModeBwd) {
        // the workgroup's columns (one window for its four wavefronts keeps
        // them on the same stages, sharing the A records)
        const int nlo = ntile * kNT;
        if (nlo >= a.N) {
            w_cnt = 0;
        } else {
            const int nhi = min(nlo + kNT - 1, a.N - 1);
            const int cxlo = nlo / g.nz / g.ny, cxhi = nhi / g.nz / g.ny;
            // r + nx - 1 from nx-1-cxhi to nx-2-cxlo+ns: reduction indices [klo, khi)
            const int klo = (g.nx - 1 - cxhi) * g.Kc, khi = (g.nx - 1 - cxlo + g.ns) * g.Kc;
            w_base = klo / kStageK;
            w_cnt = (khi + kStageK - 1) / kStageK - w_base;
        }
    }
    if (kMode == kModeGradH) {
        // rows (r, r2) of this tile and columns (x, y, z) of the workgroup: an
        // entry is kept only when 0 <= r - x < ns, so a tile with no such pair
        // has nothing to compute
        const int rlo = m0 / g.Kc, rhi = min(m0 + kMT - 1, a.M - 1) / g.Kc;
        const int nlo = ntile * kNT, nhi = min(nlo + kNT - 1, a.N - 1);
        const int xlo = nlo / g.nz / g.ny, xhi = nhi / g.nz / g.ny;
        if (m0 >= a.M || rhi < xlo || rlo - xhi > g.ns - 1) {
            w_cnt = 0;
        } else {
            // only the lenslet rows LP whose image row nx LP + r - hs lies
            // inside the image for some r of the tile give nonzero A records:
            // nx LP in [hs - rhi, R - 1 + hs - rlo]; their lenslets
            // [LP_lo Lc, (LP_hi + 1) Lc) are a contiguous run of stages
            const int d = g.hs - rhi, e = g.R - 1 + g.hs - rlo;
            const int lp_lo = d > 0 ? (d + g.nx - 1) / g.nx : 0;
            const int lp_hi = e < 0 ? -1 : min(g.Lr - 1, e / g.nx);
            if (lp_lo > lp_hi) {
                w_cnt = 0;
            } else {
                w_base = lp_lo * g.Lc / kStageK;
                w_cnt = (min(g.M, (lp_hi + 1) * g.Lc) + kStageK - 1) / kStageK - w_base;
            }
        }
    }
    const int s_begin = int(int64_t(w_cnt) * split / splits);
    const int s_end = int(int64_t(w_cnt) * (split + 1) / splits);
    const int li = lane & 31, lk = lane >> 5;
    f32x4 (*T)[4][64] = tot[wave];

    // Record r, half h of a block sits at 16-byte vector 2r + h of each of the
    // block's three vector planes; lane offsets are in bytes.
    const int64_t arows = kFwd ? int64_t(a.LRp) * a.LCp : a.Mpad;   // records per A block
    uint32_t oa[2], ob[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = m0 + 32 * i + li;
        if (kFwd) {
            const int mc = min(m, a.M - 1);   // rows past the last lenslet compute unused values
            const int Lp = int(fdiv(uint32_t(mc), g.fLc)), Lq = mc - Lp * g.Lc;
            oa[i] = uint32_t(16 * (2 * (Lp * a.LCp + Lq) + lk));
        } else {
            oa[i] = uint32_t(16 * (2 * m + lk));
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) ob[j] = uint32_t(16 * (2 * (nb + 32 * j + li) + lk));
    const char* A1 = reinterpret_cast<const char*>(a.A);
    const char* B1 = reinterpret_cast<const char*>(a.B);
    const uint32_t ablock = uint32_t(16 * kRecVec * arows), bblock = uint32_t(16 * kRecVec * a.Npad);

    // Forward window index i -> shifted patch row and column sr = s' + nx - 1,
    // tc = t' + ny - 1 and depth chunk zc (stage (sr * Kc + tc) * nzc + zc).
    struct FwdPos {
        int sr, tc, zc;
    };
    // the walk's divisors by this wavefront's row count
    const int n1 = kFwd ? a.walk.r0 * Rw * a.walk.q1 : 0;
    const FastDiv fRq1 = make_fastdiv(uint32_t(kFwd ? max(1, Rw * a.walk.q1) : 1));
    const FastDiv fRq0 = make_fastdiv(uint32_t(kFwd ? max(1, Rw * a.walk.q0) : 1));
    auto fwd_pos = [&](int i) -> FwdPos {
        const WindowWalk& w = a.walk;
        const int j = int(fdiv(uint32_t(i), a.fnzc)), zc = i - j * a.nzc;
        const bool first = j < n1;
        const int jr = first ? j : j - n1, q = first ? w.q1 : w.q0;
        const int bq = int(fdiv(uint32_t(jr), first ? fRq1 : fRq0));
        const int rem = jr - bq * Rw * q;
        const int ir = int(fdiv(uint32_t(rem), first ? w.fq1 : w.fq0)), k = rem - ir * q;
        const int ic = (first ? bq : w.r0 + bq) + k * g.ny;
        return FwdPos{sr0 + ir, tc0 + ic, zc};
    };
    // Forward A block of a window position: the phase plane px = (hs - s') mod
    // nx, py = (ht - t') mod ny and depth chunk zc, shifted by the lenslet
    // offset dP = floor((hs - s') / nx), dQ likewise.  hs - s' + nx ns =
    // hs + nx - 1 - sr + nx ns is never negative, so unsigned division finds
    // both (and dP = quotient - ns).
    auto a_rsrc_fwd = [&](const FwdPos& p) -> Rsrc {
        const uint32_t ep = uint32_t(g.hs + g.nx - 1 - p.sr + g.nx * g.ns);
        const uint32_t fq = uint32_t(g.ht + g.ny - 1 - p.tc + g.ny * g.nt);
        const int qp = int(fdiv(ep, g.fnx)), qq = int(fdiv(fq, g.fny));
        const int px = int(ep) - qp * g.nx, py = int(fq) - qq * g.ny;
        const int dP = qp - g.ns, dQ = qq - g.nt;
        const uint32_t shift = uint32_t(32 * ((dP + a.padP) * a.LCp + dQ + a.padQ));
        return make_rsrc(A1 + (int64_t(px * g.ny + py) * a.nzc + p.zc) * ablock + shift, ablock - shift);
    };

#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) T[t][q][lane] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    f32x16 acc[2][2] = {};
    // Three register sets rotate, so the loads of a stage are issued two
    // stages (~2 x 44 MFMAs per wave) before its MFMAs: enough to cover reads
    // that miss the L2.  Every load is issued unconditionally (the stage index
    // is clamped) so that the wait before a stage's MFMAs only covers that
    // stage's loads, never the prefetch behind it.
    const int s_last = max(s_begin, s_end - 1);
    // The buffer resources of stage s's records; computed one stage before
    // its loads are issued, among the MFMAs of the stage in flight.
    struct StageRsrc {
        Rsrc ra, rb;
    };
    auto rsrc_of = [&](int s) -> StageRsrc {
        const int i = min(s, s_last);
        if (kFwd) {
            const FwdPos p = fwd_pos(i);
            return StageRsrc{a_rsrc_fwd(p),
                             make_rsrc(B1 + int64_t((p.sr * g.Kc + p.tc) * a.nzc + p.zc) * bblock, bblock)};
        }
        return StageRsrc{make_rsrc(A1 + int64_t(w_base + i) * ablock, ablock),
                         make_rsrc(B1 + int64_t(w_base + i) * bblock, bblock)};
    };
    auto load = [&](const StageRsrc& r, Frag& f) {
        load_frag(r.ra, r.rb, oa, ob, uint32_t(32 * arows), uint32_t(32 * a.Npad), f);
        // keep the prefetch ahead of the MFMAs that follow (compiler barrier for
        // the optimiser, scheduling barrier for the back end)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
    };
    Frag f0, f1, f2;
    if (s_begin < s_end) {
        // Whole groups of three stages in a loop with one path through it (so
        // the wait analysis sees the same loads in flight on every entry),
        // then the zero to two stages left, whose loads the last group issued.
        StageRsrc nr = rsrc_of(s_begin);
        load(nr, f0);
        nr = rsrc_of(s_begin + 1);
        load(nr, f1);
        nr = rsrc_of(s_begin + 2);
        int s = s_begin;
        // (no branch inside a group: the scheduling regions between the loads
        // hold one stage's MFMAs and the next stage's address arithmetic)
        int groups = 0;
        for (const int s3 = s_begin + (s_end - s_begin) / 3 * 3; s < s3; s += 3) {
            load(nr, f2);
            nr = rsrc_of(s + 3);
            mma_stage(f0, acc);
            load(nr, f0);
            nr = rsrc_of(s + 4);
            mma_stage(f1, acc);
            load(nr, f1);
            nr = rsrc_of(s + 5);
            mma_stage(f2, acc);
            if (++groups == kFoldGroups) {
                fold(acc, T, lane);
                groups = 0;
            }
        }
        if (s < s_end) mma_stage(f0, acc);
        if (s + 1 < s_end) mma_stage(f1, acc);
    }
    fold(acc, T, lane);

    if (kFwd) {
        // the workgroup's partial-sum slot: the tile's 64 rows x Npad columns
        float* out = a.out + size_t(slot) * kMT * a.Npad;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 v = T[2 * i + j][q][lane];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = 32 * i + 8 * q + 4 * lk + e;
                        out[size_t(r) * a.Npad + nb + 32 * j + li] = v[e];
                    }
                }
    } else if (kMode == kModeGradH) {
        // row m = (r, r2) = (s + x, t + y), column n = (x, y, z): the entry of
        // dH[s][t][x][y][z] when s, t fall inside the patch
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = nb + 32 * j + li;
            if (n >= a.N) continue;
            const int c = int(fdiv(uint32_t(n), g.fnz)), z = n - c * g.nz;
            const int x = int(fdiv(uint32_t(c), g.fny)), y = c - x * g.ny;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 v = T[2 * i + j][q][lane];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = m0 + 32 * i + 8 * q + 4 * lk + e;
                        if (m >= a.M) continue;
                        const int r = int(fdiv(uint32_t(m), g.fKc)), r2 = m - r * g.Kc;
                        const int sp = r - x, tp = r2 - y;
                        if (unsigned(sp) < unsigned(g.ns) && unsigned(tp) < unsigned(g.nt))
                            a.out[((int64_t(sp) * g.nt + tp) * g.nx + x) * int64_t(g.ny * g.nz) + int64_t(y) * g.nz + z] =
                                v[e];
                    }
                }
        }
    } else {
        const size_t plane = size_t(g.R) * g.C;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = nb + 32 * j + li;
            if (n >= a.N) continue;
            const int c = int(fdiv(uint32_t(n), g.fnz)), z = n - c * g.nz;
            const int cx = int(fdiv(uint32_t(c), g.fny)), cy = c - cx * g.ny;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 v = T[2 * i + j][q][lane];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = m0 + 32 * i + 8 * q + 4 * lk + e;
                        if (m >= g.M) continue;
                        const int Lp = int(fdiv(uint32_t(m), g.fLc)), Lq = m - Lp * g.Lc;
                        const int P = g.nx * Lp + cx, Q = g.ny * Lq + cy;
                        if (P < g.R && Q < g.C) {
                            const size_t o = z * plane + size_t(P) * g.C + Q;
                            if (a.norm) {
                                const float nv = a.norm[o];
                                a.out[o] = nv > 0.0f ? a.gprev[o] * v[e] / nv : 0.0f;
                            } else {
                                a.out[o] = v[e];
                            }
                        }
                    }
                }
        }
    }
}

// ------------------------------------------------------------ operand packing

struct PackArgs {
    ProjGeom g;
    int N, Npad, Mpad;
    int stages;
    int nzc, LRp, LCp, padP, padQ;
    FastDiv fnzc, fLCp;
    ClassBoxes cb;    // forward column layout
};

// Item i of a block of `rows` records (i < 6 rows): vector plane v, record r,
// half h, in the block's storage order; slot0 = first slot of the 4 it holds.
struct RecItem {
    int r, slot0;
};

__device__ __forceinline__ RecItem rec_item(int i, int rows)
{
    const int v = i / (2 * rows), rem = i - v * 2 * rows;
    RecItem it;
    it.r = rem >> 1;
    it.slot0 = 12 * (rem & 1) + 4 * v;
    return it;
}

// Forward B records: record n of stage s holds, at the slot of depth z,
// H[s'+u][t'+v][(hs-s') mod nx][(ht-t') mod ny][z] for class n = (u,v) (0
// outside the patch).  A workgroup builds kNT records of one stage: it reads
// each record's run of H with six neighbouring lanes into LDS, record-major,
// then writes the block in its vector-major order, 1 KB per wavefront store.
__global__ void __launch_bounds__(256) k_pack_fwd_b(const float* H, PackArgs p, float* Bp)
{
    __shared__ f32x4 rec[kNT * kRecVec];
    const ProjGeom& g = p.g;
    const int s = int(blockIdx.x), n0 = int(blockIdx.y) * kNT;
    const FwdStage t = fwd_stage(g, p.fnzc, p.nzc, s);
    const int64_t cell = int64_t(g.nx) * g.ny * g.nz;
    const int64_t xy = (int64_t(t.px) * g.ny + t.py) * g.nz + int64_t(t.zc) * kStageK;
#pragma unroll
    for (int k = 0; k < kRecVec; ++k) {
        const int i = int(threadIdx.x) + k * kThreads;   // record i / 6, vector i % 6
        const int nl = i / kRecVec, c = i - nl * kRecVec, n = n0 + nl;
        int u = 0, v = 0;
        const bool valid = class_of_col(p.cb, g.nx, g.ny, n, u, v) && unsigned(t.sp + u) < unsigned(g.ns) &&
                           unsigned(t.tp + v) < unsigned(g.nt);
        const int64_t run = valid ? (int64_t(t.sp + u) * g.nt + (t.tp + v)) * cell + xy : 0;
        f32x4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kz = slot_k(4 * c + q);
            o[q] = (valid && kz >= 0 && t.zc * kStageK + kz < g.nz) ? H[run + kz] : 0.0f;
        }
        rec[i] = o;
    }
    __syncthreads();
    f32x4* out = reinterpret_cast<f32x4*>(Bp) + int64_t(s) * kRecVec * p.Npad;
#pragma unroll
    for (int k = 0; k < kRecVec; ++k) {
        const int j = int(threadIdx.x) + k * kThreads;   // vector plane j / 512, record, half
        const int vp = j / (2 * kNT), rem = j - vp * 2 * kNT, nl = rem >> 1, h = rem & 1;
        out[(int64_t(vp) * p.Npad + n0 + nl) * 2 + h] = rec[nl * kRecVec + 3 * h + vp];
    }
}

// g with depth innermost: gT[P][Q][z] = g[z][P][Q], through an LDS tile.
__global__ void __launch_bounds__(256) k_depth_last(const float* g, int nz, int plane, float* gT)
{
    __shared__ float tile[32][33];
    const int z0 = blockIdx.y * 32, p0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int z = z0 + r, pix = p0 + tx;
        tile[r][tx] = (z < nz && pix < plane) ? g[size_t(z) * plane + pix] : 0.0f;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int pix = p0 + r, z = z0 + tx;
        if (pix < plane && z < nz) gT[size_t(pix) * nz + z] = tile[tx][r];
    }
}

// Forward A records, g split by pixel phase with zero lenslets around it: the
// block of (px, py, depth chunk zc) holds record LP*LCp + LQ with slot values
// g[z][nx(LP-padP)+px][ny(LQ-padQ)+py] (0 outside the image).
__global__ void __launch_bounds__(256) k_pack_fwd_a(const float* gT, PackArgs p, float* gS)
{
    const ProjGeom& g = p.g;
    const int blk = int(blockIdx.x);   // (px, py, zc)
    const int rows = p.LRp * p.LCp;
    const int item = int(blockIdx.y) * 256 + int(threadIdx.x);
    if (item >= rows * kRecVec) return;
    const int pxy = int(fdiv(uint32_t(blk), p.fnzc)), zc = blk - pxy * p.nzc;
    const int px = int(fdiv(uint32_t(pxy), g.fny)), py = pxy - px * g.ny;
    const RecItem it = rec_item(item, rows);
    const int LP = int(fdiv(uint32_t(it.r), p.fLCp)), LQ = it.r - LP * p.LCp;
    const int P = g.nx * (LP - p.padP) + px, Q = g.ny * (LQ - p.padQ) + py;
    const bool valid = unsigned(P) < unsigned(g.R) && unsigned(Q) < unsigned(g.C);
    const int64_t run = valid ? (int64_t(P) * g.C + Q) * g.nz : 0;
    f32x4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = slot_k(it.slot0 + q);
        const int z = zc * kStageK + k;
        o[q] = (valid && k >= 0 && z < g.nz) ? gT[run + z] : 0.0f;
    }
    reinterpret_cast<f32x4*>(gS)[int64_t(blk) * kRecVec * rows + item] = o;
}

// Backward reduction index k (0..Kr*Kc-1) -> (r, r2).
__device__ __forceinline__ void bwd_pair(const ProjGeom& g, int k, int& r, int& r2)
{
    const int ri = int(fdiv(uint32_t(k), g.fKc));
    r = ri - (g.nx - 1);
    r2 = k - ri * g.Kc - (g.ny - 1);
}

// Backward B records: Bp[s][n][slot] = Ht[r+cx][r2+cy][(hs-r) mod nx][(ht-r2) mod ny][z]
// for column n = (cx,cy,z) and the pair (r,r2) of the slot (0 outside).
__global__ void __launch_bounds__(256) k_pack_bwd_b(const float* Ht, PackArgs p, float* Bp)
{
    const ProjGeom& g = p.g;
    const int s = int(blockIdx.x);
    const int item = int(blockIdx.y) * 256 + int(threadIdx.x);
    if (item >= p.Npad * kRecVec) return;
    const RecItem it = rec_item(item, p.Npad);
    const int n = it.r;
    const int cz = int(fdiv(uint32_t(n), g.fnz)), z = n - cz * g.nz;
    const int cx = int(fdiv(uint32_t(cz), g.fny)), cy = cz - cx * g.ny;
    const int64_t cell = int64_t(g.nx) * g.ny * g.nz;
    const int K = g.Kr * g.Kc;
    f32x4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int kk = slot_k(it.slot0 + q);
        const int k = s * kStageK + kk;
        int r = 0, r2 = 0;
        bwd_pair(g, k, r, r2);
        const bool valid = n < p.N && kk >= 0 && k < K && unsigned(r + cx) < unsigned(g.ns) &&
                           unsigned(r2 + cy) < unsigned(g.nt);
        const int x = imod(g.hs - r, g.nx), y = imod(g.ht - r2, g.ny);
        const int64_t idx = (int64_t(r + cx) * g.nt + (r2 + cy)) * cell + (int64_t(x) * g.ny + y) * g.nz + z;
        o[q] = valid ? Ht[idx] : 0.0f;
    }
    reinterpret_cast<f32x4*>(Bp)[int64_t(s) * kRecVec * p.Npad + item] = o;
}

// Backward A records: Ap[s][m][slot] = f[nx*LP + hs - r][ny*LQ + ht - r2] for
// lenslet m = (LP,LQ) and the pair (r,r2) of the slot (0 outside the image).
__global__ void __launch_bounds__(256) k_pack_bwd_a(const float* f, PackArgs p, float* Ap)
{
    const ProjGeom& g = p.g;
    const int s = int(blockIdx.x);
    const int item = int(blockIdx.y) * 256 + int(threadIdx.x);
    if (item >= p.Mpad * kRecVec) return;
    const RecItem it = rec_item(item, p.Mpad);
    const int m = it.r;
    const int LP = int(fdiv(uint32_t(m), g.fLc)), LQ = m - LP * g.Lc;
    const int K = g.Kr * g.Kc;
    f32x4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int kk = slot_k(it.slot0 + q);
        const int k = s * kStageK + kk;
        int r = 0, r2 = 0;
        bwd_pair(g, k, r, r2);
        const int P = g.nx * LP + g.hs - r, Q = g.ny * LQ + g.ht - r2;
        const bool valid = m < g.M && kk >= 0 && k < K && unsigned(P) < unsigned(g.R) && unsigned(Q) < unsigned(g.C);
        o[q] = valid ? f[valid ? int64_t(P) * g.C + Q : 0] : 0.0f;
    }
    reinterpret_cast<f32x4*>(Ap)[int64_t(s) * kRecVec * p.Mpad + item] = o;
}

// Gradient with respect to H.  With P = nx*LP + x, Q = ny*LQ + y and r = s + x,
// r2 = t + y:  dH[s][t][x][y][z] = E[(r,r2)][(x,y,z)],
//   E[(r,r2)][(x,y,z)] = sum over lenslets (LP,LQ) of
//       w[nx*LP + r - hs][ny*LQ + r2 - ht] * g[z][nx*LP + x][ny*LQ + y],
// a GEMM over the lenslets (22 per stage).  A records: row (r,r2), the image
// gradient w at the stage's lenslets (0 outside the image); B records: column
// (x,y,z), the volume g at the stage's lenslets.
__global__ void __launch_bounds__(256) k_pack_gh_a(const float* w, PackArgs p, float* Ap)
{
    const ProjGeom& g = p.g;
    const int s = int(blockIdx.x);
    const int item = int(blockIdx.y) * 256 + int(threadIdx.x);
    if (item >= p.Mpad * kRecVec) return;
    const RecItem it = rec_item(item, p.Mpad);
    const int m = it.r;
    const int r = int(fdiv(uint32_t(m), g.fKc)), r2 = m - r * g.Kc;
    const bool row = m < g.Kr * g.Kc;
    f32x4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int kk = slot_k(it.slot0 + q);
        const int k = s * kStageK + kk;   // lenslet
        const int LP = int(fdiv(uint32_t(k), g.fLc)), LQ = k - LP * g.Lc;
        const int pp = g.nx * LP + r - g.hs, qq = g.ny * LQ + r2 - g.ht;
        const bool valid = row && kk >= 0 && k < g.M && unsigned(pp) < unsigned(g.R) && unsigned(qq) < unsigned(g.C);
        o[q] = valid ? w[int64_t(pp) * g.C + qq] : 0.0f;
    }
    reinterpret_cast<f32x4*>(Ap)[int64_t(s) * kRecVec * p.Mpad + item] = o;
}

__global__ void __launch_bounds__(256) k_pack_gh_b(const float* gv, PackArgs p, float* Bp)
{
    const ProjGeom& g = p.g;
    const int s = int(blockIdx.x);
    const int item = int(blockIdx.y) * 256 + int(threadIdx.x);
    if (item >= p.Npad * kRecVec) return;
    const RecItem it = rec_item(item, p.Npad);
    const int n = it.r;
    const int c = int(fdiv(uint32_t(n), g.fnz)), z = n - c * g.nz;
    const int x = int(fdiv(uint32_t(c), g.fny)), y = c - x * g.ny;
    const int64_t plane = int64_t(g.R) * g.C;
    f32x4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int kk = slot_k(it.slot0 + q);
        const int k = s * kStageK + kk;
        const int LP = int(fdiv(uint32_t(k), g.fLc)), LQ = k - LP * g.Lc;
        const int P = g.nx * LP + x, Q = g.ny * LQ + y;
        const bool valid = n < p.N && kk >= 0 && k < g.M && P < g.R && Q < g.C;
        o[q] = valid ? gv[z * plane + int64_t(P) * g.C + Q] : 0.0f;
    }
    reinterpret_cast<f32x4*>(Bp)[int64_t(s) * kRecVec * p.Npad + item] = o;
}

// f[p][q] = sum over splits of the partial tile entry of (lenslet, class).
// With fmeas set (Richardson-Lucy, Eq. 2), the quotient fmeas / f is written
// instead, 0 where f is not positive.
__global__ void __launch_bounds__(256) k_fwd_reduce(const float* partial, const uint32_t* tab, int Npad,
                                                     ProjGeom g, ClassBoxes cb, const float* fmeas, float* f)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(g.R) * g.C) return;
    const int p = int(i / g.C), q = int(i - int64_t(p) * g.C);
    const int m = (p / g.nx) * g.Lc + q / g.ny;
    const int n = col_of_class(cb, p % g.nx, q % g.ny);
    // the row tile's partial-sum slots, in split order
    const int mt = m / kMT, r = m - mt * kMT;
    const uint32_t first = tab[mt], last = tab[mt + 1];
    double acc = 0.0;
    for (uint32_t s = first; s < last; ++s) acc += double(partial[(size_t(s) * kMT + r) * Npad + n]);
    if (fmeas)
        f[i] = acc > 0.0 ? float(double(fmeas[i]) / acc) : 0.0f;
    else
        f[i] = float(acc);
}

// ---------------------------------------------------------------- host side

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct FwdPlan {
    ProjGeom g;
    FwdLayout L;
    int N, Npad, Mpad, mtiles, ntiles;
    int splits;                  // of a row tile that needs every window row
    int slots, nwg;              // partial-sum slots (64 rows each), workgroups
    std::vector<uint32_t> tab;   // the work table (GemmArgs::tab)
    ClassBoxes cb;
    size_t gT_bytes, gS_bytes, B_bytes, part_bytes, tab_bytes;
};

// Box shape of the forward columns: at most 64 classes a box, the shape that
// minimises the wavefronts' stages, (boxes rounded up to whole workgroups) x
// (ns + bu - 1)(nt + bv - 1), with at most 2 x classes + 256 columns
// (bu = min(nx, 64) always qualifies); ties go to the squarer box.
ClassBoxes class_boxes(const ProjGeom& g)
{
    ClassBoxes best{};
    int64_t best_cost = -1;
    const int64_t classes = int64_t(g.nx) * g.ny;
    for (int bu = 1; bu <= std::min(g.nx, 64); ++bu) {
        const int bv = std::min(g.ny, 64 / bu);
        const int nbu = (g.nx + bu - 1) / bu, nbv = (g.ny + bv - 1) / bv;
        const int64_t waves = (int64_t(nbu) * nbv + kNT / 64 - 1) / (kNT / 64) * (kNT / 64);
        if (waves * 64 > 2 * classes + 256 && bu != std::min(g.nx, 64)) continue;
        const int64_t cost = waves * (g.ns + bu - 1) * (g.nt + bv - 1);
        if (best_cost < 0 || cost < best_cost ||
            (cost == best_cost && std::abs(bu - bv) < std::abs(best.bu - best.bv))) {
            best_cost = cost;
            best = ClassBoxes{bu, bv, nbv, nbu * nbv};
        }
    }
    return best;
}

FwdPlan fwd_plan(const lfbp_shape& s, int64_t R, int64_t C)
{
    FwdPlan P;
    P.g = make_geom(s, R, C);
    P.L = fwd_layout(P.g);
    P.N = P.g.nx * P.g.ny;
    P.cb = class_boxes(P.g);
    P.mtiles = (P.g.M + kMT - 1) / kMT;
    P.ntiles = (P.cb.boxes * 64 + kNT - 1) / kNT;
    P.Mpad = P.mtiles * kMT;
    P.Npad = P.ntiles * kNT;
    // Splits.  Row tiles near the top and bottom of the image need fewer
    // window rows (fwd_tile_rows), so each row tile gets splits in proportion
    // to the rows its busiest box needs and every workgroup has about the
    // same work: count(c, mt) = ceil(rows(mt) c / rows_max), with the largest
    // c (at most 64, and at most one per 64 stages) whose workgroups fit one
    // round of kTargetBlocks (two per CU on 256 CUs).  The counts depend on
    // the shape only, so the workspace size and the order of the float64
    // reduction do not depend on the device.
    std::vector<int> rows(size_t(P.mtiles), 0);
    int rows_max = 0;
    for (int mt = 0; mt < P.mtiles; ++mt) {
        for (int b = 0; b < P.cb.boxes; ++b) {
            int lo;
            rows[size_t(mt)] = std::max(rows[size_t(mt)], fwd_tile_rows(P.g, P.cb, mt, b, lo));
        }
        rows_max = std::max(rows_max, rows[size_t(mt)]);
    }
    auto count = [&](int c, int mt) {
        return rows_max == 0 ? 1 : std::max(1, int((int64_t(rows[size_t(mt)]) * c + rows_max - 1) / rows_max));
    };
    const int cap = std::max(1, std::min(64, P.L.stages / 64));
    P.splits = 1;
    for (int c = 2; c <= cap; ++c) {
        int64_t total = 0;
        for (int mt = 0; mt < P.mtiles; ++mt) total += count(c, mt);
        if (total * P.ntiles > kTargetBlocks) break;
        P.splits = c;
    }
    // the work table: first slot of every row tile, then the workgroups in
    // the order (split, column tile, row tile), so that the row tiles of one
    // split and column tile, which walk the same stages, run on one XCD
    P.tab.assign(size_t(P.mtiles) + 1, 0u);
    for (int mt = 0; mt < P.mtiles; ++mt) P.tab[size_t(mt) + 1] = P.tab[size_t(mt)] + uint32_t(count(P.splits, mt));
    P.slots = int(P.tab[size_t(P.mtiles)]);
    for (int j = 0; j < P.splits; ++j)
        for (int nt = 0; nt < P.ntiles; ++nt)
            for (int mt = 0; mt < P.mtiles; ++mt)
                if (j < count(P.splits, mt)) P.tab.push_back((uint32_t(mt * P.ntiles + nt) << 6) | uint32_t(j));
    P.nwg = int(P.tab.size()) - (P.mtiles + 1);
    P.gT_bytes = align256(size_t(P.g.nz) * P.g.R * P.g.C * sizeof(float));
    P.gS_bytes = align256(size_t(P.N) * P.L.LRp * P.L.LCp * P.L.nzc * kRec * sizeof(float));
    P.B_bytes = align256(size_t(P.L.stages) * P.Npad * kRec * sizeof(float));
    P.tab_bytes = align256(P.tab.size() * sizeof(uint32_t));
    P.part_bytes = align256(size_t(P.slots) * kMT * P.Npad * sizeof(float)) + P.tab_bytes;   // partials, table
    return P;
}

struct BwdPlan {
    ProjGeom g;
    int N, Npad, Mpad, mtiles, ntiles, stages;
    size_t A_bytes, B_bytes;
};

BwdPlan bwd_plan(const lfbp_shape& s, int64_t R, int64_t C)
{
    BwdPlan P;
    P.g = make_geom(s, R, C);
    P.N = P.g.nx * P.g.ny * P.g.nz;
    P.mtiles = (P.g.M + kMT - 1) / kMT;
    P.ntiles = (P.N + kNT - 1) / kNT;
    P.Mpad = P.mtiles * kMT;
    P.Npad = P.ntiles * kNT;
    P.stages = (P.g.Kr * P.g.Kc + kStageK - 1) / kStageK;
    P.A_bytes = align256(size_t(P.stages) * P.Mpad * kRec * sizeof(float));
    P.B_bytes = align256(size_t(P.stages) * P.Npad * kRec * sizeof(float));
    return P;
}

PackArgs pack_args(const ProjGeom& g, int N, int Npad, int Mpad, int stages)
{
    PackArgs p{};
    p.g = g;
    p.N = N;
    p.Npad = Npad;
    p.Mpad = Mpad;
    p.stages = stages;
    p.nzc = 1;
    p.LRp = 1;
    p.LCp = 1;
    p.fnzc = make_fastdiv(1);
    p.fLCp = make_fastdiv(1);
    return p;
}

unsigned blocks_for(int64_t items) { return unsigned((items + 255) / 256); }

WindowWalk window_walk(const ProjGeom& g, const ClassBoxes& cb)
{
    const int Cw = g.nt + cb.bv - 1;
    WindowWalk w;
    w.q0 = Cw / g.ny;
    w.r0 = Cw - w.q0 * g.ny;
    w.q1 = w.q0 + 1;
    w.fq1 = make_fastdiv(uint32_t(w.q1));
    w.fq0 = make_fastdiv(uint32_t(std::max(1, w.q0)));
    return w;
}


// ------------------------------------------- forward with 16-column class boxes
//
// The forward GEMM above tiles the nx * ny classes in 64-column boxes of
// 32 x 32 x 2 matrix-core steps, so 225 classes take 256 columns, and each
// box walks the window of its 8 x 8 classes.  This form takes boxes of 3 x 5
// classes in 16 columns (v_mfma_f32_16x16x4_f32): a wavefront holds up to five
// boxes stacked along u in one strip of five class columns (64 lenslet rows x
// 80 columns), and the four reduction indices of a step are four column
// shifts t', t' + ny, t' + 2 ny, t' + 3 ny of one residue (one per group of 16
// lanes), so a stage is four window positions at seven depths.  A box runs
// only the row shifts it needs: the shared A records feed every box whose
// window holds the stage's rows.  The partial sums of each split go to their
// own slot; a second kernel adds the slots in split order in float64.
//
// Records (8 floats, the last 0): A16[px][py][chunk][LP'][LQ'] holds depths
// 7 chunk .. 7 chunk + 6 of g at pixel (nx (LP' - padP) + px, ny (LQ' - padQ) +
// py), 0 outside the image; B16[s' + nx - 1][t' + ny - 1][chunk][strip][box][n]
// holds those depths of H[s' + u][t' + v][(hs - s') mod nx][(ht - t') mod ny]
// for class (u, v) = (3 box + n / 5, 5 strip + n mod 5), 0 outside the patch,
// for n = 15 and for classes past the cell.
constexpr int kBU = 3, kBV = 5, kWaveBoxes = 5, kCh = 7, kF16Fold = 48;
constexpr uint32_t kOob = 0x7FFFFFF0u;   // a byte offset past every record block: reads zeros

struct Fwd16Item {      // one wavefront: row tile, strip, box group, the window rows it needs, stages, slot
    int mt, j, h, r_lo, nrows, st_begin, st_end, slot;
};

struct Fwd16Args {
    const float* A;
    const float* B;
    float* out;                 // partial tiles [slot][64][ncols]
    const Fwd16Item* items;
    uint32_t A_bytes, B_bytes;
    int nitems, nwg;
    int ns, nt, nx, ny, M, Lc, LCp, Kt;
    int hsb, htb;          // hs + nx padP, ht + ny padQ: the biased shifts floor(/ nx) and floor(/ ny) take
    int PL;                // records of one (px, py) block: nch * LRp * LCp
    int nch, nbx, nbox, ncols;   // depth chunks, B records per (position, chunk): nstrips * nbox * 16
    uint32_t mnx, mny;     // division magics of nx and ny (mdiv)
};

__device__ __forceinline__ f32x3 ld3(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(f32x3, __builtin_amdgcn_raw_buffer_load_b96(r, int(voff), int(soff), 0));
}

__device__ __forceinline__ float rec_at(const f32x4& x, const f32x3& y, int d) { return d < 4 ? x[d] : y[d - 4]; }

// n / d for n < 2^32 / d, with m = ceil(2^32 / d) (one multiply-high), or n
// itself for d = 1 (m = 0).
__host__ __device__ inline uint32_t div_magic(uint32_t d)
{
    return d <= 1 ? 0u : uint32_t(((uint64_t(1) << 32) + d - 1) / d);
}

__device__ __forceinline__ uint32_t mdiv(uint32_t n, uint32_t m) { return m ? __umulhi(n, m) : n; }

struct Fwd16Walk {      // wavefront-uniform: residue, group of four positions, depth chunk
    int rho, g, c, ncols, groups, tfirst, P;
    uint32_t mcols;
};

__device__ __forceinline__ void f16_residue(Fwd16Walk& w, int rho, int nrows, int ny, int c_lo, int c_hi)
{
    w.rho = rho;
    w.tfirst = c_lo + imod(rho - c_lo, ny);
    w.ncols = w.tfirst <= c_hi ? (c_hi - w.tfirst) / ny + 1 : 0;
    w.P = nrows * w.ncols;
    w.groups = (w.P + 3) / 4;
    w.mcols = div_magic(uint32_t(max(1, w.ncols)));
}

struct Fwd16Set {
    f32x4 a0[4];
    f32x3 a1[4];
    f32x4 b0[kWaveBoxes];
    f32x3 b1[kWaveBoxes];
    int mask;
};

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) k_fwd16(Fwd16Args a)
{
    __shared__ float tot[kThreads / 64][4 * kWaveBoxes * 4][64];   // per wave: 80 sums x 64 lanes
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = int(threadIdx.x) & 63;
    // logical workgroup (consecutive ones on one XCD) -> its four items
    const int b = int(blockIdx.x), x = b % kXcds, qq = a.nwg / kXcds, rr = a.nwg % kXcds;
    const int it = (x * qq + min(x, rr) + b / kXcds) * 4 + wave;
    if (it >= a.nitems) return;
    const Fwd16Item I = a.items[it];
    const int mt = __builtin_amdgcn_readfirstlane(I.mt), j = __builtin_amdgcn_readfirstlane(I.j);
    const int h = __builtin_amdgcn_readfirstlane(I.h), r_lo = __builtin_amdgcn_readfirstlane(I.r_lo);
    const int nrows = __builtin_amdgcn_readfirstlane(I.nrows);
    const int st0 = __builtin_amdgcn_readfirstlane(I.st_begin), st1 = __builtin_amdgcn_readfirstlane(I.st_end);
    const int slot = __builtin_amdgcn_readfirstlane(I.slot);
    const int q = lane >> 4, n = lane & 15;
    const Rsrc ra = make_rsrc(reinterpret_cast<const char*>(a.A), a.A_bytes);
    const Rsrc rb = make_rsrc(reinterpret_cast<const char*>(a.B), a.B_bytes);
    int lb[4];   // this lane's lenslet (row 16 k + n of the tile) in the padded grid, -1 past M
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int m = kMT * mt + 16 * k + n;
        const int Lp = m / a.Lc, Lq = m - Lp * a.Lc;
        lb[k] = m < a.M ? Lp * a.LCp + Lq : -1;
    }
    const int c_lo = -min(a.ny - 1, kBV * j + kBV - 1), c_hi = a.nt - 1 - kBV * j;
    Fwd16Walk w;
    {   // the first stage: skip whole residues, then groups and chunks
        int rem = st0, rho = 0;
        f16_residue(w, 0, nrows, a.ny, c_lo, c_hi);
        while (rho < a.ny && rem >= a.nch * w.groups) {
            rem -= a.nch * w.groups;
            if (++rho < a.ny) f16_residue(w, rho, nrows, a.ny, c_lo, c_hi);
        }
        w.g = rem / a.nch;
        w.c = rem - w.g * a.nch;
    }
    for (int e = 0; e < 4 * kWaveBoxes * 4; ++e) tot[wave][e][lane] = 0.f;
    f32x4 acc[4][kWaveBoxes];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < kWaveBoxes; ++i) acc[k][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    // this lane's position in the residue's row-major sequence, and the record
    // offsets of the current group of four positions (chunk 0)
    const uint32_t CA = uint32_t(a.PL / a.nch) * 32u;
    const uint32_t CB = uint32_t(a.nbx) * 32u;
    int pos = 0, ri = 0, ci = 0, gmask = 0;
    uint32_t gA[4], gB = kOob;
    auto start_residue = [&]() {
        pos = 4 * w.g + q;
        ri = int(mdiv(uint32_t(pos), w.mcols));
        ci = pos - ri * w.ncols;
    };
    auto group_offsets = [&]() {
        const bool ok = pos < w.P;
        const int sp = r_lo + ri, tp = w.tfirst + a.ny * ci;
        const uint32_t es = uint32_t(a.hsb - sp), et = uint32_t(a.htb - tp);
        const int qs = int(mdiv(es, a.mnx)), qt = int(mdiv(et, a.mny));
        const int px = int(es) - qs * a.nx, py = int(et) - qt * a.ny;
        const int plane = (px * a.ny + py) * a.PL + qs * a.LCp + qt;
#pragma unroll
        for (int k = 0; k < 4; ++k) gA[k] = (ok && lb[k] >= 0) ? uint32_t(plane + lb[k]) * 32u : kOob;
        const int pidx = (sp + a.nx - 1) * a.Kt + (tp + a.ny - 1);
        gB = ok ? uint32_t((pidx * a.nch * a.nbx + (j * a.nbox + kWaveBoxes * h) * 16 + n)) * 32u : kOob;
        int mask = 0;
        if (w.P > 0) {
            const int p3 = min(4 * w.g + 3, w.P - 1);
            const int smin = r_lo + int(mdiv(uint32_t(4 * w.g), w.mcols));
            const int smax = r_lo + int(mdiv(uint32_t(p3), w.mcols));
#pragma unroll
            for (int i = 0; i < kWaveBoxes; ++i) {
                const int bi = kWaveBoxes * h + i;
                if (bi < a.nbox && smin <= a.ns - 1 - kBU * bi && smax >= -min(a.nx - 1, kBU * bi + kBU - 1))
                    mask |= 1 << i;
            }
        }
        gmask = __builtin_amdgcn_readfirstlane(mask);
    };
    start_residue();
    group_offsets();
    auto fill = [&](Fwd16Set& S, bool live) {
        const uint32_t sa = uint32_t(w.c) * CA, sb = uint32_t(w.c) * CB;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t off = live ? gA[k] : kOob;
            S.a0[k] = load_vec(ra, off, sa);
            S.a1[k] = ld3(ra, off + 16u, sa);
        }
        const uint32_t ob = live ? gB : kOob;
#pragma unroll
        for (int i = 0; i < kWaveBoxes; ++i) {
            S.b0[i] = load_vec(rb, ob + 512u * i, sb);
            S.b1[i] = ld3(rb, ob + 512u * i + 16u, sb);
        }
        S.mask = live ? gmask : 0;
        if (++w.c == a.nch) {   // next group of positions
            w.c = 0;
            if (++w.g >= w.groups) {
                w.g = 0;
                int rho = w.rho + 1;
                while (rho < a.ny) {
                    f16_residue(w, rho, nrows, a.ny, c_lo, c_hi);
                    if (w.groups > 0) break;
                    ++rho;
                }
                if (rho >= a.ny) w.rho = a.ny;
                start_residue();
            } else {
                pos += 4;
                ci += 4;
                while (ci >= w.ncols) {
                    ci -= w.ncols;
                    ++ri;
                }
            }
            group_offsets();
        }
    };
    auto mma = [&](const Fwd16Set& S) {
#pragma unroll
        for (int i = 0; i < kWaveBoxes; ++i) {
            if (S.mask & (1 << i)) {
#pragma unroll
                for (int d = 0; d < kCh; ++d)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        acc[k][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(rec_at(S.a0[k], S.a1[k], d),
                                                                         rec_at(S.b0[i], S.b1[i], d), acc[k][i], 0, 0, 0);
            }
        }
    };
    auto fold = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int i = 0; i < kWaveBoxes; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    tot[wave][(k * kWaveBoxes + i) * 4 + r][lane] += acc[k][i][r];
                    acc[k][i][r] = 0.f;
                }
    };
    // two register sets: the next stage's records load while the matrix
    // cores take the current one (an odd count ends with a dead stage: zero
    // records, no steps)
    Fwd16Set s0, s1;
    fill(s0, st0 < st1);
    int since = 0;
    for (int st = st0; st < st1; st += 2) {
        fill(s1, st + 1 < st1);
        __builtin_amdgcn_sched_barrier(0);
        mma(s0);
        __builtin_amdgcn_sched_barrier(0);
        fill(s0, st + 2 < st1);
        __builtin_amdgcn_sched_barrier(0);
        mma(s1);
        __builtin_amdgcn_sched_barrier(0);
        if ((since += 2) >= kF16Fold) {
            fold();
            since = 0;
        }
    }
    fold();
    float* o = a.out + size_t(slot) * kMT * a.ncols;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < kWaveBoxes; ++i) {
            const int bi = kWaveBoxes * h + i;
            if (bi < a.nbox) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    o[(16 * k + 4 * q + r) * a.ncols + (j * a.nbox + bi) * 16 + n] = tot[wave][(k * kWaveBoxes + i) * 4 + r][lane];
            }
        }
}

struct Fwd16Pack {
    ProjGeom g;
    int nch, nstrips, nbox, padP, padQ, LRp, LCp, Kt;
    FastDiv f16, f5;
};

// A16 records from g with depth innermost (gT[P][Q][z]): one record per thread.
__global__ void __launch_bounds__(256) k_pack16_a(const float* gT, Fwd16Pack p, float* A16, int64_t nrec)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= nrec) return;
    const ProjGeom& g = p.g;
    const int64_t cell = int64_t(p.LRp) * p.LCp;
    const int64_t pl = i / cell;
    const int rest = int(i - pl * cell);
    const int LP = rest / p.LCp, LQ = rest - LP * p.LCp;
    const int c = int(pl % p.nch), pxy = int(pl / p.nch);
    const int px = pxy / g.ny, py = pxy - px * g.ny;
    const int P = g.nx * (LP - p.padP) + px, Q = g.ny * (LQ - p.padQ) + py;
    const bool ok = unsigned(P) < unsigned(g.R) && unsigned(Q) < unsigned(g.C);
    const float* src = gT + (ok ? (int64_t(P) * g.C + Q) * g.nz : 0);
    float v[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) v[d] = (ok && d < kCh && kCh * c + d < g.nz) ? src[kCh * c + d] : 0.f;
    f32x4* dst = reinterpret_cast<f32x4*>(A16) + 2 * i;
    dst[0] = f32x4{v[0], v[1], v[2], v[3]};
    dst[1] = f32x4{v[4], v[5], v[6], v[7]};
}

// B16 records from H: one record per thread.
__global__ void __launch_bounds__(256) k_pack16_b(const float* H, Fwd16Pack p, float* B16, int64_t nrec)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= nrec) return;
    const ProjGeom& g = p.g;
    const int n = int(i & 15);
    int64_t r = i >> 4;
    const int bi = int(r % p.nbox);
    r /= p.nbox;
    const int j = int(r % p.nstrips);
    r /= p.nstrips;
    const int c = int(r % p.nch);
    const int64_t pidx = r / p.nch;
    const int sr = int(pidx / p.Kt), tc = int(pidx - int64_t(sr) * p.Kt);
    const int sp = sr - (g.nx - 1), tp = tc - (g.ny - 1);
    const int u = kBU * bi + n / kBV, v = kBV * j + n % kBV;
    const bool ok = n < kBU * kBV && u < g.nx && v < g.ny && unsigned(sp + u) < unsigned(g.ns) &&
                    unsigned(tp + v) < unsigned(g.nt);
    const int x = imod(g.hs - sp, g.nx), y = imod(g.ht - tp, g.ny);
    const float* src = H + (ok ? ((((int64_t(sp + u) * g.nt + (tp + v)) * g.nx + x) * g.ny + y) * g.nz) : 0);
    float vals[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) vals[d] = (ok && d < kCh && kCh * c + d < g.nz) ? src[kCh * c + d] : 0.f;
    f32x4* dst = reinterpret_cast<f32x4*>(B16) + 2 * i;
    dst[0] = f32x4{vals[0], vals[1], vals[2], vals[3]};
    dst[1] = f32x4{vals[4], vals[5], vals[6], vals[7]};
}

// f[p][q] = sum over the row tile's slots (in split order, float64) of the
// partial entry of (lenslet, class); with fmeas set (Richardson-Lucy, Eq. 2),
// the quotient fmeas / f instead, 0 where f is not positive.  One thread per
// partial entry (row tile, row, column), so that the reads of a slot coalesce.
__global__ void __launch_bounds__(256) k_fwd16_reduce(const float* partial, const uint32_t* tab, int ncols, int nbox,
                                                       ProjGeom g, const float* fmeas, float* f)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = int64_t(kMT) * ncols;
    const int mt = int(i / per);
    const int rest = int(i - int64_t(mt) * per), r = rest / ncols, col = rest - r * ncols;
    const int m = kMT * mt + r;
    if (m >= g.M) return;
    const int n = col & 15, box = col >> 4, j = box / nbox, bi = box - j * nbox;
    const int u = kBU * bi + n / kBV, v = kBV * j + n % kBV;
    if (n >= kBU * kBV || u >= g.nx || v >= g.ny) return;
    const int Lp = m / g.Lc, Lq = m - Lp * g.Lc;
    const int p = g.nx * Lp + u, q = g.ny * Lq + v;
    if (p >= g.R || q >= g.C) return;
    double acc = 0.0;
    for (uint32_t s = tab[mt]; s < tab[mt + 1]; ++s) acc += double(partial[(size_t(s) * kMT + r) * ncols + col]);
    const int64_t o = int64_t(p) * g.C + q;
    if (fmeas)
        f[o] = acc > 0.0 ? float(double(fmeas[o]) / acc) : 0.0f;
    else
        f[o] = float(acc);
}

// Plan of the 16-column forward: record and partial-sum geometry, the
// wavefront items and the slot table, from the shapes only (so the workspace
// and the order of the float64 sums do not depend on the device).
struct Fwd16Plan {
    ProjGeom g;
    bool ok;                        // record blocks within 32-bit byte offsets
    int nch, nstrips, nbox, ngroups, padP, padQ, LRp, LCp, Kt, ncols, mtiles, slots, nitems, nwg;
    std::vector<Fwd16Item> items;   // wavefront items, in launch order
    std::vector<uint32_t> tab;      // first slot of every row tile (mtiles + 1 entries)
    size_t gT_bytes, A_bytes, B_bytes, part_bytes, items_bytes, tab_bytes;
};

Fwd16Plan fwd16_plan(const lfbp_shape& s, int64_t R, int64_t C)
{
    Fwd16Plan P;
    const ProjGeom g = make_geom(s, R, C);
    P.g = g;
    P.nch = (g.nz + kCh - 1) / kCh;
    P.nstrips = (g.ny + kBV - 1) / kBV;
    P.nbox = (g.nx + kBU - 1) / kBU;
    P.ngroups = (P.nbox + kWaveBoxes - 1) / kWaveBoxes;
    P.padP = (g.ns - 1 - g.hs + g.nx - 1) / g.nx;   // lenslet offsets floor((hs - s') / nx) >= -padP
    P.padQ = (g.nt - 1 - g.ht + g.ny - 1) / g.ny;
    P.LRp = g.Lr + P.padP + (g.hs + g.nx - 1) / g.nx;
    P.LCp = g.Lc + P.padQ + (g.ht + g.ny - 1) / g.ny;
    P.Kt = g.nt + g.ny - 1;
    P.ncols = P.nstrips * P.nbox * 16;
    P.mtiles = (g.M + kMT - 1) / kMT;
    const uint64_t A_raw = uint64_t(g.nx) * g.ny * P.nch * uint64_t(P.LRp) * P.LCp * 32u;
    const uint64_t B_raw = uint64_t(g.Kr) * P.Kt * P.nch * uint64_t(P.nstrips) * P.nbox * 16u * 32u;
    P.ok = A_raw <= 0x7FFF0000u && B_raw <= 0x7FFF0000u;
    P.gT_bytes = align256(size_t(g.nz) * g.R * g.C * sizeof(float));
    P.A_bytes = align256(size_t(A_raw));
    P.B_bytes = align256(size_t(B_raw));
    // window rows of every (row tile, box group): the group's patch-row
    // shifts less those whose A records are zero for the whole tile
    std::vector<int> rlo(size_t(P.mtiles) * P.ngroups), nrow(size_t(P.mtiles) * P.ngroups), rows(size_t(P.mtiles), 0);
    int rows_max = 0;
    for (int mt = 0; mt < P.mtiles; ++mt) {
        const int lp_lo = (kMT * mt) / g.Lc, lp_hi = std::min(g.M - 1, kMT * mt + kMT - 1) / g.Lc;
        for (int h = 0; h < P.ngroups; ++h) {
            const int lo = std::max(-std::min(g.nx - 1, kBU * kWaveBoxes * h + kBU * kWaveBoxes - 1),
                                    g.nx * lp_lo + g.hs - (g.R - 1));
            const int hi = std::min(g.ns - 1 - kBU * kWaveBoxes * h, g.nx * lp_hi + g.hs);
            rlo[size_t(mt) * P.ngroups + h] = lo;
            nrow[size_t(mt) * P.ngroups + h] = std::max(0, hi - lo + 1);
            rows[size_t(mt)] = std::max(rows[size_t(mt)], std::max(0, hi - lo + 1));
        }
        rows_max = std::max(rows_max, rows[size_t(mt)]);
    }
    auto stages = [&](int mt, int j, int h) {   // the walk of one item: residues, groups of four, chunks
        const int nr = nrow[size_t(mt) * P.ngroups + h];
        const int c_lo = -std::min(g.ny - 1, kBV * j + kBV - 1), c_hi = g.nt - 1 - kBV * j;
        int64_t T = 0;
        for (int rho = 0; rho < g.ny; ++rho) {
            const int tfirst = c_lo + ((rho - c_lo) % g.ny + g.ny) % g.ny;
            const int ncols = tfirst <= c_hi ? (c_hi - tfirst) / g.ny + 1 : 0;
            T += int64_t(P.nch) * ((int64_t(nr) * ncols + 3) / 4);
        }
        return T;
    };
    int64_t Tmax = 0;
    for (int mt = 0; mt < P.mtiles; ++mt)
        for (int h = 0; h < P.ngroups; ++h) Tmax = std::max(Tmax, stages(mt, 0, h));
    auto count = [&](int c, int mt) {
        return rows_max == 0 ? 1 : std::max(1, int((int64_t(rows[size_t(mt)]) * c + rows_max - 1) / rows_max));
    };
    // splits: the most (at most 64, at most one per 64 stages) whose
    // wavefronts fill one round of kTargetBlocks workgroups
    const int per = P.nstrips * P.ngroups;
    const int cap = int(std::max<int64_t>(1, std::min<int64_t>(64, Tmax / 64)));
    int S = 1;
    for (int c = 2; c <= cap; ++c) {
        int64_t waves = 0;
        for (int mt = 0; mt < P.mtiles; ++mt) waves += int64_t(count(c, mt)) * per;
        if ((waves + 3) / 4 > kTargetBlocks) break;
        S = c;
    }
    P.tab.assign(size_t(P.mtiles) + 1, 0u);
    int cmax = 0;
    for (int mt = 0; mt < P.mtiles; ++mt) {
        P.tab[size_t(mt) + 1] = P.tab[size_t(mt)] + uint32_t(count(S, mt));
        cmax = std::max(cmax, count(S, mt));
    }
    P.slots = int(P.tab[size_t(P.mtiles)]);
    // items in the order (split, strip, box group, row tile): the row tiles of
    // one split and strip walk the same stages and share their B records
    for (int k = 0; k < cmax; ++k)
        for (int j = 0; j < P.nstrips; ++j)
            for (int h = 0; h < P.ngroups; ++h)
                for (int mt = 0; mt < P.mtiles; ++mt) {
                    const int cnt = count(S, mt);
                    if (k >= cnt) continue;
                    const int64_t T = stages(mt, j, h);
                    Fwd16Item it;
                    it.mt = mt;
                    it.j = j;
                    it.h = h;
                    it.r_lo = rlo[size_t(mt) * P.ngroups + h];
                    it.nrows = nrow[size_t(mt) * P.ngroups + h];
                    it.st_begin = int(T * k / cnt);
                    it.st_end = int(T * (k + 1) / cnt);
                    it.slot = int(P.tab[size_t(mt)]) + k;
                    P.items.push_back(it);
                }
    P.nitems = int(P.items.size());
    P.nwg = (P.nitems + 3) / 4;
    // the multiply-high divisions of the kernel are exact below 2^32 / d:
    // positions (at most Kr rows times Kt / ny + 1 columns) by their column
    // count, and the biased shifts by nx and ny
    const uint64_t cmaxcols = uint64_t(P.Kt) / g.ny + 1;
    if (uint64_t(g.Kr) * cmaxcols * cmaxcols >= (uint64_t(1) << 32)) P.ok = false;
    if (Tmax >= (int64_t(1) << 31) || P.nitems >= (1 << 24) ||
        uint64_t(P.slots) * kMT * uint64_t(P.ncols) >= (uint64_t(1) << 31))
        P.ok = false;
    P.part_bytes = align256(size_t(P.slots) * kMT * P.ncols * sizeof(float));
    P.items_bytes = align256(size_t(P.nitems) * sizeof(Fwd16Item));
    P.tab_bytes = align256(P.tab.size() * sizeof(uint32_t));
    return P;
}

// Items, then the slot table, as words (written by put_words).
std::vector<uint32_t> fwd16_words(const Fwd16Plan& P)
{
    std::vector<uint32_t> w(P.items_bytes / 4 + P.tab.size(), 0u);
    std::memcpy(w.data(), P.items.data(), P.items.size() * sizeof(Fwd16Item));
    std::memcpy(w.data() + P.items_bytes / 4, P.tab.data(), P.tab.size() * sizeof(uint32_t));
    return w;
}

Fwd16Pack fwd16_pack(const Fwd16Plan& P)
{
    Fwd16Pack p{};
    p.g = P.g;
    p.nch = P.nch;
    p.nstrips = P.nstrips;
    p.nbox = P.nbox;
    p.padP = P.padP;
    p.padQ = P.padQ;
    p.LRp = P.LRp;
    p.LCp = P.LCp;
    p.Kt = P.Kt;
    return p;
}

hipError_t pack16_b(const float* H, const Fwd16Plan& P, float* B16, hipStream_t stream)
{
    const int64_t nrec = int64_t(P.B_bytes / 32);
    hipLaunchKernelGGL(k_pack16_b, dim3(unsigned((nrec + 255) / 256)), dim3(256), 0, stream, H, fwd16_pack(P), B16,
                       nrec);
    return hipGetLastError();
}

// On a prepared operator: Bpre its B16 records, tables its items and slot
// table.  Workspace: g with depth innermost, the A16 records, the partial sums.
hipError_t forward16_impl(const Fwd16Plan& P, const float* gin, const float* fmeas, float* f, void* ws,
                          const float* Bpre, const uint32_t* tables, hipStream_t stream)
{
    if (!Bpre || !tables) return hipErrorInvalidValue;
    const ProjGeom& g = P.g;
    char* w = static_cast<char*>(ws);
    float* gT = reinterpret_cast<float*>(w);
    float* A16 = reinterpret_cast<float*>(w + P.gT_bytes);
    float* part = reinterpret_cast<float*>(w + P.gT_bytes + P.A_bytes);
    const float* B16 = Bpre;
    hipError_t e;
    const int plane = g.R * g.C;
    hipLaunchKernelGGL(k_depth_last, dim3(unsigned((plane + 31) / 32), unsigned((g.nz + 31) / 32)), dim3(256), 0,
                       stream, gin, g.nz, plane, gT);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t nrec_a = int64_t(P.A_bytes / 32);
    hipLaunchKernelGGL(k_pack16_a, dim3(unsigned((nrec_a + 255) / 256)), dim3(256), 0, stream, gT, fwd16_pack(P), A16,
                       nrec_a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    Fwd16Args a{};
    a.A = A16;
    a.B = B16;
    a.out = part;
    a.items = reinterpret_cast<const Fwd16Item*>(tables);
    a.A_bytes = uint32_t(P.A_bytes);
    a.B_bytes = uint32_t(P.B_bytes);
    a.nitems = P.nitems;
    a.nwg = P.nwg;
    a.ns = g.ns;
    a.nt = g.nt;
    a.nx = g.nx;
    a.ny = g.ny;
    a.M = g.M;
    a.Lc = g.Lc;
    a.LCp = P.LCp;
    a.Kt = P.Kt;
    a.hsb = g.hs + g.nx * P.padP;
    a.htb = g.ht + g.ny * P.padQ;
    a.PL = P.nch * P.LRp * P.LCp;
    a.nch = P.nch;
    a.nbx = P.nstrips * P.nbox * 16;
    a.nbox = P.nbox;
    a.ncols = P.ncols;
    a.mnx = div_magic(uint32_t(g.nx));
    a.mny = div_magic(uint32_t(g.ny));
    if (P.nwg > 0) {
        hipLaunchKernelGGL(k_fwd16, dim3(unsigned(P.nwg)), dim3(kThreads), 0, stream, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const uint32_t* tab = tables + P.items_bytes / 4;
    hipLaunchKernelGGL(k_fwd16_reduce, dim3(blocks_for(int64_t(P.mtiles) * kMT * P.ncols)), dim3(256), 0, stream, part,
                       tab, P.ncols, P.nbox, g, fmeas, f);
    return hipGetLastError();
}

}  // namespace

// Workspace of the forward projection: g with depth innermost, the A and B
// records, then the split partial tiles.
size_t forward_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const FwdPlan P = fwd_plan(s, R, C);
    return P.gT_bytes + P.gS_bytes + P.B_bytes + P.part_bytes;
}

// Workspace of the backprojection: the A and B records.
size_t backward_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const BwdPlan P = bwd_plan(s, R, C);
    return P.A_bytes + P.B_bytes;
}

namespace {

// Bpre: the B records of H already packed (a prepared operator), or null to
// pack them into the workspace.  Workspace: g with depth innermost, the A
// records, the B records unless prepared, the split partial tiles.
hipError_t forward_impl(const float* H, const lfbp_shape& s, const float* gin, int64_t R, int64_t C,
                        const float* fmeas, float* f, void* ws, const float* Bpre, const uint32_t* tabpre,
                        hipStream_t stream)
{
    // A prepared operator holds the 16-column forward's records.  A call that
    // packs its own records takes the 64-column forward: the 16-column records
    // and work table cost 0.9 ms a call to write against 0.4 ms (projector
    // workload), more than the faster product saves.
    if (Bpre) {
        const Fwd16Plan Q = fwd16_plan(s, R, C);
        if (Q.ok) return forward16_impl(Q, gin, fmeas, f, ws, Bpre, tabpre, stream);
    }
    const FwdPlan P = fwd_plan(s, R, C);
    const ProjGeom& g = P.g;
    if (int64_t(P.mtiles) * P.ntiles >= (int64_t(1) << 26)) return hipErrorInvalidValue;   // work table entries
    char* w = static_cast<char*>(ws);
    float* gT = reinterpret_cast<float*>(w);
    float* gS = reinterpret_cast<float*>(w + P.gT_bytes);
    float* Bp = reinterpret_cast<float*>(w + P.gT_bytes + P.gS_bytes);
    float* part = reinterpret_cast<float*>(w + P.gT_bytes + P.gS_bytes + (Bpre ? 0 : P.B_bytes));
    // the work table: prepared with the operator, else written into the
    // workspace after the partial sums (stream-ordered, no allocation)
    const uint32_t* tab = tabpre;
    if (!tab) {
        uint32_t* t = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(part) + (P.part_bytes - P.tab_bytes));
        const hipError_t et = put_words(t, P.tab.data(), P.tab.size(), stream);
        if (et != hipSuccess) return et;
        tab = t;
    }

    PackArgs p = pack_args(g, P.N, P.Npad, P.Mpad, P.L.stages);
    p.nzc = P.L.nzc;
    p.LRp = P.L.LRp;
    p.LCp = P.L.LCp;
    p.padP = P.L.padP;
    p.padQ = P.L.padQ;
    p.fnzc = make_fastdiv(uint32_t(P.L.nzc));
    p.fLCp = make_fastdiv(uint32_t(P.L.LCp));
    p.cb = P.cb;

    const int plane = g.R * g.C;
    hipLaunchKernelGGL(k_depth_last, dim3(unsigned((plane + 31) / 32), unsigned((g.nz + 31) / 32)), dim3(256), 0,
                       stream, gin, g.nz, plane, gT);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack_fwd_a, dim3(unsigned(P.N * P.L.nzc), blocks_for(int64_t(P.L.LRp) * P.L.LCp * kRecVec)),
                       dim3(256), 0, stream, gT, p, gS);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (Bpre) {
        Bp = const_cast<float*>(Bpre);
    } else {
        hipLaunchKernelGGL(k_pack_fwd_b, dim3(unsigned(P.L.stages), unsigned(P.ntiles)), dim3(kThreads), 0, stream, H,
                           p, Bp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }

    GemmArgs a{};
    a.A = gS;
    a.B = Bp;
    a.out = part;
    a.g = g;
    a.M = g.M;
    a.N = P.N;
    a.Mpad = P.Mpad;
    a.Npad = P.Npad;
    a.mtiles = P.mtiles;
    a.ntiles = P.ntiles;
    a.stages = P.L.stages;
    a.splits = P.splits;
    a.nzc = P.L.nzc;
    a.LRp = P.L.LRp;
    a.LCp = P.L.LCp;
    a.padP = P.L.padP;
    a.padQ = P.L.padQ;
    a.fnzc = p.fnzc;
    a.cb = P.cb;
    a.walk = window_walk(g, P.cb);
    a.tab = tab;
    a.nwg = P.nwg;
    hipLaunchKernelGGL(k_gemm<kModeFwd>, dim3(unsigned(P.nwg)), dim3(kThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t npix = int64_t(g.R) * g.C;
    hipLaunchKernelGGL(k_fwd_reduce, dim3(blocks_for(npix)), dim3(256), 0, stream, part, tab, P.Npad, g, P.cb, fmeas,
                       f);
    return hipGetLastError();
}

// Bpre: the B records of H' already packed, or null.  Workspace: the A
// records, then the B records unless prepared.
hipError_t backward_impl(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C,
                         const float* gprev, const float* norm, float* g_out, void* ws, const float* Bpre,
                         hipStream_t stream)
{
    const BwdPlan P = bwd_plan(s, R, C);
    const ProjGeom& g = P.g;
    char* w = static_cast<char*>(ws);
    float* Ap = reinterpret_cast<float*>(w);
    float* Bp = Bpre ? const_cast<float*>(Bpre) : reinterpret_cast<float*>(w + P.A_bytes);
    const PackArgs p = pack_args(g, P.N, P.Npad, P.Mpad, P.stages);
    hipLaunchKernelGGL(k_pack_bwd_a, dim3(unsigned(P.stages), blocks_for(int64_t(P.Mpad) * kRecVec)), dim3(256), 0,
                       stream, f, p, Ap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!Bpre) {
        hipLaunchKernelGGL(k_pack_bwd_b, dim3(unsigned(P.stages), blocks_for(int64_t(P.Npad) * kRecVec)), dim3(256),
                           0, stream, Ht, p, Bp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    GemmArgs a{};
    a.A = Ap;
    a.B = Bp;
    a.out = g_out;
    a.g = g;
    a.M = g.M;
    a.N = P.N;
    a.Mpad = P.Mpad;
    a.Npad = P.Npad;
    a.mtiles = P.mtiles;
    a.ntiles = P.ntiles;
    a.stages = P.stages;
    a.splits = 1;
    a.nzc = 1;
    a.fnzc = make_fastdiv(1);
    a.gprev = gprev;
    a.norm = norm;
    hipLaunchKernelGGL(k_gemm<kModeBwd>, dim3(unsigned(P.mtiles * P.ntiles)), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_forward_ws(const float* H, const lfbp_shape& s, const float* gin, int64_t R, int64_t C, float* f,
                             void* ws, hipStream_t stream)
{
    return forward_impl(H, s, gin, R, C, nullptr, f, ws, nullptr, nullptr, stream);
}

hipError_t launch_backward_ws(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                              void* ws, hipStream_t stream)
{
    return backward_impl(Ht, s, f, R, C, nullptr, nullptr, g, ws, nullptr, stream);
}

namespace {

struct GradPlan {
    ProjGeom g;
    int M, N, Mpad, Npad, mtiles, ntiles, stages;
    size_t A_bytes, B_bytes;
};

GradPlan grad_plan(const lfbp_shape& s, int64_t R, int64_t C)
{
    GradPlan P;
    P.g = make_geom(s, R, C);
    P.M = P.g.Kr * P.g.Kc;
    P.N = P.g.nx * P.g.ny * P.g.nz;
    P.mtiles = (P.M + kMT - 1) / kMT;
    P.ntiles = (P.N + kNT - 1) / kNT;
    P.Mpad = P.mtiles * kMT;
    P.Npad = P.ntiles * kNT;
    P.stages = (P.g.M + kStageK - 1) / kStageK;
    P.A_bytes = align256(size_t(P.stages) * P.Mpad * kRec * sizeof(float));
    P.B_bytes = align256(size_t(P.stages) * P.Npad * kRec * sizeof(float));
    return P;
}

}  // namespace

// Workspace of the gradient with respect to H: the A and B records.
size_t grad_psf_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const GradPlan P = grad_plan(s, R, C);
    return P.A_bytes + P.B_bytes;
}

// dH = d<w, H g>/dH for the image gradient w [R][C] and the volume g [nz][R][C].
hipError_t launch_grad_psf_ws(const float* w, const float* gv, const lfbp_shape& s, int64_t R, int64_t C, float* dH,
                              void* ws, hipStream_t stream)
{
    const GradPlan P = grad_plan(s, R, C);
    char* wsp = static_cast<char*>(ws);
    float* Ap = reinterpret_cast<float*>(wsp);
    float* Bp = reinterpret_cast<float*>(wsp + P.A_bytes);
    const PackArgs p = pack_args(P.g, P.N, P.Npad, P.Mpad, P.stages);
    hipLaunchKernelGGL(k_pack_gh_a, dim3(unsigned(P.stages), blocks_for(int64_t(P.Mpad) * kRecVec)), dim3(256), 0,
                       stream, w, p, Ap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack_gh_b, dim3(unsigned(P.stages), blocks_for(int64_t(P.Npad) * kRecVec)), dim3(256), 0,
                       stream, gv, p, Bp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GemmArgs a{};
    a.A = Ap;
    a.B = Bp;
    a.out = dH;
    a.g = P.g;
    a.M = P.M;
    a.N = P.N;
    a.Mpad = P.Mpad;
    a.Npad = P.Npad;
    a.mtiles = P.mtiles;
    a.ntiles = P.ntiles;
    a.stages = P.stages;
    a.splits = 1;
    a.nzc = 1;
    a.fnzc = make_fastdiv(1);
    hipLaunchKernelGGL(k_gemm<kModeGradH>, dim3(unsigned(P.mtiles * P.ntiles)), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_grad_psf(const float* w, const float* gv, const lfbp_shape& s, int64_t R, int64_t C, float* dH,
                           hipStream_t stream)
{
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, grad_psf_workspace_bytes(s, R, C), stream);
    if (e != hipSuccess) return e;
    e = launch_grad_psf_ws(w, gv, s, R, C, dH, ws, stream);
    const hipError_t e2 = hipFreeAsync(ws, stream);
    return e != hipSuccess ? e : e2;
}

// Workspace of one Richardson-Lucy step: the larger of the two projections'
// workspaces (used one after the other), then the quotient image.
size_t rl_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    return align256(std::max(forward_workspace_bytes(s, R, C), backward_workspace_bytes(s, R, C))) +
           align256(size_t(R) * size_t(C) * sizeof(float));
}

// g_out = g / (H' 1) * H'(fmeas / (H g)) (Eq. 2): the forward ends in the
// quotient, the backprojection's epilogue applies the update.  g_out may be g.
hipError_t launch_rl_step_ws(const float* H, const float* Ht, const lfbp_shape& s, const float* fmeas, int64_t R,
                             int64_t C, const float* g, const float* norm, float* g_out, void* ws,
                             hipStream_t stream)
{
    float* ratio = reinterpret_cast<float*>(
        static_cast<char*>(ws) + align256(std::max(forward_workspace_bytes(s, R, C), backward_workspace_bytes(s, R, C))));
    hipError_t e = forward_impl(H, s, g, R, C, fmeas, ratio, ws, nullptr, nullptr, stream);
    if (e != hipSuccess) return e;
    return backward_impl(Ht, s, ratio, R, C, g, norm, g_out, ws, nullptr, stream);
}

namespace {

__global__ void __launch_bounds__(256) k_fill(float* p, int64_t n, float v)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

// norm = H' 1: the backprojection of an all-ones image (the normaliser of Eq. 2).
hipError_t launch_rl_norm_ws(const float* Ht, const lfbp_shape& s, int64_t R, int64_t C, float* norm, void* ws,
                             hipStream_t stream)
{
    float* ones = reinterpret_cast<float*>(
        static_cast<char*>(ws) + align256(std::max(forward_workspace_bytes(s, R, C), backward_workspace_bytes(s, R, C))));
    const int64_t n = R * C;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, stream, ones, n, 1.0f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return backward_impl(Ht, s, ones, R, C, nullptr, nullptr, norm, ws, nullptr, stream);
}

hipError_t launch_rl_step(const float* H, const float* Ht, const lfbp_shape& s, const float* fmeas, int64_t R,
                          int64_t C, const float* g, const float* norm, float* g_out, hipStream_t stream)
{
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, rl_workspace_bytes(s, R, C), stream);
    if (e != hipSuccess) return e;
    e = launch_rl_step_ws(H, Ht, s, fmeas, R, C, g, norm, g_out, ws, stream);
    const hipError_t e2 = hipFreeAsync(ws, stream);
    return e != hipSuccess ? e : e2;
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
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, backward_workspace_bytes(s, R, C), stream);
    if (e != hipSuccess) return e;
    e = launch_backward_ws(Ht, s, f, R, C, g, ws, stream);
    const hipError_t e2 = hipFreeAsync(ws, stream);
    return e != hipSuccess ? e : e2;
}

// ------------------------------------------------------- prepared operators

// A prepared operator holds the B records of H (forward) and of H'
// (backward), which depend on the PSF only, so that a loop over volumes and
// images with one PSF (Richardson-Lucy, Eq. 2) packs them once, and the
// forward's work table, which depends on the shapes only.
namespace {

// The forward's part of a prepared operator: its B records, and its tables.
size_t op_fwd_b_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const Fwd16Plan Q = fwd16_plan(s, R, C);
    return align256(Q.ok ? Q.B_bytes : fwd_plan(s, R, C).B_bytes);
}

size_t op_fwd_tab_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const Fwd16Plan Q = fwd16_plan(s, R, C);
    return Q.ok ? Q.items_bytes + Q.tab_bytes : fwd_plan(s, R, C).tab_bytes;
}

// Workspace of a forward call on a prepared operator: g with depth
// innermost, the A records, the partial sums.
size_t op_fwd_call_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const Fwd16Plan Q = fwd16_plan(s, R, C);
    if (Q.ok) return Q.gT_bytes + Q.A_bytes + Q.part_bytes;
    const FwdPlan F = fwd_plan(s, R, C);
    return F.gT_bytes + F.gS_bytes + F.part_bytes;
}

}  // namespace

size_t operator_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    return op_fwd_b_bytes(s, R, C) + align256(bwd_plan(s, R, C).B_bytes) + op_fwd_tab_bytes(s, R, C);
}

// Workspace of every call on a prepared operator (forward, backward, one
// Richardson-Lucy update or its normaliser): the per-call records and, after
// them, one image.
size_t operator_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C)
{
    const BwdPlan Bw = bwd_plan(s, R, C);
    return align256(std::max(op_fwd_call_bytes(s, R, C), Bw.A_bytes)) + align256(size_t(R) * size_t(C) * sizeof(float));
}

namespace {

const float* op_fwd_b(const void* op) { return static_cast<const float*>(op); }

const float* op_bwd_b(const void* op, const lfbp_shape& s, int64_t R, int64_t C)
{
    return reinterpret_cast<const float*>(static_cast<const char*>(op) + op_fwd_b_bytes(s, R, C));
}

const uint32_t* op_fwd_tab(const void* op, const lfbp_shape& s, int64_t R, int64_t C)
{
    return reinterpret_cast<const uint32_t*>(static_cast<const char*>(op) + op_fwd_b_bytes(s, R, C) +
                                             align256(bwd_plan(s, R, C).B_bytes));
}

float* op_image(void* ws, const lfbp_shape& s, int64_t R, int64_t C)
{
    const BwdPlan Bw = bwd_plan(s, R, C);
    return reinterpret_cast<float*>(static_cast<char*>(ws) + align256(std::max(op_fwd_call_bytes(s, R, C), Bw.A_bytes)));
}

}  // namespace

hipError_t launch_operator_prepare(const float* H, const float* Ht, const lfbp_shape& s, int64_t R, int64_t C,
                                   void* op, hipStream_t stream)
{
    const Fwd16Plan Q = fwd16_plan(s, R, C);
    if (Q.ok) {
        hipError_t e = pack16_b(H, Q, const_cast<float*>(op_fwd_b(op)), stream);
        if (e != hipSuccess) return e;
        const std::vector<uint32_t> words = fwd16_words(Q);
        e = put_words(const_cast<uint32_t*>(op_fwd_tab(op, s, R, C)), words.data(), words.size(), stream);
        if (e != hipSuccess) return e;
        const BwdPlan Bw = bwd_plan(s, R, C);
        const PackArgs pb = pack_args(Bw.g, Bw.N, Bw.Npad, Bw.Mpad, Bw.stages);
        hipLaunchKernelGGL(k_pack_bwd_b, dim3(unsigned(Bw.stages), blocks_for(int64_t(Bw.Npad) * kRecVec)), dim3(256),
                           0, stream, Ht, pb, const_cast<float*>(op_bwd_b(op, s, R, C)));
        return hipGetLastError();
    }
    const FwdPlan F = fwd_plan(s, R, C);
    PackArgs p = pack_args(F.g, F.N, F.Npad, F.Mpad, F.L.stages);
    p.nzc = F.L.nzc;
    p.LRp = F.L.LRp;
    p.LCp = F.L.LCp;
    p.padP = F.L.padP;
    p.padQ = F.L.padQ;
    p.fnzc = make_fastdiv(uint32_t(F.L.nzc));
    p.fLCp = make_fastdiv(uint32_t(F.L.LCp));
    p.cb = F.cb;
    hipLaunchKernelGGL(k_pack_fwd_b, dim3(unsigned(F.L.stages), unsigned(F.ntiles)), dim3(kThreads), 0, stream, H, p,
                       const_cast<float*>(op_fwd_b(op)));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = put_words(const_cast<uint32_t*>(op_fwd_tab(op, s, R, C)), F.tab.data(), F.tab.size(), stream);
    if (e != hipSuccess) return e;
    const BwdPlan Bw = bwd_plan(s, R, C);
    const PackArgs pb = pack_args(Bw.g, Bw.N, Bw.Npad, Bw.Mpad, Bw.stages);
    hipLaunchKernelGGL(k_pack_bwd_b, dim3(unsigned(Bw.stages), blocks_for(int64_t(Bw.Npad) * kRecVec)), dim3(256), 0,
                       stream, Ht, pb, const_cast<float*>(op_bwd_b(op, s, R, C)));
    return hipGetLastError();
}

hipError_t launch_forward_op(const void* op, const lfbp_shape& s, const float* g, int64_t R, int64_t C, float* f,
                             void* ws, hipStream_t stream)
{
    return forward_impl(nullptr, s, g, R, C, nullptr, f, ws, op_fwd_b(op), op_fwd_tab(op, s, R, C), stream);
}

hipError_t launch_backward_op(const void* op, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                              void* ws, hipStream_t stream)
{
    return backward_impl(nullptr, s, f, R, C, nullptr, nullptr, g, ws, op_bwd_b(op, s, R, C), stream);
}

hipError_t launch_rl_step_op(const void* op, const lfbp_shape& s, const float* fmeas, int64_t R, int64_t C,
                             const float* g, const float* norm, float* g_out, void* ws, hipStream_t stream)
{
    float* ratio = op_image(ws, s, R, C);
    hipError_t e = forward_impl(nullptr, s, g, R, C, fmeas, ratio, ws, op_fwd_b(op), op_fwd_tab(op, s, R, C), stream);
    if (e != hipSuccess) return e;
    return backward_impl(nullptr, s, ratio, R, C, g, norm, g_out, ws, op_bwd_b(op, s, R, C), stream);
}

hipError_t launch_rl_norm_op(const void* op, const lfbp_shape& s, int64_t R, int64_t C, float* norm, void* ws,
                             hipStream_t stream)
{
    float* ones = op_image(ws, s, R, C);
    const int64_t n = R * C;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, stream, ones, n, 1.0f);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return backward_impl(nullptr, s, ones, R, C, nullptr, nullptr, norm, ws, op_bwd_b(op, s, R, C), stream);
}

}  // namespace lfbp
