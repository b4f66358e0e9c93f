/*
 * lfbp.h -- light-field backprojection arrays on AMD Instinct MI355X (gfx950).
 *
 * C ABI of liblfbp.so.  Every data pointer is DEVICE memory owned by the
 * caller (for example a torch allocation); the library never frees it.  Every
 * call is ordered on `stream` (a hipStream_t passed as void*; NULL means the
 * null stream), returns as soon as the work is queued and never synchronises.
 * Arguments are validated on the host before any HIP call: on an error nothing
 * is launched and the status says why.  No C++ exception and no abort crosses
 * this interface.  Calls may be made from several threads at once.
 *
 * Memory the library takes for itself, by call:
 *   none        lfbp_compute_Ht(_config), lfbp_compute_Ht_inplace,
 *               lfbp_compute_Ht_colmajor, lfbp_compute_Ht_batched_noalloc, and
 *               every _ws and _op projector call (the caller passes the
 *               workspace);
 *   plan cache  lfbp_compute_Ht_batched(_config): a plan per distinct problem
 *               table; one hipMalloc per plan only for a table of more than 16
 *               problems (descriptor table) and a captured graph only when
 *               asked for; at most 32 plans; freed by lfbp_release_plans;
 *   stream-ordered workspace  lfbp_forward, lfbp_backward, lfbp_rl_step,
 *               lfbp_grad_psf: the operand records of their matrix-core
 *               products (hundreds of MB at projector sizes) come from
 *               hipMallocAsync on `stream` and are returned with hipFreeAsync
 *               on the same stream, so these calls stay stream-ordered and
 *               never block; callers that cannot allocate use the _ws forms.
 *
 * Arrays are row-major with the last axis fastest:
 *   PSF array H and backprojection array H'   [ns][nt][nx][ny][nz]
 *       s,t = pixel row/column inside a pattern cut-out (ns x nt pixels),
 *       x,y = source position inside the elementary cell (nx x ny positions),
 *       z   = depth plane.
 *   Volume g  [nz][R][C]   and   image f  [R][C]   share the lateral grid.
 * In H' the roles of the axes are swapped (Sec. 3, Fig. 6 discussion): axes 3-4
 * hold the class (position inside a lenslet period) of an image pixel and axes
 * 1-2 the offset of a voxel from that pixel, so H'[.,.,x',y',z] is the
 * backprojection of a pixel of class (x',y') into depth plane z.
 */
#ifndef LFBP_H
#define LFBP_H

#include <stdint.h>

#if defined(__GNUC__)
#define LFBP_API __attribute__((visibility("default")))
#else
#define LFBP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LFBP_OK = 0,
    LFBP_EINVAL = -1,  /* null pointer, count <= 0, image size < 1, bad config field */
    LFBP_ESHAPE = -2,  /* a dimension < 1, an even ns/nt/nx/ny, or a size beyond the limits below */
    LFBP_EDTYPE = -3,  /* unknown element type, or one the call does not support */
    LFBP_EALIAS = -4,  /* input and output ranges overlap (in-place is not supported) */
    LFBP_EDEVICE = -5, /* a HIP call failed (launch error, no device) */
    LFBP_ENOMEM = -6,  /* the library could not allocate its own device or host memory */
    LFBP_EALIGN = -7,  /* a pointer is not aligned to its element size */
    LFBP_ECAPTURE = -8, /* the call would have to allocate, and its stream is being captured into a graph */
    LFBP_ESCRATCH = -9  /* the call needs more than the library's fixed device scratch holds */
} lfbp_status;

typedef enum { LFBP_F32 = 0, LFBP_F16 = 1 } lfbp_dtype;

typedef struct {
    int64_t ns, nt, nx, ny, nz;
} lfbp_shape;

/*
 * lfbp_compute_Ht -- the backprojection array H' from the PSF array H by pure
 * re-arrangement (Sec. 4, Eq. 3 with the index relations of Eqs. 4-9; Fig. 10).
 *
 *   H'[s'][t'][x'][y'][z] = H[ns-1-s'][nt-1-t'][(x'+s'-hs) mod nx][(y'+t'-ht) mod ny][z]
 *
 * with hs = (ns-1)/2, ht = (nt-1)/2 and mod the non-negative remainder.  This
 * is the paper's relation with the periodic extension of H (Sec. 4, Figs. 8-9)
 * applied to every entry, i.e. H' is exactly the adjoint of the forward model
 * f = H g (Sec. 2.1, Eq. 1) in convolutional form; the map is its own inverse
 * (Sec. 3: the transformation is reversible).
 *
 * H, Ht   device pointers to ns*nt*nx*ny*nz elements of `dtype`, aligned to the
 *         element size, non-overlapping.  H is read, Ht is overwritten.
 * shape   ns, nt, nx, ny odd (Sec. 4 requires odd nx, ny; the reflection of
 *         Eqs. 8-9 needs odd ns, nt), all >= 1; nz >= 1.  ns*nt*nx < 2^31,
 *         nx*ny*nz < 2^31, total bytes < 2^62.
 * dtype   LFBP_F32 or LFBP_F16; values move as raw bits (NaN payloads, -0 and
 *         denormals are preserved).
 * Errors  EINVAL, ESHAPE, EDTYPE, EALIAS, EALIGN before launch; EDEVICE if the
 *         launch fails.  Allocates nothing.
 */
LFBP_API lfbp_status lfbp_compute_Ht(const void* H, void* Ht, lfbp_shape shape, lfbp_dtype dtype, void* stream);

/*
 * Kernel choice for the re-arrangement.  variant:
 *   LFBP_GATHER_AUTO   -- the library's tuned choice for the shape (default)
 *   LFBP_GATHER_DIRECT -- each wavefront copies whole x-rows (ny*nz contiguous
 *                         elements) straight from H to H' with the rotation
 *                         applied to the read addresses (4/2-byte accesses)
 *   LFBP_GATHER_STAGED -- rows are read with 4/2-byte loads and rotated into
 *                         an LDS tile laid out like H', which is written with
 *                         16-byte stores
 *   LFBP_GATHER_WIDE   -- as STAGED, but rows are also read with 16-byte
 *                         loads (aligned supersets of each row)
 * Zero in any field selects the tuned value for that field.
 */
enum { LFBP_GATHER_AUTO = 0, LFBP_GATHER_DIRECT = 1, LFBP_GATHER_STAGED = 2, LFBP_GATHER_WIDE = 3 };

typedef struct {
    int32_t variant;        /* LFBP_GATHER_* */
    int32_t block_threads;  /* 64..512, multiple of 64 */
    int32_t rows_in_flight; /* DIRECT, STAGED: x-rows a wavefront loads before it stores, 1 or 2 */
    int32_t tile_bytes;     /* STAGED: LDS tile per workgroup, bytes (<= 65536) */
    int32_t vec_per_thread; /* WIDE: 16-byte loads per thread per work unit, 2, 4 or 8 */
    int32_t nontemporal;    /* 1: streaming stores, 2: regular stores */
    int32_t persistent;     /* 1: `grid` workgroups loop over the work units (WIDE overlaps the loads of
                               the next unit with the stores of the current one); 2: one workgroup per unit */
    int32_t grid;           /* persistent grid size; 0 = every workgroup slot of the device */
    int32_t waves_per_eu;   /* occupancy cap: at most this many wavefronts per SIMD (1..8; 8 = no cap),
                               enforced by reserving LDS per workgroup */
    int32_t schedule;       /* order in which work units meet the XCDs.  Plain WIDE launches: 1 = each XCD
                               takes one contiguous range of units, 2 = units in launch order (consecutive
                               units on different XCDs).  Batched: 1 = every XCD takes an even contiguous
                               share of every problem, largest problems first; 2 = the units of all
                               problems in launch order, largest problems first */
} lfbp_gather_config;

/* lfbp_compute_Ht with an explicit kernel choice (used by the autotuner and by
 * tests that cover each variant).  cfg may be NULL (same as lfbp_compute_Ht).
 * Errors as lfbp_compute_Ht, plus EINVAL for an out-of-range cfg field. */
LFBP_API lfbp_status lfbp_compute_Ht_config(const void* H, void* Ht, lfbp_shape shape, lfbp_dtype dtype,
                                   const lfbp_gather_config* cfg, void* stream);

/* The configuration lfbp_compute_Ht uses for this shape and dtype (every field
 * resolved, none zero).  Errors: EINVAL (cfg NULL), ESHAPE, EDTYPE. */
LFBP_API lfbp_status lfbp_default_config(lfbp_shape shape, lfbp_dtype dtype, lfbp_gather_config* cfg);

typedef struct {
    const void* H;
    void* Ht;
    lfbp_shape shape;
} lfbp_problem;

/*
 * lfbp_compute_Ht_batched -- H' for `count` independent PSF arrays (for
 * example a depth sweep, or several lens/MLA configurations) in ONE kernel
 * launch (Sec. 3.1: PSF updates inside iterative reconstruction need H'
 * recomputed often).  Each problem obeys the rules of lfbp_compute_Ht; all
 * share `dtype`.  Results are bit-identical to count separate calls.  Each
 * problem is cut into work units of its own size (the tuned size of its shape
 * class) and every XCD of the GPU takes an even share of every problem,
 * largest problems first.
 *
 * problems  HOST array of `count` descriptors (copied; may be freed on return).
 * Ownership The library keeps a plan per distinct problem table (pointers and
 *           shapes): launch parameters and, for more than 16 problems, a
 *           device descriptor table.  A call with a new table makes its plan
 *           (one hipMalloc when a device table is needed; the table is written
 *           by small kernels on `stream`, so nothing blocks); a call with a
 *           known table launches at once.  At most 32 plans are kept, least
 *           recently used dropped first; a dropped plan's device memory is
 *           freed only after every launch of it has finished.  A plan used by
 *           a call made under stream capture is kept until
 *           lfbp_release_plans(), because the caller's graph reads it.  A new
 *           plan that needs device memory (more than 16 problems, or
 *           use_graph = 1) cannot be made while `stream` is being captured:
 *           such a call returns ECAPTURE before any HIP call, and the capture
 *           stays valid (submit the table once outside the capture).
 *           lfbp_plan_count() reports the plans held.
 * Errors    EINVAL (problems NULL, count <= 0, or any pointer NULL), ESHAPE,
 *           EDTYPE, EALIGN, EALIAS (any input overlapping any output) -- all
 *           checked before anything is launched; ENOMEM, EDEVICE.
 */
LFBP_API lfbp_status lfbp_compute_Ht_batched(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype,
                                    void* stream);

/*
 * lfbp_compute_Ht_inplace -- H' written over H (the same re-arrangement as
 * lfbp_compute_Ht).  The map is its own inverse (Sec. 4: applying it to H'
 * gives H back), so the array is rewritten in disjoint pairs of x-row groups
 * with no second array; calling it twice restores H.  Requires 2*ny*nz*esize
 * <= 65536 bytes (one x-row and its partner in LDS), else ESHAPE.  Errors
 * EINVAL, EDTYPE, ESHAPE, EALIGN, EDEVICE.  Allocates nothing.
 */
LFBP_API lfbp_status lfbp_compute_Ht_inplace(void* H, lfbp_shape shape, lfbp_dtype dtype, void* stream);

/*
 * lfbp_compute_Ht_colmajor -- H' (the re-arrangement of lfbp_compute_Ht,
 * Sec. 4, Eqs. 4-9) for arrays stored COLUMN-MAJOR: element (s, t, x, y, z)
 * at ((((z*ny + y)*nx + x)*nt + t)*ns + s), s fastest -- the order of the
 * Matlab arrays the paper's implementation works on (Sec. 5, Table 1).  The
 * shape fields keep their meaning; Ht has the same layout.  Results are
 * bit-identical to lfbp_compute_Ht on the transposed arrays.
 *
 * H, Ht     DEVICE pointers, ns*nt*nx*ny*nz elements each, aligned to the
 *           element size, not overlapping; the caller owns both.
 * Shape     as lfbp_compute_Ht, and nx <= 2048 and nt*ny*nz*ns < 2^31,
 *           else ESHAPE.
 * Errors    EINVAL, EDTYPE, ESHAPE, EALIGN, EALIAS (checked before launch),
 *           EDEVICE.  Allocates nothing; asynchronous on `stream`.
 */
LFBP_API lfbp_status lfbp_compute_Ht_colmajor(const void* H, void* Ht, lfbp_shape shape, lfbp_dtype dtype,
                                              void* stream);

/*
 * lfbp_compute_Ht_batched_noalloc -- lfbp_compute_Ht_batched for callers that
 * cannot allocate device memory: code being captured into a graph, tight
 * serving loops, harnesses that forbid allocation.  Same problems, same
 * results (bit-identical), same kernels and tuned choice; no plan is kept.
 *
 * Scratch  Batches of more than 16 problems need a device descriptor table;
 *          here it lives in a fixed array compiled into the library (one per
 *          GPU, held until the process ends, LFBP_NOALLOC_MAX_PROBLEMS
 *          problems, about 160 KB), written by small kernels on `stream`
 *          before the gather kernel reads it.  Every call on one GPU uses the
 *          same array, so calls that overlap in time on one GPU (two streams,
 *          two threads) race: order them on one stream or synchronise between
 *          them.  Nothing in the array needs to start at zero.
 * Errors   as lfbp_compute_Ht_batched (checked before anything is launched),
 *          and ESCRATCH when count > LFBP_NOALLOC_MAX_PROBLEMS.  Calls no
 *          hipMalloc, hipFree or other device allocator, and never blocks.
 */
#define LFBP_NOALLOC_MAX_PROBLEMS 1024
LFBP_API lfbp_status lfbp_compute_Ht_batched_noalloc(const lfbp_problem* problems, int32_t count,
                                                     lfbp_dtype dtype, void* stream);

/* Same as lfbp_compute_Ht_batched with an explicit kernel choice shared by
 * every problem, and graph use: use_graph = 1 captures the launch into a
 * hipGraph when the plan is made and replays it on every call, 0 launches the
 * kernel directly (what lfbp_compute_Ht_batched does).  cfg may be NULL. */
LFBP_API lfbp_status lfbp_compute_Ht_batched_config(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype,
                                           const lfbp_gather_config* cfg, int32_t use_graph, void* stream);

/*
 * lfbp_forward -- forward projection f = H g (Sec. 2.1, Eq. 1): every voxel
 * adds its pattern, scaled by its value and centred on it, to the image;
 * voxel (z,P,Q) uses the pattern H[.,.,P mod nx, Q mod ny, z] and reaches
 * pixel (P+s-hs, Q+t-ht) with weight H[s][t][P mod nx][Q mod ny][z]:
 *
 *   f[p][q] = sum_z sum_{s,t} H[s][t][P mod nx][Q mod ny][z] g[z][P][Q],
 *             P = p-s+hs, Q = q-t+ht, terms with P, Q outside the image dropped.
 *
 * H  float32 [ns][nt][nx][ny][nz];  g float32 [nz][R][C];  f float32 [R][C],
 * overwritten.  Float32 products and sums on the matrix cores, with the
 * running sums folded into a second float32 accumulator every few hundred
 * terms and the split partial sums added in float64; results do not depend on
 * scheduling (no atomics).
 * Workspace: the operands are first copied into the layout the matrix cores
 * read (H as one record of 22 depth values per (patch shift, pixel class),
 * g split by pixel phase); this call takes lfbp_forward_workspace_size()
 * bytes for that from the stream-ordered allocator (hipMallocAsync) and
 * returns them on the stream; lfbp_forward_ws uses caller memory instead and
 * allocates nothing.
 * Errors EINVAL (null, R or C < 1), ESHAPE (including shapes whose operand
 * copies exceed the kernels' 32-bit index ranges, and shapes one of whose
 * launches would need 2^24 or more workgroups along a grid dimension: the
 * forward's (ns+nx-1)(nt+ny-1)ceil(nz/22) record stages, R*C/32, or its GEMM
 * tiles; the backward's and the gradient's GEMM tiles), EALIAS (f
 * overlapping H or g), EALIGN, ENOMEM, EDEVICE.
 */
LFBP_API lfbp_status lfbp_forward(const float* H, lfbp_shape shape, const float* g, int64_t R, int64_t C, float* f,
                                  void* stream);

/* Bytes of device workspace lfbp_forward_ws needs for this shape and image
 * (0 when the shape or image is invalid). */
LFBP_API int64_t lfbp_forward_workspace_size(lfbp_shape shape, int64_t R, int64_t C);

/* lfbp_forward with a caller-provided device workspace of at least
 * lfbp_forward_workspace_size() bytes, 256-byte aligned, not overlapping H, g
 * or f; its contents are scratch.  Errors as lfbp_forward, plus EINVAL when
 * the workspace is NULL, too small or misaligned.  Allocates nothing. */
LFBP_API lfbp_status lfbp_forward_ws(const float* H, lfbp_shape shape, const float* g, int64_t R, int64_t C,
                                     float* f, void* workspace, int64_t workspace_bytes, void* stream);

/*
 * lfbp_backward -- backprojection of an image into the volume with H'
 * (the bracketed term of Eq. 2, Sec. 3): every pixel adds its slice of H',
 * scaled by its value, to the voxels it receives light from:
 *
 *   g[z][P][Q] = sum_{p,q} f[p][q] Ht[P-p+hs][Q-q+ht][p mod nx][q mod ny][z],
 *
 * terms with the H' index outside 0..ns-1 / 0..nt-1 dropped.  With Ht from
 * lfbp_compute_Ht(H) this is exactly the adjoint of lfbp_forward(H).
 * Ht float32 [ns][nt][nx][ny][nz]; f float32 [R][C]; g float32 [nz][R][C],
 * overwritten.  Float32 on the matrix cores with the two-level accumulation
 * of lfbp_forward; deterministic.  Like lfbp_forward it first copies its
 * operands into the matrix-core layout, in lfbp_backward_workspace_size()
 * bytes taken from the stream-ordered allocator; lfbp_backward_ws uses
 * caller memory instead.  Errors EINVAL, ESHAPE, EALIAS, EALIGN, ENOMEM,
 * EDEVICE.
 */
LFBP_API lfbp_status lfbp_backward(const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C, float* g,
                                   void* stream);

/* Bytes of device workspace lfbp_backward_ws needs for this shape and image
 * (0 when the shape or image is invalid). */
LFBP_API int64_t lfbp_backward_workspace_size(lfbp_shape shape, int64_t R, int64_t C);

/* lfbp_backward with a caller-provided device workspace of at least
 * lfbp_backward_workspace_size() bytes, 256-byte aligned, not overlapping
 * Ht, f or g; its contents are scratch.  Errors as lfbp_backward, plus EINVAL
 * when the workspace is NULL, too small or misaligned.  Allocates nothing. */
LFBP_API lfbp_status lfbp_backward_ws(const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C,
                                      float* g, void* workspace, int64_t workspace_bytes, void* stream);

/*
 * lfbp_rl_step -- one Richardson-Lucy update of a volume estimate (Eq. 2):
 *
 *   g_out = g / (H' 1) * H' ( f / (H g) ),
 *
 * elementwise products and quotients; H g is lfbp_forward(H, g) and H' x is
 * lfbp_backward(Ht, x).  Where (H g)[p][q] is 0 the quotient is taken as 0;
 * where norm = H' 1 is 0 (a voxel that reaches no pixel of the image) g_out
 * is 0.  The quotient is formed in float64 from the float64 sum of the
 * forward projection; the update is formed in float32 in the backprojection's
 * epilogue, so no intermediate volume is stored.
 * H, Ht float32 [ns][nt][nx][ny][nz] (Ht = lfbp_compute_Ht(H)); f float32
 * [R][C] (the measured image); g, norm, g_out float32 [nz][R][C]; norm is
 * the backprojection of an all-ones image, computed once by the caller with
 * lfbp_backward.  g_out may be g (update in place); it must not overlap any
 * other argument.  Workspace: lfbp_rl_workspace_size() bytes from the
 * stream-ordered allocator; lfbp_rl_step_ws takes caller memory and
 * allocates nothing.  Errors as lfbp_forward and lfbp_backward.
 */
LFBP_API lfbp_status lfbp_rl_step(const float* H, const float* Ht, lfbp_shape shape, const float* f, int64_t R,
                                  int64_t C, const float* g, const float* norm, float* g_out, void* stream);

/* Bytes of device workspace lfbp_rl_step_ws needs (0 when invalid). */
LFBP_API int64_t lfbp_rl_workspace_size(lfbp_shape shape, int64_t R, int64_t C);

/* lfbp_rl_step with a caller workspace of at least lfbp_rl_workspace_size()
 * bytes, 256-byte aligned, overlapping no argument.  Allocates nothing. */
LFBP_API lfbp_status lfbp_rl_step_ws(const float* H, const float* Ht, lfbp_shape shape, const float* f, int64_t R,
                                     int64_t C, const float* g, const float* norm, float* g_out, void* workspace,
                                     int64_t workspace_bytes, void* stream);

/* norm = H' 1, the backprojection of an all-ones R x C image (the normaliser
 * of lfbp_rl_step), with a caller workspace of lfbp_rl_workspace_size() bytes
 * (256-byte aligned, overlapping neither Ht nor norm).  norm float32
 * [nz][R][C].  Allocates nothing.  Errors as lfbp_backward_ws. */
LFBP_API lfbp_status lfbp_rl_norm_ws(const float* Ht, lfbp_shape shape, int64_t R, int64_t C, float* norm,
                                     void* workspace, int64_t workspace_bytes, void* stream);

/*
 * lfbp_grad_psf -- gradient of a loss with respect to the PSF array, given
 * its gradient w = dL/df with respect to the image of f = H g (Eq. 1):
 *
 *   dH[s][t][x][y][z] = sum over voxels (P,Q) of class (x,y) of
 *                       w[P+s-hs][Q+t-ht] * g[z][P][Q]
 *
 * (pixels outside the image dropped), the derivative of <w, H g> with respect
 * to H (f is linear in H).  For calibrating or refining H from data (the
 * motivation of Sec. 3.1); H' of the updated H is a new lfbp_compute_Ht.
 * w float32 [R][C]; g float32 [nz][R][C]; dH float32 [ns][nt][nx][ny][nz],
 * overwritten, not overlapping the inputs.  Float32 on the matrix cores, one
 * sum per entry over the lenslets, with the two-level accumulation of
 * lfbp_forward.  Workspace from the stream-ordered allocator
 * (lfbp_grad_psf_workspace_size() bytes); lfbp_grad_psf_ws takes caller
 * memory and allocates nothing.  Errors EINVAL, ESHAPE, EALIAS, EALIGN,
 * ENOMEM, EDEVICE.
 */
LFBP_API lfbp_status lfbp_grad_psf(const float* w, const float* g, lfbp_shape shape, int64_t R, int64_t C, float* dH,
                                   void* stream);

/* Bytes of device workspace lfbp_grad_psf_ws needs (0 when invalid). */
LFBP_API int64_t lfbp_grad_psf_workspace_size(lfbp_shape shape, int64_t R, int64_t C);

/* lfbp_grad_psf with a caller workspace of at least
 * lfbp_grad_psf_workspace_size() bytes, 256-byte aligned, overlapping no
 * argument.  Allocates nothing. */
LFBP_API lfbp_status lfbp_grad_psf_ws(const float* w, const float* g, lfbp_shape shape, int64_t R, int64_t C,
                                      float* dH, void* workspace, int64_t workspace_bytes, void* stream);

/*
 * Prepared operators.  The forward projection and the backprojection turn H
 * and H' into packed operand records before their matrix products (about
 * 0.35 ms each for a 165x165x15x15x21 PSF and a 600 x 600 image; 0.73 ms for
 * the 16-column forward records an operator holds).  These
 * records depend on the PSF and the image size only, so a loop that applies
 * one PSF to many volumes or images -- the Richardson-Lucy iteration of Eq. 2,
 * which uses H and H' unchanged in every update -- can pack them once into a
 * caller buffer (the "operator") and pass it to the _op calls below.  The
 * backprojection and the normaliser are bit-identical to the unprepared
 * calls.  The forward projection (also inside lfbp_rl_step_op) runs on
 * records of 16-column class boxes that only a prepared operator holds (3 x 5
 * classes in 16 matrix-core columns, which pay off once the records are
 * packed), so it agrees with lfbp_forward to float32 rounding (a different
 * summation order; both within the relative L2 bound of 1e-5 of the float64
 * result) rather than bit for bit; every call on one operator gives the same
 * bits.
 *
 * op        DEVICE buffer of lfbp_operator_size() bytes, 256-byte aligned,
 *           owned by the caller; valid while H and H' are unchanged.
 * workspace DEVICE buffer of lfbp_operator_workspace_size() bytes, 256-byte
 *           aligned, for every _op call (one per stream at a time).
 * Errors    EINVAL (NULL or short buffers, misaligned op or workspace),
 *           ESHAPE, EALIGN, EALIAS (op, workspace, inputs and outputs must be
 *           disjoint, except g_out == g in lfbp_rl_step_op), EDEVICE.  None
 *           of these calls allocates.
 */
LFBP_API int64_t lfbp_operator_size(lfbp_shape shape, int64_t R, int64_t C);
LFBP_API int64_t lfbp_operator_workspace_size(lfbp_shape shape, int64_t R, int64_t C);

/* Pack H (forward) and H' (backward) into op, with the forward's work table
 * (which row tile and split each workgroup takes; it depends on the shapes only). */
LFBP_API lfbp_status lfbp_operator_prepare(const float* H, const float* Ht, lfbp_shape shape, int64_t R, int64_t C,
                                           void* op, int64_t op_bytes, void* stream);

/* lfbp_forward on a prepared operator: f [R][C] = H g, g [nz][R][C]. */
LFBP_API lfbp_status lfbp_forward_op(const void* op, int64_t op_bytes, lfbp_shape shape, const float* g, int64_t R,
                                     int64_t C, float* f, void* workspace, int64_t workspace_bytes, void* stream);

/* lfbp_backward on a prepared operator: g [nz][R][C] = H' f, f [R][C]. */
LFBP_API lfbp_status lfbp_backward_op(const void* op, int64_t op_bytes, lfbp_shape shape, const float* f, int64_t R,
                                      int64_t C, float* g, void* workspace, int64_t workspace_bytes, void* stream);

/* lfbp_rl_step on a prepared operator (Eq. 2); g_out may be g. */
LFBP_API lfbp_status lfbp_rl_step_op(const void* op, int64_t op_bytes, lfbp_shape shape, const float* f, int64_t R,
                                     int64_t C, const float* g, const float* norm, float* g_out, void* workspace,
                                     int64_t workspace_bytes, void* stream);

/* The Richardson-Lucy normaliser H'1 [nz][R][C] on a prepared operator. */
LFBP_API lfbp_status lfbp_rl_norm_op(const void* op, int64_t op_bytes, lfbp_shape shape, int64_t R, int64_t C,
                                     float* norm, void* workspace, int64_t workspace_bytes, void* stream);

/* Static text for a status code (never NULL). */
LFBP_API const char* lfbp_status_string(lfbp_status s);

/* Frees every batched plan (device descriptor tables and graph executables),
 * after waiting for the launches of each that are still running.  The caller
 * must not replay afterwards a graph of its own that captured a batched call
 * of more than 16 problems: such a launch reads the plan's device table (up to
 * 16 descriptors travel in the kernel arguments and need no table). */
LFBP_API void lfbp_release_plans(void);

/* Batched plans currently held (kept, and dropped but not yet freed). */
LFBP_API int32_t lfbp_plan_count(void);

/* Library version string, e.g. "lfbp 0.1 gfx950". */
LFBP_API const char* lfbp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LFBP_H */
