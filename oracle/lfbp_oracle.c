/*
 * CPU oracle for the light-field backprojection array H'.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call this code; the product library never does, and the two
 * share no code, headers or tables.
 *
 * What it computes, and from which definition
 * -------------------------------------------
 * The forward model f = H g (Sec. 2.1, Eq. 1) distributes a copy of the PSF
 * pattern of every voxel, scaled by the voxel value, onto the image; the
 * pattern of a voxel is the cut-out stored in H for the source position inside
 * the elementary cell that the voxel occupies (lenslet periodicity, Sec. 2.1),
 * and the cut-out is centred on the voxel (cut-outs move with the source,
 * Sec. 2.1).  Written as a matrix, the entry linking image pixel (p,q) with
 * voxel (z,P,Q) is
 *
 *     A[(p,q),(z,P,Q)] = H[p-P+hs][q-Q+ht][P mod nx][Q mod ny][z]
 *
 * when both patch indices lie inside the patch, and 0 otherwise
 * (hs = (ns-1)/2, ht = (nt-1)/2; image and volume share the lateral grid).
 *
 * The backprojection array H' (Sec. 3, Fig. 6 discussion) collects, for one
 * image pixel, the contribution of every voxel: it is the transposed operator
 * A^T laid out in the same convolutional form as H.  Its slice for a pixel of
 * class (x',y') (position inside the lenslet) lists the voxels at offsets
 * (s'-hs, t'-ht) from that pixel:
 *
 *     H'[s'][t'][x'][y'][z] = A^T[(z, p+s'-hs, q+t'-ht), (p,q)]
 *
 * for any pixel (p,q) of class (x',y') far enough from the image border.
 * oracle_Ht_dense materialises A for a small lenslet grid, transposes it
 * explicitly and reads H' back; oracle_Ht_rows evaluates the same entries of A
 * one by one without storing A.  Neither uses the paper's index relations
 * (Eqs. 4-9): those are what the GPU path implements and what this oracle
 * checks.
 *
 * Values are moved as raw payloads of esize = 2 or 4 bytes, so NaN payloads,
 * -0 and denormals pass through unchanged, as they must for a pure
 * re-arrangement (Sec. 3: no summations are involved).
 *
 * The projectors (oracle_forward, oracle_backward) evaluate A g and A^T f in
 * float64 from H, never from H'.
 *
 * All arrays are row-major, last axis fastest: H and H' are [ns][nt][nx][ny][nz],
 * a volume g is [nz][R][C] and an image f is [R][C].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t ns, nt, nx, ny, nz;
} oshape;

static oshape mkshape(const int64_t* d)
{
    oshape s = {d[0], d[1], d[2], d[3], d[4]};
    return s;
}

static int64_t mod_nonneg(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

static int nthreads_or_default(int n) { return n > 0 ? n : omp_get_max_threads(); }

/*
 * Flat index into H of the measurement-matrix entry A[(p,q),(z,P,Q)], or -1
 * when the entry is a structural zero (the voxel's pattern does not reach the
 * pixel).  Pixel and voxel coordinates are absolute image/volume positions.
 */
static int64_t A_index(const oshape* h, int64_t p, int64_t q, int64_t z, int64_t P, int64_t Q)
{
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    const int64_t s = p - P + hs; /* patch row of pixel p in the pattern of voxel row P */
    const int64_t t = q - Q + ht;
    if (s < 0 || s >= h->ns || t < 0 || t >= h->nt) return -1;
    const int64_t x = mod_nonneg(P, h->nx); /* source position inside the cell */
    const int64_t y = mod_nonneg(Q, h->ny);
    return (((s * h->nt + t) * h->nx + x) * h->ny + y) * h->nz + z;
}

static void copy_payload(void* dst, int64_t di, const void* src, int64_t si, int esize)
{
    memcpy((char*)dst + di * esize, (const char*)src + si * esize, (size_t)esize);
}

/* Central lenslet of the smallest grid on which every voxel offset of H' seen
 * from a pixel of that lenslet stays inside the image. */
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/*
 * Dense measurement matrix on an Lr x Lc lenslet grid (R = Lr*nx rows of
 * pixels, C = Lc*ny columns).  A has R*C rows (pixel p*C+q) and nz*R*C columns
 * (voxel (z*R+P)*C+Q); each entry is an H payload or zero bits.
 */
int oracle_A_dense(const void* H, int esize, const int64_t* dims, int64_t R, int64_t C, void* A)
{
    if (esize != 2 && esize != 4) return -1;
    const oshape h = mkshape(dims);
    const int64_t ncol = h.nz * R * C;
    memset(A, 0, (size_t)(R * C * ncol * esize));
    for (int64_t p = 0; p < R; ++p)
        for (int64_t q = 0; q < C; ++q)
            for (int64_t z = 0; z < h.nz; ++z)
                for (int64_t P = 0; P < R; ++P)
                    for (int64_t Q = 0; Q < C; ++Q) {
                        const int64_t k = A_index(&h, p, q, z, P, Q);
                        if (k >= 0) copy_payload(A, (p * C + q) * ncol + (z * R + P) * C + Q, H, k, esize);
                    }
    return 0;
}

/*
 * H' by materialising A on an Lr x Lc lenslet grid, transposing it explicitly
 * and reading the slices of the pixels in lenslet (lr, lc) back out.
 * Returns 0, or -2 when a needed voxel falls outside the grid (the chosen
 * lenslet is too close to the border), or -1 for a bad element size.
 * Lr = Lc = 0 selects the smallest grid with a central lenslet that works.
 */
int oracle_Ht_dense_grid(const void* H, int esize, const int64_t* dims, int64_t Lr, int64_t Lc,
                         int64_t lr, int64_t lc, void* Ht)
{
    if (esize != 2 && esize != 4) return -1;
    const oshape h = mkshape(dims);
    const int64_t hs = (h.ns - 1) / 2, ht = (h.nt - 1) / 2;
    if (Lr <= 0 || Lc <= 0) {
        const int64_t cr = ceil_div(hs, h.nx), cc = ceil_div(ht, h.ny);
        Lr = 2 * cr + 1;
        Lc = 2 * cc + 1;
        lr = cr;
        lc = cc;
    }
    const int64_t R = Lr * h.nx, C = Lc * h.ny;
    const int64_t nrow = R * C, ncol = h.nz * R * C;
    char* A = (char*)malloc((size_t)(nrow * ncol * esize));
    char* At = (char*)malloc((size_t)(nrow * ncol * esize));
    if (!A || !At) {
        free(A);
        free(At);
        return -3;
    }
    oracle_A_dense(H, esize, dims, R, C, A);
    /* explicit transpose: At[col][row] = A[row][col] */
    for (int64_t r = 0; r < nrow; ++r)
        for (int64_t c = 0; c < ncol; ++c) copy_payload(At, c * nrow + r, A, r * ncol + c, esize);
    int rc = 0;
    for (int64_t sp = 0; sp < h.ns; ++sp)
        for (int64_t tp = 0; tp < h.nt; ++tp)
            for (int64_t xp = 0; xp < h.nx; ++xp)
                for (int64_t yp = 0; yp < h.ny; ++yp) {
                    const int64_t p = lr * h.nx + xp, q = lc * h.ny + yp; /* pixel of class (x',y') */
                    const int64_t P = p + sp - hs, Q = q + tp - ht;       /* voxel at offset (s',t') */
                    for (int64_t z = 0; z < h.nz; ++z) {
                        const int64_t out = (((sp * h.nt + tp) * h.nx + xp) * h.ny + yp) * h.nz + z;
                        if (P < 0 || P >= R || Q < 0 || Q >= C) {
                            memset((char*)Ht + out * esize, 0, (size_t)esize);
                            rc = -2;
                            continue;
                        }
                        copy_payload(Ht, out, At, ((z * R + P) * C + Q) * nrow + (p * C + q), esize);
                    }
                }
    free(A);
    free(At);
    return rc;
}

int oracle_Ht_dense(const void* H, int esize, const int64_t* dims, void* Ht)
{
    return oracle_Ht_dense_grid(H, esize, dims, 0, 0, 0, 0, Ht);
}

/* One element of H' (flat index i) from the definition, without storing A:
 * the entry of A linking the reference pixel of class (x',y') in the central
 * lenslet with the voxel at offset (s'-hs, t'-ht) from it. */
static int64_t Ht_source(const oshape* h, int64_t i)
{
    const int64_t z = i % h->nz;
    int64_t r = i / h->nz;
    const int64_t yp = r % h->ny;
    r /= h->ny;
    const int64_t xp = r % h->nx;
    r /= h->nx;
    const int64_t tp = r % h->nt;
    const int64_t sp = r / h->nt;
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    const int64_t p = ceil_div(hs, h->nx) * h->nx + xp;
    const int64_t q = ceil_div(ht, h->ny) * h->ny + yp;
    return A_index(h, p, q, z, p + sp - hs, q + tp - ht);
}

/* Full H' by evaluating the needed entries of A one by one (OpenMP over rows). */
int oracle_Ht_rows(const void* H, int esize, const int64_t* dims, void* Ht, int nthreads)
{
    if (esize != 2 && esize != 4) return -1;
    const oshape h = mkshape(dims);
    const int64_t n = h.ns * h.nt * h.nx * h.ny * h.nz;
    const int64_t per = h.nx * h.ny * h.nz;
    int bad = 0;
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(static) reduction(| : bad)
    for (int64_t st = 0; st < h.ns * h.nt; ++st)
        for (int64_t i = st * per; i < (st + 1) * per && i < n; ++i) {
            const int64_t k = Ht_source(&h, i);
            if (k < 0) {
                memset((char*)Ht + i * esize, 0, (size_t)esize);
                bad = 1;
            } else {
                copy_payload(Ht, i, H, k, esize);
            }
        }
    return bad ? -2 : 0;
}

/* Selected elements of H' (flat indices idx[0..n)), for checks at full size. */
int oracle_Ht_at(const void* H, int esize, const int64_t* dims, const int64_t* idx, int64_t n, void* out,
                 int nthreads)
{
    if (esize != 2 && esize != 4) return -1;
    const oshape h = mkshape(dims);
    int bad = 0;
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < n; ++k) {
        const int64_t src = Ht_source(&h, idx[k]);
        if (src < 0) {
            memset((char*)out + k * esize, 0, (size_t)esize);
            bad = 1;
        } else {
            copy_payload(out, k, H, src, esize);
        }
    }
    return bad ? -2 : 0;
}

/* Forward projection f = A g at one pixel, float64. */
static double forward_pixel(const oshape* h, const float* H, const float* g, int64_t R, int64_t C, int64_t p,
                            int64_t q)
{
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    double acc = 0.0;
    for (int64_t z = 0; z < h->nz; ++z)
        for (int64_t P = p - hs; P <= p + hs; ++P) {
            if (P < 0 || P >= R) continue;
            for (int64_t Q = q - ht; Q <= q + ht; ++Q) {
                if (Q < 0 || Q >= C) continue;
                const int64_t k = A_index(h, p, q, z, P, Q);
                if (k < 0) continue;
                acc += (double)H[k] * (double)g[(z * R + P) * C + Q];
            }
        }
    return acc;
}

/* Back projection A^T f at one voxel, float64, computed from H. */
static double backward_voxel(const oshape* h, const float* H, const float* f, int64_t R, int64_t C, int64_t z,
                             int64_t P, int64_t Q)
{
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    double acc = 0.0;
    for (int64_t p = P - hs; p <= P + hs; ++p) {
        if (p < 0 || p >= R) continue;
        for (int64_t q = Q - ht; q <= Q + ht; ++q) {
            if (q < 0 || q >= C) continue;
            const int64_t k = A_index(h, p, q, z, P, Q);
            if (k < 0) continue;
            acc += (double)H[k] * (double)f[p * C + q];
        }
    }
    return acc;
}

/* f[R][C] = A g for g[nz][R][C]; float64 result. */
int oracle_forward(const float* H, const int64_t* dims, const float* g, int64_t R, int64_t C, double* f,
                   int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 1)
    for (int64_t p = 0; p < R; ++p)
        for (int64_t q = 0; q < C; ++q) f[p * C + q] = forward_pixel(&h, H, g, R, C, p, q);
    return 0;
}

/* f at the listed pixels pix[2k], pix[2k+1]. */
int oracle_forward_at(const float* H, const int64_t* dims, const float* g, int64_t R, int64_t C,
                      const int64_t* pix, int64_t n, double* out, int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) out[k] = forward_pixel(&h, H, g, R, C, pix[2 * k], pix[2 * k + 1]);
    return 0;
}

/* g[nz][R][C] = A^T f for f[R][C]; float64 result, computed from H. */
int oracle_backward(const float* H, const int64_t* dims, const float* f, int64_t R, int64_t C, double* g,
                    int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 1) collapse(2)
    for (int64_t z = 0; z < h.nz; ++z)
        for (int64_t P = 0; P < R; ++P)
            for (int64_t Q = 0; Q < C; ++Q) g[(z * R + P) * C + Q] = backward_voxel(&h, H, f, R, C, z, P, Q);
    return 0;
}

/* A^T f at the listed voxels vox[3k..3k+2] = (z, P, Q). */
int oracle_backward_at(const float* H, const int64_t* dims, const float* f, int64_t R, int64_t C,
                       const int64_t* vox, int64_t n, double* out, int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k)
        out[k] = backward_voxel(&h, H, f, R, C, vox[3 * k], vox[3 * k + 1], vox[3 * k + 2]);
    return 0;
}

/* The same two projections with a float64 volume or image (the iterates of
 * the Richardson-Lucy oracle, Eq. 2, stay in float64). */
static double forward_pixel_d(const oshape* h, const float* H, const double* g, int64_t R, int64_t C, int64_t p,
                              int64_t q)
{
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    double acc = 0.0;
    for (int64_t z = 0; z < h->nz; ++z)
        for (int64_t P = p - hs; P <= p + hs; ++P) {
            if (P < 0 || P >= R) continue;
            for (int64_t Q = q - ht; Q <= q + ht; ++Q) {
                if (Q < 0 || Q >= C) continue;
                const int64_t k = A_index(h, p, q, z, P, Q);
                if (k < 0) continue;
                acc += (double)H[k] * g[(z * R + P) * C + Q];
            }
        }
    return acc;
}

static double backward_voxel_d(const oshape* h, const float* H, const double* f, int64_t R, int64_t C, int64_t z,
                               int64_t P, int64_t Q)
{
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    double acc = 0.0;
    for (int64_t p = P - hs; p <= P + hs; ++p) {
        if (p < 0 || p >= R) continue;
        for (int64_t q = Q - ht; q <= Q + ht; ++q) {
            if (q < 0 || q >= C) continue;
            const int64_t k = A_index(h, p, q, z, P, Q);
            if (k < 0) continue;
            acc += (double)H[k] * f[p * C + q];
        }
    }
    return acc;
}

int oracle_forward_d(const float* H, const int64_t* dims, const double* g, int64_t R, int64_t C, double* f,
                     int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 1)
    for (int64_t p = 0; p < R; ++p)
        for (int64_t q = 0; q < C; ++q) f[p * C + q] = forward_pixel_d(&h, H, g, R, C, p, q);
    return 0;
}

int oracle_backward_d(const float* H, const int64_t* dims, const double* f, int64_t R, int64_t C, double* g,
                      int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 1) collapse(2)
    for (int64_t z = 0; z < h.nz; ++z)
        for (int64_t P = 0; P < R; ++P)
            for (int64_t Q = 0; Q < C; ++Q) g[(z * R + P) * C + Q] = backward_voxel_d(&h, H, f, R, C, z, P, Q);
    return 0;
}

/* Gradient of <w, A g> with respect to H (the forward model is linear in H):
 * the entry H[s][t][x][y][z] links every voxel (z,P,Q) of class (x,y) with the
 * pixel (P+s-hs, Q+t-ht), so its derivative sums w at that pixel times g at the
 * voxel over all voxels of the class whose pixel lies in the image.  float64. */
static double grad_psf_entry(const oshape* h, const float* w, const float* g, int64_t R, int64_t C, int64_t s,
                             int64_t t, int64_t x, int64_t y, int64_t z)
{
    const int64_t hs = (h->ns - 1) / 2, ht = (h->nt - 1) / 2;
    double acc = 0.0;
    for (int64_t P = x; P < R; P += h->nx) {
        const int64_t p = P + s - hs;
        if (p < 0 || p >= R) continue;
        for (int64_t Q = y; Q < C; Q += h->ny) {
            const int64_t q = Q + t - ht;
            if (q < 0 || q >= C) continue;
            acc += (double)w[p * C + q] * (double)g[(z * R + P) * C + Q];
        }
    }
    return acc;
}

/*
 * The two projections again, summed over the nonzero entries of H only.  Read
 * from the H side, entry H[s][t][x][y][z] of the pattern of cell position
 * (x,y) links every voxel (z,P,Q) with P mod nx = x and Q mod ny = y to the
 * pixel (P+s-hs, Q+t-ht) when that pixel lies in the image: the same entries
 * of A as above.  A zero entry of H adds nothing to either sum, so skipping it
 * leaves A g and A^T f unchanged up to the order of the float64 additions; the
 * cost scales with the nonzeros of H, which makes full projector-sized images
 * affordable.
 */
static int64_t nonzero_entries(const oshape* h, const float* H, int64_t** idx)
{
    const int64_t E = h->ns * h->nt * h->nx * h->ny * h->nz;
    int64_t n = 0;
    for (int64_t k = 0; k < E; ++k) n += H[k] != 0.0f;
    *idx = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!*idx) return -1;
    n = 0;
    for (int64_t k = 0; k < E; ++k)
        if (H[k] != 0.0f) (*idx)[n++] = k;
    return n;
}

/* f[R][C] = A g over the nonzero entries of H; each thread sums its share of
 * the entries into an image of its own, and the images are added in thread
 * order. */
int oracle_forward_sparse(const float* H, const int64_t* dims, const float* g, int64_t R, int64_t C, double* f,
                          int nthreads)
{
    const oshape h = mkshape(dims);
    const int64_t hs = (h.ns - 1) / 2, ht = (h.nt - 1) / 2;
    int64_t* nz_idx = NULL;
    const int64_t n = nonzero_entries(&h, H, &nz_idx);
    if (n < 0) return -3;
    const int T = nthreads_or_default(nthreads);
    double* part = (double*)calloc((size_t)T * (size_t)(R * C), sizeof(double));
    if (!part) {
        free(nz_idx);
        return -3;
    }
#pragma omp parallel num_threads(T)
    {
        const int tid = omp_get_thread_num();
        double* fp = part + (size_t)tid * (size_t)(R * C);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < n; ++e) {
            int64_t k = nz_idx[e];
            const double v = (double)H[k];
            const int64_t z = k % h.nz;
            k /= h.nz;
            const int64_t y = k % h.ny;
            k /= h.ny;
            const int64_t x = k % h.nx;
            k /= h.nx;
            const int64_t t = k % h.nt;
            const int64_t s = k / h.nt;
            for (int64_t P = x; P < R; P += h.nx) {
                const int64_t p = P + s - hs;
                if (p < 0 || p >= R) continue;
                for (int64_t Q = y; Q < C; Q += h.ny) {
                    const int64_t q = Q + t - ht;
                    if (q < 0 || q >= C) continue;
                    fp[p * C + q] += v * (double)g[(z * R + P) * C + Q];
                }
            }
        }
    }
    for (int64_t i = 0; i < R * C; ++i) {
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += part[(size_t)t * (size_t)(R * C) + (size_t)i];
        f[i] = acc;
    }
    free(part);
    free(nz_idx);
    return 0;
}

/* g[nz][R][C] = A^T f over the nonzero entries of H; each depth plane is
 * summed by one thread. */
int oracle_backward_sparse(const float* H, const int64_t* dims, const float* f, int64_t R, int64_t C, double* g,
                           int nthreads)
{
    const oshape h = mkshape(dims);
    const int64_t hs = (h.ns - 1) / 2, ht = (h.nt - 1) / 2;
    int64_t* nz_idx = NULL;
    const int64_t n = nonzero_entries(&h, H, &nz_idx);
    if (n < 0) return -3;
    memset(g, 0, (size_t)(h.nz * R * C) * sizeof(double));
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 1)
    for (int64_t z = 0; z < h.nz; ++z) {
        double* gz = g + z * R * C;
        for (int64_t e = 0; e < n; ++e) {
            int64_t k = nz_idx[e];
            if (k % h.nz != z) continue;
            const double v = (double)H[k];
            k /= h.nz;
            const int64_t y = k % h.ny;
            k /= h.ny;
            const int64_t x = k % h.nx;
            k /= h.nx;
            const int64_t t = k % h.nt;
            const int64_t s = k / h.nt;
            for (int64_t P = x; P < R; P += h.nx) {
                const int64_t p = P + s - hs;
                if (p < 0 || p >= R) continue;
                for (int64_t Q = y; Q < C; Q += h.ny) {
                    const int64_t q = Q + t - ht;
                    if (q < 0 || q >= C) continue;
                    gz[P * C + Q] += v * (double)f[p * C + q];
                }
            }
        }
    }
    free(nz_idx);
    return 0;
}

int oracle_grad_psf(const int64_t* dims, const float* w, const float* g, int64_t R, int64_t C, double* dH,
                    int nthreads)
{
    const oshape h = mkshape(dims);
    const int64_t E = h.ns * h.nt * h.nx * h.ny * h.nz;
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 64)
    for (int64_t i = 0; i < E; ++i) {
        int64_t r = i;
        const int64_t z = r % h.nz; r /= h.nz;
        const int64_t y = r % h.ny; r /= h.ny;
        const int64_t x = r % h.nx; r /= h.nx;
        const int64_t t = r % h.nt, s = r / h.nt;
        dH[i] = grad_psf_entry(&h, w, g, R, C, s, t, x, y, z);
    }
    return 0;
}

/* The same at the listed flat indices of H. */
int oracle_grad_psf_at(const int64_t* dims, const float* w, const float* g, int64_t R, int64_t C, const int64_t* idx,
                       int64_t n, double* out, int nthreads)
{
    const oshape h = mkshape(dims);
#pragma omp parallel for num_threads(nthreads_or_default(nthreads)) schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        int64_t r = idx[k];
        const int64_t z = r % h.nz; r /= h.nz;
        const int64_t y = r % h.ny; r /= h.ny;
        const int64_t x = r % h.nx; r /= h.nx;
        const int64_t t = r % h.nt, s = r / h.nt;
        out[k] = grad_psf_entry(&h, w, g, R, C, s, t, x, y, z);
    }
    return 0;
}
