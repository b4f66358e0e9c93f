/*
 * The paper's own method for H' (Sec. 4, Eq. 3 with the index relations of
 * Eqs. 4-9 and the loop structure of Fig. 10), in C, for timing on the host.
 *
 * TEST INFRASTRUCTURE ONLY.  The benchmark's CPU-baseline leg times it as
 * "the paper's method on this host" beside the oracle; the tests check it
 * against the per-axis relations and against the oracle.  The product library
 * never calls it, and it shares no code with the oracle or the product.
 *
 * Eqs. 4-9 relate, separately on each lateral axis, four 1-based indices: a
 * patch row s of H and a source slice x, and their places s' and x' in H'.
 * The slice x comes from a position alpha of the periodically extended slice
 * sequence (the nx slices of the cell plus the ns - nx slices added around
 * them, Figs. 8-9): Eq. 4 gives alpha from the loop position m, Eq. 5 wraps
 * alpha back into 1..nx.  Eq. 6 places the pair (s, alpha) at x' inside H',
 * and a pair is kept when 1 <= x' <= nx; Eq. 8 mirrors the patch row,
 * s' = ns - s + (ns mod 2), kept when s' >= 1.  The second axis (t, y, t', y';
 * Eqs. 7 and 9) works the same way with nt and ny.
 *
 * So per axis the method first lists, for every patch row, the (x, x') pairs
 * it contributes (m runs over the ns positions of the extended sequence), and
 * the copy of Eq. 3 then moves, for every patch-row pair (s, t) and every
 * combination of their listed pairs, the whole depth column H(s,t,x,y,:) to
 * H'(s',t',x',y',:) -- depth planes are independent (Sec. 4).  Arrays are
 * row-major [ns][nt][nx][ny][nz], depth fastest, so each move is one
 * contiguous block of nz values.  Entries of H' that no pair reaches are left
 * as the caller set them: with the printed loop bounds c(c+1) of the ns*nx
 * (s', x') combinations per axis are never reached (c = floor(nx/2)), all in
 * the border bands of the patch.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* floor(a / b) for b > 0 and any sign of a */
static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

/* Eq. 5: the source slice (1..n) of extended slice position alpha */
static int64_t source_slice(int64_t alpha, int64_t n)
{
    if (alpha > n) return alpha - floor_div(alpha - 1, n) * n;
    if (alpha <= 0) return alpha - floor_div(alpha - 1, n) * n;  /* + ceil((1 - alpha)/n) * n */
    return alpha;
}

/* The pairs one axis contributes: for patch row s (1..ns) with a valid mirror
 * row, cnt[s-1] pairs (x, x') at pairs[(s-1)*ns + k], 1-based; mirror[s-1] = s'
 * or 0 when Eq. 8 gives no row. */
typedef struct {
    int64_t ns;
    int64_t* mirror;
    int64_t* cnt;
    int64_t* px;   /* x  */
    int64_t* pxp;  /* x' */
} axis_pairs;

static int axis_build(axis_pairs* a, int64_t ns, int64_t nx)
{
    a->ns = ns;
    a->mirror = malloc(sizeof(int64_t) * (size_t)ns);
    a->cnt = calloc((size_t)ns, sizeof(int64_t));
    a->px = malloc(sizeof(int64_t) * (size_t)(ns * ns));
    a->pxp = malloc(sizeof(int64_t) * (size_t)(ns * ns));
    if (!a->mirror || !a->cnt || !a->px || !a->pxp) return -1;
    const int64_t shift = floor_div(ns - nx, 2);   /* floor((ns - nx) / 2), Eqs. 4 and 6 */
    const int64_t half = (nx - 1) / 2;            /* floor((nx - 1) / 2), Eq. 6 */
    for (int64_t s = 1; s <= ns; ++s) {
        const int64_t sp = ns - s + ns % 2;       /* Eq. 8 */
        a->mirror[s - 1] = sp > 0 ? sp : 0;
        if (sp <= 0) continue;
        for (int64_t m = 1; m <= ns; ++m) {
            const int64_t alpha = m - shift;                      /* Eq. 4 */
            const int64_t xp = s - nx + alpha + half - shift;     /* Eq. 6 */
            if (xp < 1 || xp > nx) continue;
            const int64_t k = a->cnt[s - 1]++;
            a->px[(s - 1) * ns + k] = source_slice(alpha, nx);    /* Eq. 5 */
            a->pxp[(s - 1) * ns + k] = xp;
        }
    }
    return 0;
}

static void axis_free(axis_pairs* a)
{
    free(a->mirror);
    free(a->cnt);
    free(a->px);
    free(a->pxp);
}

/* H' entries the paper's relations reach, written into Ht (the rest is left
 * untouched).  *columns (may be NULL) receives the number of depth columns
 * written.  Returns 0, or -1 on bad arguments or no memory. */
int paper_Ht(const void* H, int esize, const int64_t* dims, void* Ht, int nthreads, int64_t* columns)
{
    if (!H || !Ht || !dims || (esize != 2 && esize != 4)) return -1;
    const int64_t ns = dims[0], nt = dims[1], nx = dims[2], ny = dims[3], nz = dims[4];
    if (ns < 1 || nt < 1 || nx < 1 || ny < 1 || nz < 1) return -1;
    axis_pairs as, at;
    if (axis_build(&as, ns, nx) || axis_build(&at, nt, ny)) {
        axis_free(&as);
        axis_free(&at);
        return -1;
    }
    const size_t col = (size_t)nz * (size_t)esize;
    const char* src = (const char*)H;
    char* dst = (char*)Ht;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads()) \
    reduction(+ : total)
    for (int64_t s = 1; s <= ns; ++s) {
        const int64_t sp = as.mirror[s - 1];
        if (!sp) continue;
        for (int64_t t = 1; t <= nt; ++t) {
            const int64_t tp = at.mirror[t - 1];
            if (!tp) continue;
            /* the (s, t) block of H and the (s', t') block of H' */
            const char* hb = src + (size_t)(((s - 1) * nt + (t - 1)) * nx * ny) * col;
            char* tb = dst + (size_t)(((sp - 1) * nt + (tp - 1)) * nx * ny) * col;
            for (int64_t i = 0; i < as.cnt[s - 1]; ++i) {
                const int64_t x = as.px[(s - 1) * ns + i], xp = as.pxp[(s - 1) * ns + i];
                for (int64_t j = 0; j < at.cnt[t - 1]; ++j) {
                    const int64_t y = at.px[(t - 1) * nt + j], yp = at.pxp[(t - 1) * nt + j];
                    memcpy(tb + (size_t)((xp - 1) * ny + (yp - 1)) * col,
                           hb + (size_t)((x - 1) * ny + (y - 1)) * col, col);   /* Eq. 3 */
                }
            }
            total += as.cnt[s - 1] * at.cnt[t - 1];
        }
    }
    axis_free(&as);
    axis_free(&at);
    if (columns) *columns = total;
    return 0;
}
