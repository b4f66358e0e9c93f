/* Runs the oracle's entry points on small shapes under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py with gcc):
 * every read and write stays inside its array, no arithmetic is undefined,
 * and the dense, row-wise and sampled forms agree.  Exit status 0 on
 * success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_A_dense(const void* H, int esize, const int64_t* dims, int64_t R, int64_t C, void* A);
int oracle_Ht_dense(const void* H, int esize, const int64_t* dims, void* Ht);
int oracle_Ht_rows(const void* H, int esize, const int64_t* dims, void* Ht, int nthreads);
int oracle_Ht_at(const void* H, int esize, const int64_t* dims, const int64_t* idx, int64_t n, void* out,
                 int nthreads);
int oracle_forward(const float* H, const int64_t* dims, const float* g, int64_t R, int64_t C, double* f,
                   int nthreads);
int oracle_forward_at(const float* H, const int64_t* dims, const float* g, int64_t R, int64_t C,
                      const int64_t* pix, int64_t n, double* out, int nthreads);
int oracle_backward(const float* H, const int64_t* dims, const float* f, int64_t R, int64_t C, double* g,
                    int nthreads);
int oracle_backward_at(const float* H, const int64_t* dims, const float* f, int64_t R, int64_t C,
                       const int64_t* vox, int64_t n, double* out, int nthreads);
int oracle_grad_psf(const int64_t* dims, const float* w, const float* g, int64_t R, int64_t C, double* dH,
                    int nthreads);
int oracle_grad_psf_at(const int64_t* dims, const float* w, const float* g, int64_t R, int64_t C, const int64_t* idx,
                       int64_t n, double* out, int nthreads);

static uint64_t state = 88172645463325252ull;
static uint32_t next_u32(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)(state >> 16);
}
static float next_f(void) { return (float)(next_u32() & 0xFFFF) / 65536.0f; }

static int fail(const char* what, const int64_t* d)
{
    fprintf(stderr, "%s failed for [%lld %lld %lld %lld %lld]\n", what, (long long)d[0], (long long)d[1],
            (long long)d[2], (long long)d[3], (long long)d[4]);
    return 1;
}

static int close_enough(double a, double b) { return fabs(a - b) <= 1e-9 * (1.0 + fabs(a) + fabs(b)); }

static int one_shape(const int64_t* d, int64_t R, int64_t C)
{
    const int64_t E = d[0] * d[1] * d[2] * d[3] * d[4];
    float* H = malloc(sizeof(float) * E);
    uint32_t* Hd = malloc(4 * E);
    uint32_t* Hr = malloc(4 * E);
    for (int64_t i = 0; i < E; ++i) H[i] = next_f();
    if (oracle_Ht_dense(H, 4, d, Hd) != 0) return fail("Ht_dense", d);
    if (oracle_Ht_rows(H, 4, d, Hr, 2) != 0) return fail("Ht_rows", d);
    if (memcmp(Hd, Hr, 4 * E) != 0) return fail("dense == rows", d);
    int64_t idx[7] = {0, E - 1, E / 2, E / 3, 1 % E, (E * 5) / 7, E - 2 >= 0 ? E - 2 : 0};
    uint32_t at[7];
    if (oracle_Ht_at(H, 4, d, idx, 7, at, 2) != 0) return fail("Ht_at", d);
    for (int k = 0; k < 7; ++k)
        if (at[k] != Hr[idx[k]]) return fail("Ht_at == rows", d);
    /* the dense matrix itself, on a small grid */
    const int64_t nz = d[4], npix = R * C, nvox = nz * R * C;
    uint32_t* A = malloc(4 * npix * nvox);
    if (oracle_A_dense(H, 4, d, R, C, A) != 0) return fail("A_dense", d);
    /* projectors: full against sampled, and the gradient */
    float* g = malloc(sizeof(float) * nvox);
    float* f = malloc(sizeof(float) * npix);
    for (int64_t i = 0; i < nvox; ++i) g[i] = next_f();
    for (int64_t i = 0; i < npix; ++i) f[i] = next_f();
    double* fo = malloc(sizeof(double) * npix);
    double* go = malloc(sizeof(double) * nvox);
    double* dH = malloc(sizeof(double) * E);
    if (oracle_forward(H, d, g, R, C, fo, 2) != 0) return fail("forward", d);
    if (oracle_backward(H, d, f, R, C, go, 2) != 0) return fail("backward", d);
    if (oracle_grad_psf(d, f, g, R, C, dH, 2) != 0) return fail("grad_psf", d);
    int64_t pix[4] = {0, 0, R - 1, C - 1};
    double fa[2];
    if (oracle_forward_at(H, d, g, R, C, pix, 2, fa, 2) != 0) return fail("forward_at", d);
    if (!close_enough(fa[0], fo[0]) || !close_enough(fa[1], fo[npix - 1])) return fail("forward_at == forward", d);
    int64_t vox[6] = {0, 0, 0, nz - 1, R - 1, C - 1};
    double ga[2];
    if (oracle_backward_at(H, d, f, R, C, vox, 2, ga, 2) != 0) return fail("backward_at", d);
    if (!close_enough(ga[0], go[0]) || !close_enough(ga[1], go[nvox - 1])) return fail("backward_at == backward", d);
    int64_t hi[2] = {0, E - 1};
    double da[2];
    if (oracle_grad_psf_at(d, f, g, R, C, hi, 2, da, 2) != 0) return fail("grad_psf_at", d);
    if (!close_enough(da[0], dH[0]) || !close_enough(da[1], dH[E - 1])) return fail("grad_psf_at == grad_psf", d);
    /* adjoint identity <A g, f> = <g, A' f> in float64 */
    double lhs = 0, rhs = 0;
    for (int64_t i = 0; i < npix; ++i) lhs += fo[i] * f[i];
    for (int64_t i = 0; i < nvox; ++i) rhs += go[i] * g[i];
    if (fabs(lhs - rhs) > 1e-9 * (fabs(lhs) + 1.0)) return fail("adjoint identity", d);
    free(H); free(Hd); free(Hr); free(A); free(g); free(f); free(fo); free(go); free(dH);
    return 0;
}

int main(void)
{
    static const int64_t shapes[][7] = {
        /* ns, nt, nx, ny, nz, R, C */
        {15, 15, 3, 3, 3, 9, 12}, {9, 7, 3, 5, 2, 7, 11}, {3, 5, 5, 3, 1, 6, 4}, {1, 1, 1, 1, 2, 3, 3},
        {11, 7, 1, 1, 2, 5, 4},   {5, 5, 9, 1, 3, 10, 3}, {1, 3, 1, 1, 1, 1, 2}, {7, 9, 3, 3, 4, 4, 5},
    };
    int bad = 0;
    for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i) bad |= one_shape(shapes[i], shapes[i][5], shapes[i][6]);
    if (!bad) printf("oracle harness: all shapes passed\n");
    return bad;
}
