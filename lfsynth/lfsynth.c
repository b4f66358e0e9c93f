/*
 * lfsynth: seeded synthetic inputs for light-field PSF arrays.
 *
 * This module produces input data only.  It holds no part of the
 * H -> H' re-arrangement, of the forward model or of its adjoint, so both the
 * HIP library's tests and the CPU oracle's tests may draw their inputs from it.
 *
 * Random numbers come from the SplitMix64 output function (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), applied to
 * (linear index + seed * golden-ratio increment), so every element is a pure
 * function of (seed, index) and generation is order-independent.
 *
 * Arrays are row-major with the last axis fastest.  A PSF array H has axes
 * [ns][nt][nx][ny][nz]: patch row, patch column, source row and source column
 * inside the elementary cell, depth.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* 64-bit word number idx of stream seed. */
uint64_t lfsynth_word(uint64_t seed, uint64_t idx) { return mix64(idx + seed * GOLDEN); }

/* Uniform on [0,1) with 24 random bits: exactly representable in float32. */
static inline double unit24(uint64_t seed, uint64_t idx)
{
    return (double)(mix64(idx + seed * GOLDEN) >> 40) * 0x1p-24;
}

static int threads_or_default(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

/*
 * Gaussian-envelope PSF patterns times uniform noise, with small entries cut:
 *   v = exp(-((s-cs)^2 + (t-ct)^2) / (2 sig(z)^2)) * u(seed, idx)
 *   cs = hs + (a - hx),  ct = ht + (b - hy)       (pattern follows its source)
 *   sig(z) = sig0 + slope * |z - zc|
 * and v is set to 0 where v < thr * max(v).  hs = (ns-1)/2 etc.
 * Writes float32 values to out (ns*nt*nx*ny*nz entries).  Returns the number
 * of zero entries; *vmax receives the maximum before the cut.
 */
int64_t lfsynth_gauss_f32(int64_t ns, int64_t nt, int64_t nx, int64_t ny, int64_t nz,
                          double sig0, double slope, double zc, uint64_t seed, double thr,
                          float* out, double* vmax, int nthreads)
{
    const int nth = threads_or_default(nthreads);
    const double hs = (double)((ns - 1) / 2), ht = (double)((nt - 1) / 2);
    const double hx = (double)((nx - 1) / 2), hy = (double)((ny - 1) / 2);
    const int64_t inner = nx * ny * nz;
    float m = 0.0f;
#pragma omp parallel for num_threads(nth) schedule(static) reduction(max : m)
    for (int64_t st = 0; st < ns * nt; ++st) {
        const int64_t s = st / nt, t = st % nt;
        float* row = out + st * inner;
        for (int64_t a = 0; a < nx; ++a)
            for (int64_t b = 0; b < ny; ++b)
                for (int64_t z = 0; z < nz; ++z) {
                    const double sig = sig0 + slope * fabs((double)z - zc);
                    const double ds = (double)s - (hs + (double)a - hx);
                    const double dt = (double)t - (ht + (double)b - hy);
                    const int64_t k = (a * ny + b) * nz + z;
                    const uint64_t idx = (uint64_t)(st * inner + k);
                    const float v = (float)(exp(-(ds * ds + dt * dt) / (2.0 * sig * sig)) * unit24(seed, idx));
                    row[k] = v;
                    if (v > m) m = v;
                }
    }
    const float cut = (float)(thr * (double)m);
    int64_t zeros = 0;
    const int64_t n = ns * nt * inner;
#pragma omp parallel for num_threads(nth) schedule(static) reduction(+ : zeros)
    for (int64_t i = 0; i < n; ++i) {
        if (out[i] < cut) out[i] = 0.0f;
        if (out[i] == 0.0f) ++zeros;
    }
    if (vmax) *vmax = (double)m;
    return zeros;
}

/* Special 32-bit payloads that must survive a pure re-arrangement unchanged:
 * +0, -0, +inf, -inf, quiet and signalling NaNs with payloads, smallest and
 * largest denormals, smallest normal. */
static const uint32_t SPECIAL32[] = {0x00000000u, 0x80000000u, 0x7f800000u, 0xff800000u,
                                     0x7fc00001u, 0x7f800001u, 0xffbfffffu, 0x00000001u,
                                     0x007fffffu, 0x80000001u, 0x00800000u};
static const uint16_t SPECIAL16[] = {0x0000u, 0x8000u, 0x7c00u, 0xfc00u, 0x7e01u,
                                     0x7c01u, 0xfdffu, 0x0001u, 0x03ffu, 0x8001u, 0x0400u};

/* Random 32-bit payloads; every 97th element is one of the special payloads. */
void lfsynth_bits_u32(int64_t n, uint64_t seed, uint32_t* out, int nthreads)
{
    const int nth = threads_or_default(nthreads);
    const int nsp = (int)(sizeof(SPECIAL32) / sizeof(SPECIAL32[0]));
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t w = mix64((uint64_t)i + seed * GOLDEN);
        out[i] = (i % 97 == 13) ? SPECIAL32[(w >> 60) % nsp] : (uint32_t)(w >> 32);
    }
}

/* Random 16-bit payloads; every 97th element is one of the special payloads. */
void lfsynth_bits_u16(int64_t n, uint64_t seed, uint16_t* out, int nthreads)
{
    const int nth = threads_or_default(nthreads);
    const int nsp = (int)(sizeof(SPECIAL16) / sizeof(SPECIAL16[0]));
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t w = mix64((uint64_t)i + seed * GOLDEN);
        out[i] = (i % 97 == 13) ? SPECIAL16[(w >> 60) % nsp] : (uint16_t)(w >> 48);
    }
}

/* Uniform [0,1) float32 values (24 random bits each). */
void lfsynth_uniform_f32(int64_t n, uint64_t seed, float* out, int nthreads)
{
    const int nth = threads_or_default(nthreads);
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = (float)unit24(seed, (uint64_t)i);
}

/* Small non-negative integers 0..k-1 as float32 (exact sums in float64). */
void lfsynth_small_int_f32(int64_t n, uint64_t seed, int32_t k, float* out, int nthreads)
{
    const int nth = threads_or_default(nthreads);
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = (float)(mix64((uint64_t)i + seed * GOLDEN) % (uint64_t)k);
}
