// Light-field forward projection f = H g (Sec. 2.1, Eq. 1) and backprojection
// g = H' f (the bracketed operator of Eq. 2), float32 on gfx950.
//
// Forward:   f[p][q] = sum_z sum_{s,t} H[s][t][P mod nx][Q mod ny][z] g[z][P][Q],
//            P = p - s + hs, Q = q - t + ht (terms outside the image dropped).
// Backward:  g[z][P][Q] = sum_{s',t'} f[p][q] Ht[s'][t'][p mod nx][q mod ny][z],
//            p = P - s' + hs, q = Q - t' + ht.
// Sums are blocked (inner sum over one patch row, then over rows, then over
// depths) so that float32 rounding grows with the block lengths, not with the
// full number of terms.
#include <hip/hip_runtime.h>

#include "lfbp_internal.h"

namespace lfbp {

struct ProjShape {
    int ns, nt, nx, ny, nz, hs, ht, R, C;
};

__global__ void __launch_bounds__(256) k_forward_simple(const float* __restrict__ H, ProjShape sh,
                                                        const float* __restrict__ g, float* __restrict__ f)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y * blockDim.y + threadIdx.y;
    if (p >= sh.R || q >= sh.C) return;
    float total = 0.0f;
    for (int z = 0; z < sh.nz; ++z) {
        float accz = 0.0f;
        for (int s = 0; s < sh.ns; ++s) {
            const int P = p - s + sh.hs;
            if (P < 0 || P >= sh.R) continue;
            const int xm = P % sh.nx;
            float accs = 0.0f;
            const float* hrow = H + (size_t(s) * sh.nt * sh.nx + xm) * size_t(sh.ny) * sh.nz;
            const float* grow = g + (size_t(z) * sh.R + P) * sh.C;
            for (int t = 0; t < sh.nt; ++t) {
                const int Q = q - t + sh.ht;
                if (Q < 0 || Q >= sh.C) continue;
                const float hv = hrow[(size_t(t) * sh.nx * sh.ny + (Q % sh.ny)) * sh.nz + z];
                accs = fmaf(hv, grow[Q], accs);
            }
            accz += accs;
        }
        total += accz;
    }
    f[size_t(p) * sh.C + q] = total;
}

__global__ void __launch_bounds__(256) k_backward_simple(const float* __restrict__ Ht, ProjShape sh,
                                                         const float* __restrict__ f, float* __restrict__ g)
{
    const int Q = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (P >= sh.R || Q >= sh.C) return;
    float acc = 0.0f;
    for (int sp = 0; sp < sh.ns; ++sp) {
        const int p = P - sp + sh.hs;
        if (p < 0 || p >= sh.R) continue;
        const int xm = p % sh.nx;
        float accs = 0.0f;
        const float* hrow = Ht + (size_t(sp) * sh.nt * sh.nx + xm) * size_t(sh.ny) * sh.nz;
        const float* frow = f + size_t(p) * sh.C;
        for (int tp = 0; tp < sh.nt; ++tp) {
            const int q = Q - tp + sh.ht;
            if (q < 0 || q >= sh.C) continue;
            const float hv = hrow[(size_t(tp) * sh.nx * sh.ny + (q % sh.ny)) * sh.nz + z];
            accs = fmaf(hv, frow[q], accs);
        }
        acc += accs;
    }
    g[(size_t(z) * sh.R + P) * sh.C + Q] = acc;
}

static ProjShape proj_shape(const lfbp_shape& s, int64_t R, int64_t C)
{
    ProjShape p;
    p.ns = int(s.ns);
    p.nt = int(s.nt);
    p.nx = int(s.nx);
    p.ny = int(s.ny);
    p.nz = int(s.nz);
    p.hs = (p.ns - 1) / 2;
    p.ht = (p.nt - 1) / 2;
    p.R = int(R);
    p.C = int(C);
    return p;
}

hipError_t project_init(int max_lds)
{
    (void)max_lds;
    return hipSuccess;
}

hipError_t launch_forward(const float* H, const lfbp_shape& s, const float* g, int64_t R, int64_t C, float* f,
                          hipStream_t stream)
{
    const ProjShape sh = proj_shape(s, R, C);
    const dim3 block(64, 4);
    const dim3 grid(unsigned((C + 63) / 64), unsigned((R + 3) / 4));
    hipLaunchKernelGGL(k_forward_simple, grid, block, 0, stream, H, sh, g, f);
    return hipGetLastError();
}

hipError_t launch_backward(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                           hipStream_t stream)
{
    const ProjShape sh = proj_shape(s, R, C);
    const dim3 block(64, 4);
    const dim3 grid(unsigned((C + 63) / 64), unsigned((R + 3) / 4), unsigned(s.nz));
    hipLaunchKernelGGL(k_backward_simple, grid, block, 0, stream, Ht, sh, f, g);
    return hipGetLastError();
}

}  // namespace lfbp
