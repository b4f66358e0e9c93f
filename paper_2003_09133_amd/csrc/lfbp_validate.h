// Host-only argument checks of the C ABI.  No HIP header is included here:
// every check runs before the first HIP call of an entry point.
#pragma once

#include <stdint.h>

#include "lfbp.h"

namespace lfbp {

// Element size of a dtype, 0 if unknown.
int dtype_size(lfbp_dtype dt);

// Shape rules of the re-arrangement (odd ns, nt, nx, ny; all >= 1; size limits).
lfbp_status check_shape(const lfbp_shape& s, int esize);

// Full check of one lfbp_compute_Ht call.
lfbp_status check_gather(const void* H, const void* Ht, const lfbp_shape& s, lfbp_dtype dt);

// Configuration fields (0 = tuned default is always accepted).
lfbp_status check_config(const lfbp_gather_config* cfg);

// Which projector products a call runs (their launches have different sizes).
enum ProjOps : unsigned { kProjFwd = 1, kProjBwd = 2, kProjGrad = 4 };

// Shape and image size of a projection (no pointers): EINVAL for R or C < 1,
// ESHAPE for shapes outside the kernels' index ranges or, for the products
// in `ops`, the launch sizes.
lfbp_status check_project_shape(const lfbp_shape& s, int64_t R, int64_t C, unsigned ops);

// Full check of one projector call.  forward: psf = H, in2 = g [nz][R][C],
// out = f [R][C]; else psf = H', in2 = f [R][C], out = g [nz][R][C].
lfbp_status check_project(const float* psf, const lfbp_shape& s, const float* in2, int64_t R, int64_t C,
                          const float* out, bool forward);

// Full check of one Richardson-Lucy step: g_out may be g itself but must not
// overlap any other argument.
lfbp_status check_rl(const float* H, const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C,
                     const float* g, const float* norm, const float* g_out);

// Full check of one gradient-with-respect-to-H call: w [R][C], g [nz][R][C],
// dH the shape of H, not overlapping the inputs.
lfbp_status check_grad_psf(const float* w, const float* g, const lfbp_shape& s, int64_t R, int64_t C,
                           const float* dH);

// True when [a, a+na) and [b, b+nb) (bytes) overlap.
bool ranges_overlap(const void* a, uint64_t na, const void* b, uint64_t nb);

uint64_t shape_elems(const lfbp_shape& s);

}  // namespace lfbp
