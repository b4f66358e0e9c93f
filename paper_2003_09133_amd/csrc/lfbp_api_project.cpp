// C ABI of the projector pair: f = H g and g = H' f (argument checks, workspace
// handling, launches).  The kernels are in lfbp_project.hip.
#include <hip/hip_runtime.h>

#include <initializer_list>
#include <utility>

#include "lfbp.h"
#include "lfbp_validate.h"

namespace lfbp {

hipError_t ensure_init();
size_t forward_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C);
size_t backward_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C);
hipError_t launch_forward(const float* H, const lfbp_shape& s, const float* g, int64_t R, int64_t C, float* f,
                          hipStream_t stream);
hipError_t launch_backward(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                           hipStream_t stream);
hipError_t launch_forward_ws(const float* H, const lfbp_shape& s, const float* gin, int64_t R, int64_t C, float* f,
                             void* ws, hipStream_t stream);
hipError_t launch_backward_ws(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                              void* ws, hipStream_t stream);
size_t rl_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C);
hipError_t launch_rl_step(const float* H, const float* Ht, const lfbp_shape& s, const float* fmeas, int64_t R,
                          int64_t C, const float* g, const float* norm, float* g_out, hipStream_t stream);
hipError_t launch_rl_step_ws(const float* H, const float* Ht, const lfbp_shape& s, const float* fmeas, int64_t R,
                             int64_t C, const float* g, const float* norm, float* g_out, void* ws,
                             hipStream_t stream);
hipError_t launch_rl_norm_ws(const float* Ht, const lfbp_shape& s, int64_t R, int64_t C, float* norm, void* ws,
                             hipStream_t stream);
size_t grad_psf_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C);
hipError_t launch_grad_psf(const float* w, const float* gv, const lfbp_shape& s, int64_t R, int64_t C, float* dH,
                           hipStream_t stream);
hipError_t launch_grad_psf_ws(const float* w, const float* gv, const lfbp_shape& s, int64_t R, int64_t C, float* dH,
                              void* ws, hipStream_t stream);

size_t operator_bytes(const lfbp_shape& s, int64_t R, int64_t C);
size_t operator_workspace_bytes(const lfbp_shape& s, int64_t R, int64_t C);
hipError_t launch_operator_prepare(const float* H, const float* Ht, const lfbp_shape& s, int64_t R, int64_t C,
                                   void* op, hipStream_t stream);
hipError_t launch_forward_op(const void* op, const lfbp_shape& s, const float* g, int64_t R, int64_t C, float* f,
                             void* ws, hipStream_t stream);
hipError_t launch_backward_op(const void* op, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                              void* ws, hipStream_t stream);
hipError_t launch_rl_step_op(const void* op, const lfbp_shape& s, const float* fmeas, int64_t R, int64_t C,
                             const float* g, const float* norm, float* g_out, void* ws, hipStream_t stream);
hipError_t launch_rl_norm_op(const void* op, const lfbp_shape& s, int64_t R, int64_t C, float* norm, void* ws,
                             hipStream_t stream);

namespace {

typedef std::pair<const void*, uint64_t> Range;

// A prepared operator buffer (op) and a call workspace (ws): present, 256-byte
// aligned and large enough (EINVAL); data arguments present and 4-byte aligned
// (EINVAL, EALIGN); op, ws and every data range mutually disjoint except the
// pairs the caller may share (EALIAS): `outs` must not overlap anything but
// themselves, `ins` may overlap each other.
lfbp_status check_op_call(const void* op, int64_t op_bytes, const lfbp_shape& s, int64_t R, int64_t C,
                          const void* ws, int64_t ws_bytes, std::initializer_list<Range> ins,
                          std::initializer_list<Range> outs)
{
    const lfbp_status st = check_project_shape(s, R, C, kProjFwd | kProjBwd);
    if (st != LFBP_OK) return st;
    const int64_t op_need = int64_t(operator_bytes(s, R, C));
    if (!op || op_bytes < op_need || reinterpret_cast<uintptr_t>(op) % 256) return LFBP_EINVAL;
    const int64_t ws_need = int64_t(operator_workspace_bytes(s, R, C));
    if (!ws || ws_bytes < ws_need || reinterpret_cast<uintptr_t>(ws) % 256) return LFBP_EINVAL;
    for (const Range& r : ins)
        if (!r.first) return LFBP_EINVAL;
    for (const Range& r : outs)
        if (!r.first) return LFBP_EINVAL;
    for (const Range& r : ins)
        if (reinterpret_cast<uintptr_t>(r.first) % 4) return LFBP_EALIGN;
    for (const Range& r : outs)
        if (reinterpret_cast<uintptr_t>(r.first) % 4) return LFBP_EALIGN;
    if (ranges_overlap(op, uint64_t(op_need), ws, uint64_t(ws_need))) return LFBP_EALIAS;
    for (const Range& r : ins)
        if (ranges_overlap(ws, uint64_t(ws_need), r.first, r.second)) return LFBP_EALIAS;
    for (const Range& o : outs) {
        if (ranges_overlap(o.first, o.second, op, uint64_t(op_need)) ||
            ranges_overlap(o.first, o.second, ws, uint64_t(ws_need)))
            return LFBP_EALIAS;
        for (const Range& r : ins)
            if (ranges_overlap(o.first, o.second, r.first, r.second)) return LFBP_EALIAS;
    }
    return LFBP_OK;
}

lfbp_status op_status(hipError_t e) { return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE; }

}  // namespace

}  // namespace lfbp

using namespace lfbp;

extern "C" {

lfbp_status lfbp_forward(const float* H, lfbp_shape shape, const float* g, int64_t R, int64_t C, float* f,
                         void* stream)
{
    const lfbp_status st = check_project(H, shape, g, R, C, f, true);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    const hipError_t e = launch_forward(H, shape, g, R, C, f, static_cast<hipStream_t>(stream));
    if (e == hipErrorOutOfMemory) return LFBP_ENOMEM;
    return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

int64_t lfbp_forward_workspace_size(lfbp_shape shape, int64_t R, int64_t C)
{
    if (check_project_shape(shape, R, C, kProjFwd) != LFBP_OK) return 0;
    return int64_t(forward_workspace_bytes(shape, R, C));
}

lfbp_status lfbp_forward_ws(const float* H, lfbp_shape shape, const float* g, int64_t R, int64_t C, float* f,
                            void* workspace, int64_t workspace_bytes, void* stream)
{
    lfbp_status st = check_project(H, shape, g, R, C, f, true);
    if (st != LFBP_OK) return st;
    const int64_t need = int64_t(forward_workspace_bytes(shape, R, C));
    if (!workspace || workspace_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256) return LFBP_EINVAL;
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz);
    if (ranges_overlap(workspace, uint64_t(need), H, shape_elems(shape) * 4) ||
        ranges_overlap(workspace, uint64_t(need), g, vol) || ranges_overlap(workspace, uint64_t(need), f, img))
        return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_forward_ws(H, shape, g, R, C, f, workspace, static_cast<hipStream_t>(stream)) == hipSuccess
               ? LFBP_OK
               : LFBP_EDEVICE;
}

lfbp_status lfbp_backward(const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C, float* g,
                          void* stream)
{
    const lfbp_status st = check_project(Ht, shape, f, R, C, g, false);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    const hipError_t e = launch_backward(Ht, shape, f, R, C, g, static_cast<hipStream_t>(stream));
    if (e == hipErrorOutOfMemory) return LFBP_ENOMEM;
    return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

int64_t lfbp_backward_workspace_size(lfbp_shape shape, int64_t R, int64_t C)
{
    if (check_project_shape(shape, R, C, kProjBwd) != LFBP_OK) return 0;
    return int64_t(backward_workspace_bytes(shape, R, C));
}

lfbp_status lfbp_backward_ws(const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C, float* g,
                             void* workspace, int64_t workspace_bytes, void* stream)
{
    lfbp_status st = check_project(Ht, shape, f, R, C, g, false);
    if (st != LFBP_OK) return st;
    const int64_t need = int64_t(backward_workspace_bytes(shape, R, C));
    if (!workspace || workspace_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256) return LFBP_EINVAL;
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz);
    if (ranges_overlap(workspace, uint64_t(need), Ht, shape_elems(shape) * 4) ||
        ranges_overlap(workspace, uint64_t(need), f, img) || ranges_overlap(workspace, uint64_t(need), g, vol))
        return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_backward_ws(Ht, shape, f, R, C, g, workspace, static_cast<hipStream_t>(stream)) == hipSuccess
               ? LFBP_OK
               : LFBP_EDEVICE;
}

lfbp_status lfbp_rl_step(const float* H, const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C,
                         const float* g, const float* norm, float* g_out, void* stream)
{
    const lfbp_status st = check_rl(H, Ht, shape, f, R, C, g, norm, g_out);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    const hipError_t e = launch_rl_step(H, Ht, shape, f, R, C, g, norm, g_out, static_cast<hipStream_t>(stream));
    if (e == hipErrorOutOfMemory) return LFBP_ENOMEM;
    return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

int64_t lfbp_rl_workspace_size(lfbp_shape shape, int64_t R, int64_t C)
{
    if (check_project_shape(shape, R, C, kProjFwd | kProjBwd) != LFBP_OK) return 0;
    return int64_t(rl_workspace_bytes(shape, R, C));
}

lfbp_status lfbp_rl_step_ws(const float* H, const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C,
                            const float* g, const float* norm, float* g_out, void* workspace, int64_t workspace_bytes,
                            void* stream)
{
    const lfbp_status st = check_rl(H, Ht, shape, f, R, C, g, norm, g_out);
    if (st != LFBP_OK) return st;
    const int64_t need = int64_t(rl_workspace_bytes(shape, R, C));
    if (!workspace || workspace_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256) return LFBP_EINVAL;
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz), psf = shape_elems(shape) * 4;
    for (const std::pair<const void*, uint64_t>& r : {std::pair<const void*, uint64_t>(H, psf), {Ht, psf}, {f, img},
                                                      {g, vol}, {norm, vol}, {g_out, vol}})
        if (ranges_overlap(workspace, uint64_t(need), r.first, r.second)) return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_rl_step_ws(H, Ht, shape, f, R, C, g, norm, g_out, workspace, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? LFBP_OK
               : LFBP_EDEVICE;
}

lfbp_status lfbp_rl_norm_ws(const float* Ht, lfbp_shape shape, int64_t R, int64_t C, float* norm, void* workspace,
                            int64_t workspace_bytes, void* stream)
{
    if (!Ht || !norm) return LFBP_EINVAL;
    const lfbp_status st = check_project_shape(shape, R, C, kProjBwd);
    if (st != LFBP_OK) return st;
    if (reinterpret_cast<uintptr_t>(Ht) % 4 || reinterpret_cast<uintptr_t>(norm) % 4) return LFBP_EALIGN;
    const uint64_t vol = uint64_t(R) * uint64_t(C) * uint64_t(shape.nz) * 4, psf = shape_elems(shape) * 4;
    if (ranges_overlap(norm, vol, Ht, psf)) return LFBP_EALIAS;
    const int64_t need = int64_t(rl_workspace_bytes(shape, R, C));
    if (!workspace || workspace_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256) return LFBP_EINVAL;
    if (ranges_overlap(workspace, uint64_t(need), Ht, psf) || ranges_overlap(workspace, uint64_t(need), norm, vol))
        return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_rl_norm_ws(Ht, shape, R, C, norm, workspace, static_cast<hipStream_t>(stream)) == hipSuccess
               ? LFBP_OK
               : LFBP_EDEVICE;
}

lfbp_status lfbp_grad_psf(const float* w, const float* g, lfbp_shape shape, int64_t R, int64_t C, float* dH,
                          void* stream)
{
    const lfbp_status st = check_grad_psf(w, g, shape, R, C, dH);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    const hipError_t e = launch_grad_psf(w, g, shape, R, C, dH, static_cast<hipStream_t>(stream));
    if (e == hipErrorOutOfMemory) return LFBP_ENOMEM;
    return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

int64_t lfbp_grad_psf_workspace_size(lfbp_shape shape, int64_t R, int64_t C)
{
    if (check_project_shape(shape, R, C, kProjGrad) != LFBP_OK) return 0;
    return int64_t(grad_psf_workspace_bytes(shape, R, C));
}

lfbp_status lfbp_grad_psf_ws(const float* w, const float* g, lfbp_shape shape, int64_t R, int64_t C, float* dH,
                             void* workspace, int64_t workspace_bytes, void* stream)
{
    const lfbp_status st = check_grad_psf(w, g, shape, R, C, dH);
    if (st != LFBP_OK) return st;
    const int64_t need = int64_t(grad_psf_workspace_bytes(shape, R, C));
    if (!workspace || workspace_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256) return LFBP_EINVAL;
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz), psf = shape_elems(shape) * 4;
    if (ranges_overlap(workspace, uint64_t(need), w, img) || ranges_overlap(workspace, uint64_t(need), g, vol) ||
        ranges_overlap(workspace, uint64_t(need), dH, psf))
        return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_grad_psf_ws(w, g, shape, R, C, dH, workspace, static_cast<hipStream_t>(stream)) == hipSuccess
               ? LFBP_OK
               : LFBP_EDEVICE;
}

int64_t lfbp_operator_size(lfbp_shape shape, int64_t R, int64_t C)
{
    if (check_project_shape(shape, R, C, kProjFwd | kProjBwd) != LFBP_OK) return 0;
    return int64_t(operator_bytes(shape, R, C));
}

int64_t lfbp_operator_workspace_size(lfbp_shape shape, int64_t R, int64_t C)
{
    if (check_project_shape(shape, R, C, kProjFwd | kProjBwd) != LFBP_OK) return 0;
    return int64_t(operator_workspace_bytes(shape, R, C));
}

lfbp_status lfbp_operator_prepare(const float* H, const float* Ht, lfbp_shape shape, int64_t R, int64_t C, void* op,
                                  int64_t op_bytes, void* stream)
{
    if (!H || !Ht) return LFBP_EINVAL;
    const lfbp_status st = check_project_shape(shape, R, C, kProjFwd | kProjBwd);
    if (st != LFBP_OK) return st;
    const int64_t need = int64_t(operator_bytes(shape, R, C));
    if (!op || op_bytes < need || reinterpret_cast<uintptr_t>(op) % 256) return LFBP_EINVAL;
    if (reinterpret_cast<uintptr_t>(H) % 4 || reinterpret_cast<uintptr_t>(Ht) % 4) return LFBP_EALIGN;
    const uint64_t psf = shape_elems(shape) * 4;
    if (ranges_overlap(op, uint64_t(need), H, psf) || ranges_overlap(op, uint64_t(need), Ht, psf)) return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return op_status(launch_operator_prepare(H, Ht, shape, R, C, op, static_cast<hipStream_t>(stream)));
}

lfbp_status lfbp_forward_op(const void* op, int64_t op_bytes, lfbp_shape shape, const float* g, int64_t R, int64_t C,
                            float* f, void* workspace, int64_t workspace_bytes, void* stream)
{
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz > 0 ? shape.nz : 0);
    const lfbp_status st =
        check_op_call(op, op_bytes, shape, R, C, workspace, workspace_bytes, {Range(g, vol)}, {Range(f, img)});
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return op_status(launch_forward_op(op, shape, g, R, C, f, workspace, static_cast<hipStream_t>(stream)));
}

lfbp_status lfbp_backward_op(const void* op, int64_t op_bytes, lfbp_shape shape, const float* f, int64_t R, int64_t C,
                             float* g, void* workspace, int64_t workspace_bytes, void* stream)
{
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz > 0 ? shape.nz : 0);
    const lfbp_status st =
        check_op_call(op, op_bytes, shape, R, C, workspace, workspace_bytes, {Range(f, img)}, {Range(g, vol)});
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return op_status(launch_backward_op(op, shape, f, R, C, g, workspace, static_cast<hipStream_t>(stream)));
}

lfbp_status lfbp_rl_step_op(const void* op, int64_t op_bytes, lfbp_shape shape, const float* f, int64_t R, int64_t C,
                            const float* g, const float* norm, float* g_out, void* workspace, int64_t workspace_bytes,
                            void* stream)
{
    const uint64_t img = uint64_t(R) * uint64_t(C) * 4, vol = img * uint64_t(shape.nz > 0 ? shape.nz : 0);
    // g_out may be g itself (an in-place update) or apart from it
    const lfbp_status st =
        g_out == g ? check_op_call(op, op_bytes, shape, R, C, workspace, workspace_bytes,
                                   {Range(f, img), Range(norm, vol)}, {Range(g_out, vol)})
                   : check_op_call(op, op_bytes, shape, R, C, workspace, workspace_bytes,
                                   {Range(f, img), Range(g, vol), Range(norm, vol)}, {Range(g_out, vol)});
    if (st != LFBP_OK) return st;
    if (g_out == g && ranges_overlap(workspace, uint64_t(operator_workspace_bytes(shape, R, C)), g, vol))
        return LFBP_EALIAS;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return op_status(
        launch_rl_step_op(op, shape, f, R, C, g, norm, g_out, workspace, static_cast<hipStream_t>(stream)));
}

lfbp_status lfbp_rl_norm_op(const void* op, int64_t op_bytes, lfbp_shape shape, int64_t R, int64_t C, float* norm,
                            void* workspace, int64_t workspace_bytes, void* stream)
{
    const uint64_t vol = uint64_t(R) * uint64_t(C) * 4 * uint64_t(shape.nz > 0 ? shape.nz : 0);
    const lfbp_status st =
        check_op_call(op, op_bytes, shape, R, C, workspace, workspace_bytes, {}, {Range(norm, vol)});
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return op_status(launch_rl_norm_op(op, shape, R, C, norm, workspace, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
