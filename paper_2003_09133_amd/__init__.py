"""Light-field backprojection arrays on AMD Instinct MI355X (gfx950).

Python binding of liblfbp.so.  Every function here only marshals arguments
(device pointers, shapes, the current HIP stream) into the C ABI of
include/lfbp.h; all computation runs in the library's HIP kernels.  PyTorch
provides device memory and streams.

    compute_Ht(H)              H' from H by pure re-arrangement (Sec. 4)
    compute_Ht_batched([H..])  many PSF arrays in one persistent launch (BatchedHt: prepared once)
    compute_Ht_inplace(H)      H' written over H (the map is its own inverse)
    compute_Ht_colmajor(H)     H' of a column-major (Matlab order) H
    forward(H, g)              f = H g (Sec. 2.1, Eq. 1)
    backward(Ht, f)            g = H' f (Eq. 2, backprojection)
    LFProject, project         torch.autograd.Function: forward by H, gradients by H' (g) and grad_psf (H)
    grad_psf(w, g, shape)      d<w, H g>/dH
    rl_step(H, Ht, f, g, norm) one Richardson-Lucy update (Eq. 2); richardson_lucy(H, f, n)
    LFOperator(H, R, C)        H and H' packed once for many projections or updates
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from ._abi import (F16, F32, GATHER_AUTO, GATHER_DIRECT, GATHER_STAGED, GATHER_WIDE, GatherConfig,
                   LfbpError, Problem, Shape)

__all__ = ["compute_Ht", "compute_Ht_into", "compute_Ht_inplace", "compute_Ht_colmajor", "compute_Ht_batched",
           "BatchedHt", "forward", "forward_workspace_size", "backward", "backward_workspace_size", "grad_psf",
           "grad_psf_workspace_size", "LFProject", "project", "rl_norm", "rl_step", "rl_workspace_size",
           "richardson_lucy", "LFOperator", "default_config", "GatherConfig", "LfbpError", "release_plans", "plan_count",
           "version", "GATHER_AUTO", "GATHER_DIRECT", "GATHER_STAGED", "GATHER_WIDE"]

_DTYPES = {torch.float32: F32, torch.float16: F16}


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_device(t: torch.Tensor, name: str):
    # The library launches on the current device's stream with raw pointers,
    # so a tensor of another device would be read through the wrong mapping.
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} lives on {t.device}, not on the current device cuda:{torch.cuda.current_device()}")


def _check_psf(H: torch.Tensor, name: str = "H"):
    if not isinstance(H, torch.Tensor) or H.dim() != 5:
        raise ValueError(f"{name} must be a 5-D tensor [ns, nt, nx, ny, nz]")
    if not H.is_cuda:
        raise ValueError(f"{name} must live on a GPU")
    _check_device(H, name)
    if not H.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major, depth fastest)")
    if H.dtype not in _DTYPES:
        raise TypeError(f"{name} must be float32 or float16, got {H.dtype}")


def _config(cfg) -> GatherConfig | None:
    if cfg is None:
        return None
    if isinstance(cfg, GatherConfig):
        return cfg
    c = GatherConfig()
    for k, v in dict(cfg).items():
        setattr(c, k, int(v))
    return c


def compute_Ht_into(H: torch.Tensor, Ht: torch.Tensor, config=None, stream=None) -> torch.Tensor:
    """Write H' of H into the preallocated tensor Ht (same shape and dtype)."""
    _check_psf(H)
    _check_psf(Ht, "Ht")
    if Ht.shape != H.shape or Ht.dtype != H.dtype:
        raise ValueError("Ht must have the shape and dtype of H")
    cfg = _config(config)
    L = _abi.lib()
    if cfg is None:
        st = L.lfbp_compute_Ht(H.data_ptr(), Ht.data_ptr(), Shape.of(H.shape), _DTYPES[H.dtype],
                               _stream(stream))
    else:
        st = L.lfbp_compute_Ht_config(H.data_ptr(), Ht.data_ptr(), Shape.of(H.shape), _DTYPES[H.dtype],
                                      ctypes.byref(cfg), _stream(stream))
    _abi.check(st, "lfbp_compute_Ht")
    return Ht


def compute_Ht(H: torch.Tensor, config=None, stream=None) -> torch.Tensor:
    """H' of H (Sec. 4): a new tensor of the same shape and dtype."""
    _check_psf(H)
    return compute_Ht_into(H, torch.empty_like(H), config, stream)


def compute_Ht_inplace(H: torch.Tensor, stream=None) -> torch.Tensor:
    """Overwrite H with H' (the map is its own inverse: a second call restores
    H).  Returns H."""
    _check_psf(H, "H")
    _abi.check(_abi.lib().lfbp_compute_Ht_inplace(H.data_ptr(), Shape.of(H.shape), _DTYPES[H.dtype],
                                                  _stream(stream)), "lfbp_compute_Ht_inplace")
    return H


def _is_colmajor(H: torch.Tensor) -> bool:
    """5-D tensor whose storage is dense with the FIRST index fastest."""
    expect, st = 1, []
    for n in H.shape:
        st.append(expect)
        expect *= n
    return all(n == 1 or s == e for n, s, e in zip(H.shape, H.stride(), st))


def compute_Ht_colmajor(H: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """H' (Sec. 4) of a column-major H of shape [ns, nt, nx, ny, nz] (s
    fastest in memory, the layout of Matlab arrays; e.g. the
    permute(4, 3, 2, 1, 0) view of a contiguous [nz, ny, nx, nt, ns] tensor).
    Returns H' in the same layout (a new tensor unless `out` is given)."""
    if not isinstance(H, torch.Tensor) or H.dim() != 5:
        raise ValueError("H must be a 5-D tensor [ns, nt, nx, ny, nz]")
    if not H.is_cuda:
        raise ValueError("H must live on a GPU")
    _check_device(H, "H")
    if H.dtype not in _DTYPES:
        raise TypeError(f"H must be float32 or float16, got {H.dtype}")
    if not _is_colmajor(H):
        raise ValueError("H must be column-major (s fastest): a permute(4, 3, 2, 1, 0) view of a contiguous tensor")
    if out is None:
        out = torch.empty(tuple(reversed(H.shape)), dtype=H.dtype, device=H.device).permute(4, 3, 2, 1, 0)
    elif out.shape != H.shape or out.dtype != H.dtype or not out.is_cuda or not _is_colmajor(out):
        raise ValueError("out must be a column-major GPU tensor of H's shape and dtype")
    else:
        _check_device(out, "out")
    _abi.check(_abi.lib().lfbp_compute_Ht_colmajor(H.data_ptr(), out.data_ptr(), Shape.of(H.shape),
                                                   _DTYPES[H.dtype], _stream(stream)), "lfbp_compute_Ht_colmajor")
    return out


def compute_Ht_batched(Hs, outs=None, config=None, use_graph: bool = False, stream=None):
    """H' of every tensor in Hs with one persistent kernel launch (replayed
    from a hipGraph captured with the plan when use_graph).  All tensors share
    one dtype."""
    Hs = list(Hs)
    if not Hs:
        raise ValueError("empty batch")
    for i, H in enumerate(Hs):
        _check_psf(H, f"Hs[{i}]")
    if len({H.dtype for H in Hs}) != 1:
        raise TypeError("all PSF arrays of a batch must share one dtype")
    outs = [torch.empty_like(H) for H in Hs] if outs is None else list(outs)
    if len(outs) != len(Hs):
        raise ValueError("outs must match Hs")
    for i, (H, o) in enumerate(zip(Hs, outs)):
        _check_psf(o, f"outs[{i}]")
        if o.shape != H.shape or o.dtype != H.dtype:
            raise ValueError(f"outs[{i}] must have the shape and dtype of Hs[{i}]")
    probs = (Problem * len(Hs))(*[Problem(H.data_ptr(), o.data_ptr(), Shape.of(H.shape))
                                  for H, o in zip(Hs, outs)])
    cfg = _config(config)
    L = _abi.lib()
    if cfg is None and not use_graph:
        st = L.lfbp_compute_Ht_batched(probs, len(Hs), _DTYPES[Hs[0].dtype], _stream(stream))
    else:
        st = L.lfbp_compute_Ht_batched_config(probs, len(Hs), _DTYPES[Hs[0].dtype],
                                              ctypes.byref(cfg) if cfg is not None else None,
                                              1 if use_graph else 0, _stream(stream))
    _abi.check(st, "lfbp_compute_Ht_batched")
    return outs


class BatchedHt:
    """A batch prepared once: the tensors are checked and the problem table is
    built here, so that each call costs one C call (for repeated H' builds of
    the same buffers, e.g. in a loop that refreshes the PSFs in place).
    use_graph: replay the launch from a hipGraph captured with the plan;
    config: an explicit kernel choice (dict of lfbp_gather_config fields)."""

    def __init__(self, Hs, outs=None, use_graph: bool = False, config=None):
        self.Hs = list(Hs)
        if not self.Hs:
            raise ValueError("empty batch")
        for i, H in enumerate(self.Hs):
            _check_psf(H, f"Hs[{i}]")
        if len({H.dtype for H in self.Hs}) != 1:
            raise TypeError("all PSF arrays of a batch must share one dtype")
        self.outs = [torch.empty_like(H) for H in self.Hs] if outs is None else list(outs)
        if len(self.outs) != len(self.Hs):
            raise ValueError("outs must match Hs")
        for i, (H, o) in enumerate(zip(self.Hs, self.outs)):
            _check_psf(o, f"outs[{i}]")
            if o.shape != H.shape or o.dtype != H.dtype:
                raise ValueError(f"outs[{i}] must have the shape and dtype of Hs[{i}]")
        self._probs = (Problem * len(self.Hs))(*[Problem(H.data_ptr(), o.data_ptr(), Shape.of(H.shape))
                                                 for H, o in zip(self.Hs, self.outs)])
        self._dtype = _DTYPES[self.Hs[0].dtype]
        self._graph = 1 if use_graph else 0
        self._cfg = _config(config)
        self._cfg_ref = ctypes.byref(self._cfg) if self._cfg is not None else None

    def __call__(self, stream=None):
        _abi.check(_abi.lib().lfbp_compute_Ht_batched_config(self._probs, len(self.Hs), self._dtype, self._cfg_ref,
                                                             self._graph, _stream(stream)),
                   "lfbp_compute_Ht_batched")
        return self.outs


def default_config(shape, dtype=torch.float32) -> dict:
    """The kernel configuration compute_Ht uses for this shape and dtype."""
    c = GatherConfig()
    _abi.check(_abi.lib().lfbp_default_config(Shape.of(shape), _DTYPES[dtype], ctypes.byref(c)),
               "lfbp_default_config")
    return c.as_dict()


def _check_f32(t: torch.Tensor, name: str, dim: int):
    if not isinstance(t, torch.Tensor) or t.dim() != dim:
        raise ValueError(f"{name} must be a {dim}-D tensor")
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
    _check_device(t, name)


def forward_workspace_size(shape, R: int, C: int) -> int:
    """Bytes of scratch device memory the forward projection needs."""
    return int(_abi.lib().lfbp_forward_workspace_size(Shape.of(shape), int(R), int(C)))


def forward(H: torch.Tensor, g: torch.Tensor, out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
            stream=None) -> torch.Tensor:
    """Forward projection f = H g: g [nz, R, C] -> f [R, C] (float32).
    The scratch workspace comes from torch's allocator unless given."""
    _check_f32(H, "H", 5)
    _check_f32(g, "g", 3)
    nz, R, C = g.shape
    if nz != H.shape[4]:
        raise ValueError("g must have nz depth planes")
    f = torch.empty((R, C), dtype=torch.float32, device=g.device) if out is None else out
    _check_f32(f, "out", 2)
    workspace = _workspace(workspace, forward_workspace_size(H.shape, R, C), g.device)
    _abi.check(_abi.lib().lfbp_forward_ws(H.data_ptr(), Shape.of(H.shape), g.data_ptr(), R, C, f.data_ptr(),
                                          workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                          _stream(stream)), "lfbp_forward")
    return f


def backward_workspace_size(shape, R: int, C: int) -> int:
    """Bytes of scratch device memory the backprojection needs."""
    return int(_abi.lib().lfbp_backward_workspace_size(Shape.of(shape), int(R), int(C)))


def _workspace(workspace, need, device):
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=device)
    if workspace.numel() * workspace.element_size() < need or not workspace.is_cuda:
        raise ValueError(f"workspace must be a GPU tensor of at least {need} bytes")
    _check_device(workspace, "workspace")
    return workspace


def backward(Ht: torch.Tensor, f: torch.Tensor, out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """Backprojection g = H' f: f [R, C] -> g [nz, R, C] (float32).
    The scratch workspace comes from torch's allocator unless given."""
    _check_f32(Ht, "Ht", 5)
    _check_f32(f, "f", 2)
    R, C = f.shape
    g = torch.empty((Ht.shape[4], R, C), dtype=torch.float32, device=f.device) if out is None else out
    _check_f32(g, "out", 3)
    workspace = _workspace(workspace, backward_workspace_size(Ht.shape, R, C), f.device)
    _abi.check(_abi.lib().lfbp_backward_ws(Ht.data_ptr(), Shape.of(Ht.shape), f.data_ptr(), R, C, g.data_ptr(),
                                           workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                           _stream(stream)), "lfbp_backward")
    return g


def grad_psf_workspace_size(shape, R: int, C: int) -> int:
    """Bytes of scratch device memory the gradient with respect to H needs."""
    return int(_abi.lib().lfbp_grad_psf_workspace_size(Shape.of(shape), int(R), int(C)))


def grad_psf(w: torch.Tensor, g: torch.Tensor, shape, out: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """d<w, H g>/dH for an image gradient w [R, C] and a volume g [nz, R, C]:
    a float32 array of the PSF's shape [ns, nt, nx, ny, nz]."""
    _check_f32(w, "w", 2)
    _check_f32(g, "g", 3)
    R, C = w.shape
    shape = tuple(int(v) for v in shape)
    if len(shape) != 5 or g.shape != (shape[4], R, C):
        raise ValueError("g must be [nz, R, C] for the PSF shape given")
    dH = torch.empty(shape, dtype=torch.float32, device=w.device) if out is None else out
    _check_f32(dH, "out", 5)
    workspace = _workspace(workspace, grad_psf_workspace_size(shape, R, C), w.device)
    _abi.check(_abi.lib().lfbp_grad_psf_ws(w.data_ptr(), g.data_ptr(), Shape.of(shape), R, C, dH.data_ptr(),
                                           workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                           _stream(stream)), "lfbp_grad_psf")
    return dH


class LFProject(torch.autograd.Function):
    """f = H g with the gradients g_grad = H' f_grad and, when H requires it,
    H_grad = d<f_grad, H g>/dH.

    The projector is linear in g, so its vector-Jacobian product with respect
    to g is the adjoint, which is exactly the backprojection with H' (Sec. 3);
    it is also linear in H, so the product with respect to H needs only g.
    Saved: H' and, only when H requires a gradient, g.  H' gets no gradient."""

    @staticmethod
    def forward(ctx, g, H, Ht):
        ctx.psf_shape = tuple(H.shape)
        ctx.save_for_backward(Ht, g if H.requires_grad else None)
        return forward(H, g.contiguous())

    @staticmethod
    def backward(ctx, grad_f):
        Ht, g = ctx.saved_tensors
        grad_f = grad_f.contiguous()
        grad_g = backward(Ht, grad_f) if ctx.needs_input_grad[0] else None
        grad_H = grad_psf(grad_f, g.contiguous(), ctx.psf_shape) if ctx.needs_input_grad[1] else None
        return grad_g, grad_H, None


def project(g: torch.Tensor, H: torch.Tensor, Ht: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable f = H g; H' is built on the GPU when not given."""
    if Ht is None:
        Ht = compute_Ht(H)
    return LFProject.apply(g, H, Ht)


def rl_norm(Ht: torch.Tensor, R: int, C: int, workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """H' 1: the backprojection of an all-ones R x C image, the normaliser of
    the Richardson-Lucy update (Eq. 2)."""
    _check_f32(Ht, "Ht", 5)
    norm = torch.empty((Ht.shape[4], R, C), dtype=torch.float32, device=Ht.device)
    workspace = _workspace(workspace, rl_workspace_size(Ht.shape, R, C), Ht.device)
    _abi.check(_abi.lib().lfbp_rl_norm_ws(Ht.data_ptr(), Shape.of(Ht.shape), int(R), int(C), norm.data_ptr(),
                                          workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                          _stream(stream)), "lfbp_rl_norm_ws")
    return norm


def rl_workspace_size(shape, R: int, C: int) -> int:
    """Bytes of scratch device memory one Richardson-Lucy step needs."""
    return int(_abi.lib().lfbp_rl_workspace_size(Shape.of(shape), int(R), int(C)))


def rl_step(H: torch.Tensor, Ht: torch.Tensor, f: torch.Tensor, g: torch.Tensor, norm: torch.Tensor,
            out: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """One Richardson-Lucy update g / (H' 1) * H'(f / (H g)) (Eq. 2).  out may
    be g itself (in-place update)."""
    _check_f32(H, "H", 5)
    _check_f32(Ht, "Ht", 5)
    _check_f32(f, "f", 2)
    _check_f32(g, "g", 3)
    _check_f32(norm, "norm", 3)
    R, C = f.shape
    if H.shape != Ht.shape or g.shape != (H.shape[4], R, C) or norm.shape != g.shape:
        raise ValueError("H, Ht, f, g and norm shapes do not match")
    out = torch.empty_like(g) if out is None else out
    _check_f32(out, "out", 3)
    workspace = _workspace(workspace, rl_workspace_size(H.shape, R, C), g.device)
    _abi.check(_abi.lib().lfbp_rl_step_ws(H.data_ptr(), Ht.data_ptr(), Shape.of(H.shape), f.data_ptr(), R, C,
                                          g.data_ptr(), norm.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                          workspace.numel() * workspace.element_size(), _stream(stream)),
               "lfbp_rl_step")
    return out


class LFOperator:
    """H and H' packed once for R x C images (a prepared operator): forward
    projections, backprojections and Richardson-Lucy updates on it skip the
    per-call packing of the PSF; the backprojection is bit-identical to the
    unprepared call, the forward projection (on 16-column class-box records
    only an operator holds) agrees with it to float32 rounding.  The packed
    records are copies: H and H' may be freed or changed afterwards (a changed
    PSF needs a new operator).  One workspace serves every call, so calls on
    one operator must not run concurrently on different streams."""

    def __init__(self, H: torch.Tensor, R: int, C: int, Ht: torch.Tensor | None = None, stream=None):
        _check_f32(H, "H", 5)
        Ht = compute_Ht(H, stream=stream) if Ht is None else Ht
        _check_f32(Ht, "Ht", 5)
        if Ht.shape != H.shape:
            raise ValueError("Ht must have the shape of H")
        L = _abi.lib()
        self.shape, self.R, self.C = tuple(H.shape), int(R), int(C)
        self._s = Shape.of(self.shape)
        nbytes = int(L.lfbp_operator_size(self._s, self.R, self.C))
        wbytes = int(L.lfbp_operator_workspace_size(self._s, self.R, self.C))
        if nbytes <= 0 or wbytes <= 0:
            raise ValueError(f"shape {self.shape} with a {R} x {C} image is outside the projector's limits")
        self.records = torch.empty(nbytes, dtype=torch.uint8, device=H.device)
        self.workspace = torch.empty(wbytes, dtype=torch.uint8, device=H.device)
        _abi.check(L.lfbp_operator_prepare(H.data_ptr(), Ht.data_ptr(), self._s, self.R, self.C,
                                           self.records.data_ptr(), nbytes, _stream(stream)),
                   "lfbp_operator_prepare")

    def _op(self):
        return self.records.data_ptr(), self.records.numel()

    def _ws(self):
        return self.workspace.data_ptr(), self.workspace.numel()

    def _vol(self, name, t):
        _check_f32(t, name, 3)
        if tuple(t.shape) != (self.shape[4], self.R, self.C):
            raise ValueError(f"{name} must be [nz, R, C] = {(self.shape[4], self.R, self.C)}")

    def _img(self, name, t):
        _check_f32(t, name, 2)
        if tuple(t.shape) != (self.R, self.C):
            raise ValueError(f"{name} must be [R, C] = {(self.R, self.C)}")

    def forward(self, g: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """f = H g (Eq. 1)."""
        self._vol("g", g)
        out = torch.empty((self.R, self.C), dtype=torch.float32, device=g.device) if out is None else out
        self._img("out", out)
        _abi.check(_abi.lib().lfbp_forward_op(*self._op(), self._s, g.data_ptr(), self.R, self.C, out.data_ptr(),
                                              *self._ws(), _stream(stream)), "lfbp_forward_op")
        return out

    def backward(self, f: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """g = H' f (the bracketed operator of Eq. 2)."""
        self._img("f", f)
        out = torch.empty((self.shape[4], self.R, self.C), dtype=torch.float32, device=f.device) if out is None else out
        self._vol("out", out)
        _abi.check(_abi.lib().lfbp_backward_op(*self._op(), self._s, f.data_ptr(), self.R, self.C, out.data_ptr(),
                                               *self._ws(), _stream(stream)), "lfbp_backward_op")
        return out

    def project(self, g: torch.Tensor) -> torch.Tensor:
        """Differentiable f = H g on the operator: the gradient with respect
        to g is the backprojection of the output gradient (H is fixed here;
        use project() for a gradient with respect to H)."""
        return _LFOpProject.apply(g, self)

    def rl_norm(self, stream=None) -> torch.Tensor:
        """H' 1, the normaliser of the Richardson-Lucy update."""
        norm = torch.empty((self.shape[4], self.R, self.C), dtype=torch.float32, device=self.records.device)
        _abi.check(_abi.lib().lfbp_rl_norm_op(*self._op(), self._s, self.R, self.C, norm.data_ptr(), *self._ws(),
                                              _stream(stream)), "lfbp_rl_norm_op")
        return norm

    def rl_step(self, f: torch.Tensor, g: torch.Tensor, norm: torch.Tensor, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
        """One Richardson-Lucy update (Eq. 2); out may be g itself."""
        self._img("f", f)
        self._vol("g", g)
        self._vol("norm", norm)
        out = torch.empty_like(g) if out is None else out
        self._vol("out", out)
        _abi.check(_abi.lib().lfbp_rl_step_op(*self._op(), self._s, f.data_ptr(), self.R, self.C, g.data_ptr(),
                                              norm.data_ptr(), out.data_ptr(), *self._ws(), _stream(stream)),
                   "lfbp_rl_step_op")
        return out


class _LFOpProject(torch.autograd.Function):
    """f = H g on a prepared operator, with g_grad = H' f_grad."""

    @staticmethod
    def forward(ctx, g, op):
        ctx.op = op
        return op.forward(g.contiguous())

    @staticmethod
    def backward(ctx, grad_f):
        return ctx.op.backward(grad_f.contiguous()), None


def richardson_lucy(H: torch.Tensor, f: torch.Tensor, iters: int, g0: torch.Tensor | None = None,
                    Ht: torch.Tensor | None = None) -> torch.Tensor:
    """iters Richardson-Lucy updates of a volume from the image f, starting
    from g0 (default: ones); H' is built on the GPU when not given.  H and H'
    are packed once (LFOperator) for all the updates."""
    R, C = f.shape
    op = LFOperator(H, R, C, Ht=Ht)
    norm = op.rl_norm()
    g = torch.ones((H.shape[4], R, C), dtype=torch.float32, device=f.device) if g0 is None else g0.clone()
    for _ in range(iters):
        op.rl_step(f, g, norm, out=g)
    return g


def plan_count() -> int:
    """Batched plans the library currently holds (kept, or dropped and not yet freed)."""
    return int(_abi.lib().lfbp_plan_count())


def release_plans():
    _abi.lib().lfbp_release_plans()


def version() -> str:
    return _abi.lib().lfbp_version().decode()
