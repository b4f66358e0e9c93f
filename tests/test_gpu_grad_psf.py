"""The gradient with respect to the PSF array, d<w, H g>/dH (lfbp_grad_psf and
LFProject's backward for H), against the float64 oracle: relative L2 <= 1e-5,
finite differences, autograd, and the full projector grid at sampled entries."""
import numpy as np
import pytest
import torch

import lfsynth
import oracle
import paper_2003_09133_amd as lf
from gpu_util import DEV, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


SHAPES = [((15, 15, 3, 3, 3), 21, 21), ((15, 15, 3, 3, 3), 20, 23), ((9, 7, 3, 5, 2), 12, 10),
          ((5, 5, 5, 5, 1), 7, 8), ((7, 9, 1, 1, 3), 11, 9), ((1, 1, 1, 1, 2), 4, 5), ((3, 3, 7, 7, 2), 14, 21),
          ((33, 25, 11, 5, 4), 55, 40), ((21, 21, 17, 17, 2), 40, 36), ((9, 9, 3, 3, 30), 10, 10),
          ((45, 45, 15, 15, 5), 90, 75),
          # tall images: tiles whose r reach only part of the lenslet rows skip the other rows' stages
          ((15, 15, 1, 1, 2), 40, 50), ((9, 9, 3, 3, 2), 90, 60)]


@pytest.mark.parametrize("shape,R,C", SHAPES)
def test_grad_psf_vs_oracle(shape, R, C):
    w = lfsynth.uniform_f32((R, C), 1) - np.float32(0.5)
    g = lfsynth.uniform_f32((shape[4], R, C), 2)
    dH = lf.grad_psf(to_dev(w), to_dev(g), shape)
    torch.cuda.synchronize()
    assert rel_l2(dH.cpu().numpy(), oracle.grad_psf(shape, w, g)) <= TOL


def test_autograd_and_finite_differences_in_H():
    shape, R, C = (21, 21, 5, 5, 4), 40, 45
    H = to_dev(lfsynth.uniform_f32(shape, 3))
    g = to_dev(lfsynth.uniform_f32((shape[4], R, C), 4))
    w = to_dev(lfsynth.uniform_f32((R, C), 5))
    Hr = H.clone().requires_grad_(True)
    gr = g.clone().requires_grad_(True)
    loss = torch.sum(lf.project(gr, Hr) * w)
    loss.backward()
    assert rel_l2(Hr.grad.cpu().numpy(), oracle.grad_psf(shape, w.cpu().numpy(), g.cpu().numpy())) <= TOL
    assert rel_l2(gr.grad.cpu().numpy(), oracle.backward(H.cpu().numpy(), w.cpu().numpy())) <= TOL
    grad = Hr.grad.double()
    rng = np.random.default_rng(1)
    for k in range(3):
        D = torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).to(DEV)
        lp = torch.sum(lf.forward(H + D, g).double() * w.double())     # linear in H: exact differences
        lm = torch.sum(lf.forward(H - D, g).double() * w.double())
        fd = ((lp - lm) / 2).item()
        an = torch.sum(grad * D.double()).item()
        scale = torch.sum(torch.abs(grad) * torch.abs(D.double())).item()
        assert abs(fd - an) <= 1e-5 * scale, (k, fd, an)


def test_no_gradient_for_H_unless_asked():
    shape, R, C = (9, 9, 3, 3, 2), 12, 12
    H = to_dev(lfsynth.uniform_f32(shape, 6))
    g = to_dev(lfsynth.uniform_f32((shape[4], R, C), 7)).requires_grad_(True)
    lf.project(g, H).sum().backward()
    assert H.grad is None and g.grad is not None


def test_workspace_forms_agree():
    import ctypes
    from paper_2003_09133_amd import _abi
    shape, R, C = (45, 45, 15, 15, 5), 97, 120
    w = to_dev(lfsynth.uniform_f32((R, C), 8))
    g = to_dev(lfsynth.uniform_f32((shape[4], R, C), 9))
    ref = lf.grad_psf(w, g, shape)
    out = torch.empty(shape, device=DEV)
    st = _abi.lib().lfbp_grad_psf(w.data_ptr(), g.data_ptr(), _abi.Shape.of(shape), R, C, out.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(ref, out)


def test_projector_grid_sampled():
    """The projector workload's grid and PSF shape (600 x 600 px, H[165,165,15,15,21]):
    sampled entries of dH, the patch borders included."""
    pw = lfsynth.PROJECTOR
    shape = pw.psf.shape
    R, C = pw.image
    w = lfsynth.uniform_f32((R, C), 10) - np.float32(0.5)
    g = lfsynth.uniform_f32((shape[4], R, C), pw.g_seed)
    dH = lf.grad_psf(to_dev(w), to_dev(g), shape).cpu().numpy().ravel()
    rng = np.random.default_rng(2)
    E = int(np.prod(shape))
    corners = np.ravel_multi_index(np.array([(0, 0, 0, 0, 0), (164, 164, 14, 14, 20), (0, 164, 7, 3, 10),
                                             (82, 82, 7, 7, 10), (164, 0, 0, 14, 0)]).T, shape)
    idx = np.concatenate([rng.integers(0, E, 3000), corners])
    assert rel_l2(dH[idx], oracle.grad_psf_at(shape, w, g, idx)) <= TOL
