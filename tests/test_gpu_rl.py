"""Richardson-Lucy updates (Eq. 2) on the GPU against the float64 oracle:
relative L2 <= 1e-5 per step, the zero readings, in-place updates and the
workspace forms."""
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


def problem(shape, R, C, seed):
    """H, a positive volume, and a noisy image of a second volume."""
    H = lfsynth.uniform_f32(shape, seed)
    g = (lfsynth.uniform_f32((shape[4], R, C), seed + 1) + 0.05).astype(np.float32)
    g_true = (lfsynth.uniform_f32((shape[4], R, C), seed + 2) + 0.05).astype(np.float32)
    f = (oracle.forward(H, g_true) * (0.9 + 0.2 * lfsynth.uniform_f32((R, C), seed + 3))).astype(np.float32)
    return H, g, f


SHAPES = [((15, 15, 3, 3, 3), 21, 21), ((9, 7, 3, 5, 2), 12, 10), ((7, 9, 1, 1, 3), 11, 9),
          ((33, 25, 11, 5, 4), 55, 40), ((5, 5, 3, 3, 45), 6, 7), ((21, 21, 17, 17, 2), 40, 36)]


@pytest.mark.parametrize("shape,R,C", SHAPES)
def test_norm_and_one_step_vs_oracle(shape, R, C):
    H, g, f = problem(shape, R, C, 10)
    dH = to_dev(H)
    dHt = lf.compute_Ht(dH)
    n = lf.rl_norm(dHt, R, C)
    g1 = lf.rl_step(dH, dHt, to_dev(f), to_dev(g), n)
    torch.cuda.synchronize()
    n_ref = oracle.rl_norm(H, R, C)
    assert rel_l2(n.cpu().numpy(), n_ref) <= TOL
    assert rel_l2(g1.cpu().numpy(), oracle.rl_step(H, f, g, norm=n_ref)) <= TOL


def test_in_place_and_workspace_forms_agree():
    import ctypes
    from paper_2003_09133_amd import _abi
    shape, R, C = (45, 45, 15, 15, 5), 97, 120
    H, g, f = problem(shape, R, C, 20)
    dH, df, dg = to_dev(H), to_dev(f), to_dev(g)
    dHt = lf.compute_Ht(dH)
    n = lf.rl_norm(dHt, R, C)
    ref = lf.rl_step(dH, dHt, df, dg, n)
    inplace = dg.clone()
    lf.rl_step(dH, dHt, df, inplace, n, out=inplace)
    alloc = torch.empty_like(dg)
    st = _abi.lib().lfbp_rl_step(dH.data_ptr(), dHt.data_ptr(), _abi.Shape.of(shape), df.data_ptr(), R, C,
                                 dg.data_ptr(), n.data_ptr(), alloc.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(ref, inplace) and torch.equal(ref, alloc)


def test_zero_denominators_on_gpu():
    """A voxel class whose pattern is all zero gets exactly 0; pixels where the
    forward projection is 0 give a zero quotient (the oracle's readings)."""
    shape, R, C = (5, 5, 3, 3, 2), 9, 9
    H = lfsynth.uniform_f32(shape, 12)
    H[:, :, 1, 2, 0] = 0.0
    g = (lfsynth.uniform_f32((shape[4], R, C), 13) + 0.05).astype(np.float32)
    g[:, :4, :] = 0.0
    f = (lfsynth.uniform_f32((R, C), 14) + 0.1).astype(np.float32)
    dH = to_dev(H)
    dHt = lf.compute_Ht(dH)
    n = lf.rl_norm(dHt, R, C)
    g1 = lf.rl_step(dH, dHt, to_dev(f), to_dev(g), n).cpu().numpy()
    assert np.all(n.cpu().numpy()[0, 1::3, 2::3] == 0)
    assert np.all(g1[0, 1::3, 2::3] == 0) and np.all(np.isfinite(g1))
    assert rel_l2(g1, oracle.rl_step(H, f, g)) <= TOL


def test_five_iterations_vs_oracle():
    """Five updates from a flat start; each step's float32 rounding carries
    into the next, so the bar is the per-step bar times the step count."""
    shape, R, C = (21, 21, 5, 5, 4), 40, 45
    H, _, f = problem(shape, R, C, 30)
    dH = to_dev(H)
    g_gpu = lf.richardson_lucy(dH, to_dev(f), 5)
    g = np.ones((shape[4], R, C))
    n = oracle.rl_norm(H, R, C)
    for _ in range(5):
        g = oracle.rl_step(H, f, g, norm=n)
    assert rel_l2(g_gpu.cpu().numpy(), g) <= 5 * TOL


def test_poisson_data_one_step_and_five_iterations():
    """Shot-noise data, f = Poisson(H g_true) with 50 photons per pixel on
    average, on a 4 x 4-lenslet crop of the microscope PSF: one update from a
    flat start against the oracle, and five updates."""
    w = lfsynth.MICROSCOPE
    H, _ = lfsynth.make_H(w)
    R = C = 4 * w.shape[2]
    g_true = (lfsynth.uniform_f32((w.shape[4], R, C), 50) ** 4).astype(np.float32)
    mean = oracle.forward(H, g_true)
    lam = mean * (50.0 / mean.mean())
    f = lfsynth.poisson_counts(lam, 51)
    assert (f == np.round(f)).all() and abs(np.var(f - lam) / lam.mean() - 1.0) < 0.2   # counts, var = mean
    dH = to_dev(H)
    dHt = lf.compute_Ht(dH)
    n = lf.rl_norm(dHt, R, C)
    g0 = np.ones((w.shape[4], R, C), np.float32)
    g1 = lf.rl_step(dH, dHt, to_dev(f), to_dev(g0), n)
    n_ref = oracle.rl_norm(H, R, C)
    assert rel_l2(g1.cpu().numpy(), oracle.rl_step(H, f, g0, norm=n_ref)) <= TOL
    g5 = lf.richardson_lucy(dH, to_dev(f), 5)
    g = np.ones((w.shape[4], R, C))
    for _ in range(5):
        g = oracle.rl_step(H, f, g, norm=n_ref)
    assert rel_l2(g5.cpu().numpy(), g) <= 5 * TOL


def test_projector_crop_one_step():
    """A 4 x 4-lenslet crop of the projector workload (microscope PSF, 60 x 60
    px, 21 depths)."""
    w = lfsynth.MICROSCOPE
    H, _ = lfsynth.make_H(w)
    R = C = 4 * w.shape[2]
    g = (lfsynth.uniform_f32((w.shape[4], R, C), 40) + 0.05).astype(np.float32)
    f = (lfsynth.uniform_f32((R, C), 41) + 0.5).astype(np.float32)
    dH = to_dev(H)
    dHt = lf.compute_Ht(dH)
    g1 = lf.rl_step(dH, dHt, to_dev(f), to_dev(g), lf.rl_norm(dHt, R, C))
    assert rel_l2(g1.cpu().numpy(), oracle.rl_step(H, f, g)) <= TOL
