"""Pins of the float64 oracle of d<w, H g>/dH (the gradient with respect to
the PSF array): the exact adjoint identity with the pinned forward oracle, a
brute-force derivative through torch's CPU autograd on tiny grids, and the
single-position cell, where it is a 2-D correlation (scipy)."""
import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

import lfsynth
import oracle


@pytest.mark.parametrize("shape,R,C", [((9, 7, 3, 5, 2), 12, 10), ((5, 5, 3, 3, 3), 9, 11), ((3, 5, 5, 3, 1), 7, 8),
                                       ((15, 15, 3, 3, 2), 21, 20)])
def test_adjoint_identity_exact(shape, R, C):
    """<dH(w, g), D> = <w, A(D) g> for any direction D: exact in float64 on
    small integers (f is linear in H)."""
    w = lfsynth.small_int_f32((R, C), 1, 8)
    g = lfsynth.small_int_f32((shape[4], R, C), 2, 8)
    D = lfsynth.small_int_f32(shape, 3, 8)
    lhs = float(np.sum(oracle.grad_psf(shape, w, g) * D.astype(np.float64)))
    rhs = float(np.sum(w.astype(np.float64) * oracle.forward(D, g)))
    assert lhs == rhs


def torch_forward(H, g):
    """f = A(H) g written with torch ops on the CPU: every voxel adds its
    pattern H[:, :, P mod nx, Q mod ny, z], centred on it, to the image."""
    ns, nt, nx, ny, nz = H.shape
    _, R, C = g.shape
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    f = torch.zeros((R + ns, C + nt), dtype=torch.float64)
    for z in range(nz):
        for P in range(R):
            for Q in range(C):
                f = f.index_put((torch.arange(P, P + ns)[:, None], torch.arange(Q, Q + nt)[None, :]),
                                g[z, P, Q] * H[:, :, P % nx, Q % ny, z], accumulate=True)
    return f[hs:hs + R, ht:ht + C]


@pytest.mark.parametrize("shape,R,C", [((5, 3, 3, 1, 2), 6, 4), ((3, 3, 1, 3, 1), 5, 7)])
def test_matches_torch_autograd_brute_force(shape, R, C):
    H = lfsynth.uniform_f32(shape, 4)
    g = lfsynth.uniform_f32((shape[4], R, C), 5)
    w = lfsynth.uniform_f32((R, C), 6)
    Ht = torch.from_numpy(H.astype(np.float64)).requires_grad_(True)
    f = torch_forward(Ht, torch.from_numpy(g.astype(np.float64)))
    assert np.allclose(f.detach().numpy(), oracle.forward(H, g), rtol=1e-12)
    (f * torch.from_numpy(w.astype(np.float64))).sum().backward()
    assert np.allclose(Ht.grad.numpy(), oracle.grad_psf(shape, w, g), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape,R,C", [((7, 5, 1, 1, 3), 12, 10), ((9, 9, 1, 1, 1), 15, 11)])
def test_one_position_cell_is_a_correlation(shape, R, C):
    """nx = ny = 1: dH[:, :, 0, 0, z] = correlation of w with g[z], centred."""
    ns, nt = shape[0], shape[1]
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    w = lfsynth.uniform_f32((R, C), 7).astype(np.float64)
    g = lfsynth.uniform_f32((shape[4], R, C), 8).astype(np.float64)
    dH = oracle.grad_psf(shape, w, g)
    for z in range(shape[4]):
        full = correlate2d(w, g[z], mode="full")      # index (d + R-1, e + C-1) = sum w[P+d][Q+e] g[P][Q]
        ref = full[R - 1 - hs:R - 1 - hs + ns, C - 1 - ht:C - 1 - ht + nt]
        assert np.allclose(dH[:, :, 0, 0, z], ref, rtol=1e-12)


def test_sampled_entries_match_full():
    shape, R, C = (9, 9, 3, 3, 2), 12, 15
    w = lfsynth.uniform_f32((R, C), 9)
    g = lfsynth.uniform_f32((shape[4], R, C), 10)
    full = oracle.grad_psf(shape, w, g).ravel()
    idx = np.random.default_rng(0).integers(0, full.size, 300)
    assert np.array_equal(oracle.grad_psf_at(shape, w, g, idx), full[idx])
