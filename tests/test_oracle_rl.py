"""Pins of the float64 Richardson-Lucy oracle (Eq. 2) against what the
mathematics fixes: the true volume is a fixed point of noise-free data, the
update conserves flux, it never lowers the Poisson log-likelihood (it is an
expectation-maximisation step), it reduces to ordinary 2-D Richardson-Lucy with
scipy's convolutions when the elementary cell has one position, and it follows
the stated readings where a quotient has a zero denominator."""
import numpy as np
import pytest
from scipy.signal import convolve2d, correlate2d

import lfsynth
import oracle

SHAPES = [((9, 7, 3, 5, 2), 12, 10), ((15, 15, 3, 3, 3), 21, 20), ((5, 5, 5, 5, 1), 7, 8), ((7, 9, 1, 1, 3), 11, 9)]


def positive_volume(shape, R, C, seed):
    return lfsynth.uniform_f32((shape[4], R, C), seed).astype(np.float64) + 0.05


@pytest.mark.parametrize("shape,R,C", SHAPES)
def test_true_volume_is_a_fixed_point(shape, R, C):
    H = lfsynth.uniform_f32(shape, 1)
    g = positive_volume(shape, R, C, 2)
    f = oracle.forward64(H, g)
    g1 = oracle.rl_step(H, f, g)
    assert np.allclose(g1, g, rtol=1e-12, atol=0)


@pytest.mark.parametrize("shape,R,C", SHAPES)
def test_flux_is_conserved(shape, R, C):
    """sum_v (A^T 1)_v g'_v = sum_p f_p over pixels where A g > 0."""
    H = lfsynth.uniform_f32(shape, 3)
    g = positive_volume(shape, R, C, 4)
    f = lfsynth.uniform_f32((R, C), 5).astype(np.float64)
    n = oracle.rl_norm(H, R, C)
    g1 = oracle.rl_step(H, f, g, norm=n)
    fp = oracle.forward64(H, g)
    assert np.isclose(np.sum(n * g1), np.sum(f[fp > 0]), rtol=1e-12)


def log_likelihood(H, f, g):
    fp = oracle.forward64(H, g)
    m = fp > 0
    return float(np.sum(f[m] * np.log(fp[m])) - np.sum(fp))


@pytest.mark.parametrize("shape,R,C", SHAPES[:3])
def test_each_step_raises_the_poisson_likelihood(shape, R, C):
    H = lfsynth.uniform_f32(shape, 6)
    g_true = positive_volume(shape, R, C, 7)
    f = oracle.forward64(H, g_true) * (1.0 + 0.2 * (lfsynth.uniform_f32((R, C), 8) - 0.5))
    g = np.ones_like(g_true)
    L = log_likelihood(H, f, g)
    for _ in range(5):
        g = oracle.rl_step(H, f, g)
        L1 = log_likelihood(H, f, g)
        assert L1 >= L - 1e-9 * abs(L)
        L = L1


@pytest.mark.parametrize("shape,R,C", [((7, 5, 1, 1, 3), 12, 10), ((9, 9, 1, 1, 2), 15, 11)])
def test_one_position_cell_is_2d_richardson_lucy(shape, R, C):
    """nx = ny = 1: forward = sum over depths of 'same' convolutions, backward =
    the matching correlations; the update written with scipy."""
    H = lfsynth.uniform_f32(shape, 9)
    g = positive_volume(shape, R, C, 10)
    f = lfsynth.uniform_f32((R, C), 11).astype(np.float64) + 0.1
    k = [H[:, :, 0, 0, z].astype(np.float64) for z in range(shape[4])]
    fp = sum(convolve2d(g[z], k[z], mode="same") for z in range(shape[4]))
    ratio = f / fp
    ref = np.stack([g[z] * correlate2d(ratio, k[z], mode="same") / correlate2d(np.ones((R, C)), k[z], mode="same")
                    for z in range(shape[4])])
    assert np.allclose(oracle.rl_step(H, f, g), ref, rtol=1e-12)


def test_zero_denominators_follow_the_readings():
    """A voxel class with an all-zero pattern reaches no pixel (A^T 1 = 0): its
    update is 0.  Pixels where A g = 0 contribute a zero quotient."""
    shape, R, C = (5, 5, 3, 3, 2), 9, 9
    H = lfsynth.uniform_f32(shape, 12)
    H[:, :, 1, 2, 0] = 0.0                         # class (1,2) at depth 0 sees nothing
    g = positive_volume(shape, R, C, 13)
    g[:, :4, :] = 0.0                               # dark top rows: A g = 0 near them
    f = lfsynth.uniform_f32((R, C), 14).astype(np.float64) + 0.1
    n = oracle.rl_norm(H, R, C)
    assert np.all(n[0, 1::3, 2::3] == 0) and np.all(n[1] > 0)
    fp = oracle.forward64(H, g)
    assert np.any(fp == 0)
    g1 = oracle.rl_step(H, f, g, norm=n)
    assert np.all(g1[0, 1::3, 2::3] == 0)
    assert np.all(np.isfinite(g1)) and np.all(g1 >= 0)
    ratio = np.where(fp > 0, f / np.where(fp > 0, fp, 1), 0.0)
    ref = np.where(n > 0, g * oracle.backward64(H, ratio) / np.where(n > 0, n, 1), 0.0)
    assert np.allclose(g1, ref, rtol=1e-13, atol=0)


def test_float64_projections_agree_with_the_float32_input_forms():
    shape, R, C = (9, 9, 3, 3, 2), 12, 15
    H = lfsynth.uniform_f32(shape, 15)
    g = lfsynth.uniform_f32((shape[4], R, C), 16)
    f = lfsynth.uniform_f32((R, C), 17)
    assert np.array_equal(oracle.forward64(H, g.astype(np.float64)), oracle.forward(H, g))
    assert np.array_equal(oracle.backward64(H, f.astype(np.float64)), oracle.backward(H, f))
