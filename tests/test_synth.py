"""The seeded input generator: deterministic, in range, shaped like the workloads."""
import numpy as np

import lfsynth
from lfsynth import workloads


def test_word_is_splitmix64():
    """SplitMix64 (Steele, Lea & Flood 2014): with state increment 0x9E3779B97F4A7C15,
    the first output of seed 0 is the finaliser applied to the increment."""
    assert lfsynth.word(0, 0x9E3779B97F4A7C15) == lfsynth.word(1, 0)
    assert lfsynth.word(0, 0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    assert lfsynth.word(0, 0) == 0


def test_deterministic_and_seed_dependent():
    a = lfsynth.bits_u32((1000,), 5)
    assert np.array_equal(a, lfsynth.bits_u32((1000,), 5))
    assert not np.array_equal(a, lfsynth.bits_u32((1000,), 6))
    assert np.array_equal(lfsynth.bits_u32((1000,), 5, nthreads=1), lfsynth.bits_u32((1000,), 5, nthreads=8))


def test_special_payloads_present():
    a = lfsynth.bits_u32((100000,), 1)
    for v in (0x80000000, 0x7F800000, 0xFF800000, 0x7FC00001, 0x00000001):
        assert (a == v).any()
    b = lfsynth.bits_u16((100000,), 1)
    for v in (0x8000, 0x7C00, 0x7E01, 0x0001):
        assert (b == v).any()


def test_uniform_range():
    u = lfsynth.uniform_f32((100000,), 3)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01


def test_gauss_tiny():
    w = workloads.TINY
    H, zf, vmax = lfsynth.gauss_f32(w.shape, w.sig0, w.slope, w.zc, w.seed)
    assert H.shape == w.shape and H.dtype == np.float32
    assert H.max() == np.float32(vmax) and H.min() == 0.0
    nz = H[H != 0]
    assert nz.min() >= np.float32(0.05 * vmax)
    assert 0.5 < zf < 0.99
    H2, _, _ = lfsynth.gauss_f32(w.shape, w.sig0, w.slope, w.zc, w.seed, nthreads=1)
    assert np.array_equal(H, H2)


def test_gauss_envelope_follows_source():
    """The pattern of source (a, b) peaks near the patch centre shifted by the
    source's offset from the cell centre."""
    shape = (31, 31, 5, 5, 1)
    H, _, _ = lfsynth.gauss_f32(shape, 1.5, 0.0, 0.0, 9, thr=0.0)
    weights = np.zeros((5, 5, 2))
    s = np.arange(31)
    for a in range(5):
        for b in range(5):
            pat = H[:, :, a, b, 0].astype(np.float64)
            weights[a, b] = [(pat.sum(1) * s).sum() / pat.sum(), (pat.sum(0) * s).sum() / pat.sum()]
            assert abs(weights[a, b, 0] - (15 + a - 2)) < 0.6
            assert abs(weights[a, b, 1] - (15 + b - 2)) < 0.6


def test_batched_table_covers_all_sizes():
    sets = workloads.BATCHED_SETS
    assert len(sets) == 16
    assert sorted({w.shape[2] for w in sets}) == [7, 11, 15, 19]
    assert sorted({w.shape[0] // w.shape[2] for w in sets}) == [9, 11, 13, 15, 17, 19, 21, 23, 25]
    assert all(9 <= w.shape[4] <= 41 for w in sets)
    assert all(w.shape[0] % 2 == 1 and w.shape[2] % 2 == 1 for w in sets)
    assert sum(w.elements for w in sets) == 6_466_033_897
