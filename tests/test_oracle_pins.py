"""Pins of the CPU oracle to what the paper and the mathematics fix.

Each test checks the oracle (tests never compare the oracle with itself
through a retyped formula) against one of:
  * values the paper states for its worked examples (tests/golden/),
  * the paper's own index relations, Eqs. 4-9 (tests/paper_eqs.py),
  * properties the paper states (reversibility, slice sums, depth independence),
  * special cases that reduce to a library routine (scipy convolve/correlate),
  * brute force on tiny inputs (a scatter-form forward projection, exact
    adjoint identities on small integers).
"""
import itertools

import numpy as np
import pytest
from scipy.signal import convolve2d, correlate2d

import lfsynth
import oracle
import paper_eqs

ODD = (1, 3, 5, 7, 9, 11, 13, 15)


def tiny_shapes(limit=None, seed=0):
    """Odd shapes with every side <= 15, including nx != ny, ns < nx, nx = 1."""
    shapes = []
    for ns, nt in itertools.product((1, 3, 5, 7, 9, 15), repeat=2):
        for nx, ny in itertools.product((1, 3, 5), repeat=2):
            shapes.append((ns, nt, nx, ny, 2))
    shapes += [(15, 15, 3, 3, 3), (7, 9, 3, 5, 2), (9, 11, 5, 3, 2), (3, 5, 5, 3, 1),
               (11, 7, 1, 1, 2), (13, 13, 5, 5, 1), (5, 5, 5, 5, 1), (3, 3, 7, 7, 1),
               (15, 13, 15, 11, 1), (1, 1, 1, 1, 1), (5, 5, 3, 3, 4)]
    if limit is not None:
        rng = np.random.default_rng(seed)
        keep = rng.choice(len(shapes), size=min(limit, len(shapes)), replace=False)
        shapes = [shapes[i] for i in sorted(keep)] + shapes[-11:]
    return shapes


def rand_H(shape, seed, dtype=np.float32):
    return lfsynth.bits(shape, seed, dtype)


def same_bits(a, b):
    return a.dtype == b.dtype and a.shape == b.shape and a.tobytes() == b.tobytes()


# ---------------------------------------------------------------- paper values

def test_fig8_extended_slice_order(golden):
    """Sec. 4, Fig. 8: ns = 5, nx = 3 -> extended slice order C A B C A.
    Pins Eq. 5 of the helper and the oracle's wrap direction: the slice of H'
    of the middle pixel draws, for s' = 1..5, on H's slices in that order."""
    fx = golden("fig8_extended_slices.txt")
    ns, nx = int(fx["ns"][0]), int(fx["nx"][0])
    seq = fx["sequence"]
    names = {1: "A", 2: "B", 3: "C"}
    assert [names[x] for x in paper_eqs.extended_slices(ns, nx)] == seq
    # H[s][x] = code of slice x, one column, one depth: read which slice feeds H'.
    H = np.zeros((ns, 1, nx, 1, 1), dtype=np.float32)
    for x in range(nx):
        H[:, 0, x, 0, 0] = x + 1
    for Ht in (oracle.Ht_dense(H), oracle.Ht_rows(H)):
        middle = (nx - 1) // 2
        got = [names[int(v)] for v in Ht[:, 0, middle, 0, 0]]
        assert got == seq


def test_fig6_single_cell_contributions(golden):
    """Sec. 3, Fig. 6: with ns = nx = 3 and no added slices, the paper's
    relations give the centre pixel 9 contributors and the blue pixel 4."""
    fx = golden("fig6_contributions.txt")
    shape = tuple(int(fx[k][0]) for k in ("ns", "nt", "nx", "ny")) + (1,)
    H = rand_H(shape, 7)
    _, written, mult = paper_eqs.literal_Ht(H)
    per_slice = written[..., ].sum(axis=(0, 1))          # count per (x', y') pixel slice
    c = (shape[2] - 1) // 2, (shape[3] - 1) // 2
    assert per_slice[c] == int(fx["centre"][0])
    assert per_slice.max() == int(fx["centre"][0])
    assert int(fx["blue"][0]) in set(per_slice.ravel().tolist())
    assert mult.max() == 1


# ------------------------------------------------- the paper's index relations

@pytest.mark.parametrize("shape", tiny_shapes(limit=40, seed=1))
def test_oracle_matches_paper_relations_where_they_write(shape):
    """Eqs. 4-9 assign each H' entry at most once, and every entry they assign
    equals the oracle's.  Entries they leave unassigned (border bands, where
    the loop over m = 1..ns does not reach) number exactly
    (ns*nx - c(c+1)) ... per axis, with c = floor(nx/2) when ns >= nx."""
    H = rand_H(shape, 11)
    Ht = oracle.Ht_rows(H)
    lit, written, mult = paper_eqs.literal_Ht(H)
    assert mult.max() <= 1
    w = np.broadcast_to(written[..., None], H.shape)
    assert np.array_equal(lit.view(np.uint32)[w], Ht.view(np.uint32)[w])
    ns, nt, nx, ny, _ = shape
    if ns >= nx and nt >= ny:
        cx, cy = nx // 2, ny // 2
        assert paper_eqs.unwritten_per_axis(ns, nx) == cx * (cx + 1)
        assert paper_eqs.unwritten_per_axis(nt, ny) == cy * (cy + 1)
        assert written.sum() == (ns * nx - cx * (cx + 1)) * (nt * ny - cy * (cy + 1))


@pytest.mark.parametrize("shape", [(15, 15, 3, 3, 3), (13, 9, 5, 3, 2), (21, 21, 5, 5, 1)])
def test_oracle_equals_paper_relations_when_border_bands_are_zero(shape):
    """Where H vanishes on the border bands that Eqs. 4-9 never read from,
    the paper's assignment and the oracle agree on every entry."""
    ns, nt, nx, ny, _ = shape
    H = rand_H(shape, 3)
    cx, cy = nx // 2, ny // 2
    H[:cx], H[ns - cx:], H[:, :cy], H[:, nt - cy:] = 0, 0, 0, 0
    lit, _, _ = paper_eqs.literal_Ht(H)
    assert same_bits(lit, oracle.Ht_rows(H))


# ------------------------------------------------ stated properties of the map

@pytest.mark.parametrize("shape", [(15, 15, 1, 1, 3), (9, 5, 1, 1, 2), (1, 7, 1, 1, 1)])
def test_single_position_cell_is_rotation_by_180(shape):
    """Sec. 3, side note after Fig. 11: summed slices of H' equal the summed
    H rotated by 180 degrees.  With a one-position cell (nx = ny = 1) there is
    one slice, so H' itself is H rotated by 180 degrees in (s, t)."""
    H = rand_H(shape, 5)
    assert same_bits(oracle.Ht_rows(H), np.ascontiguousarray(H[::-1, ::-1]))


@pytest.mark.parametrize("shape", tiny_shapes(limit=20, seed=2))
def test_slice_sum_is_rotated_psf_sum(shape):
    """Sec. 3, side note after Fig. 11, on general shapes (exact integer sums)."""
    H = lfsynth.small_int_f32(shape, 9, 1000).astype(np.float64)
    Ht = oracle.Ht_rows(H.astype(np.float32)).astype(np.float64)
    assert np.array_equal(Ht.sum(axis=(2, 3)), H.sum(axis=(2, 3))[::-1, ::-1])


@pytest.mark.parametrize("shape", tiny_shapes(limit=25, seed=3))
def test_reversible(shape):
    """Sec. 3 and Sec. 6: the transformation is reversible -- applying it to H'
    gives back H, bit for bit."""
    for dtype in (np.float32, np.float16):
        H = rand_H(shape, 21, dtype)
        assert same_bits(oracle.Ht_rows(oracle.Ht_rows(H)), H)


@pytest.mark.parametrize("shape", tiny_shapes(limit=15, seed=4))
def test_pure_rearrangement_per_fibre(shape):
    """Sec. 3: no summation, a pure re-arrangement.  For each (s', t', z) the
    nx*ny values of H' are exactly the values of one pattern pixel of H."""
    H = rand_H(shape, 31)
    Ht = oracle.Ht_rows(H)
    ns, nt = shape[:2]
    hb, htb = H.view(np.uint32), Ht.view(np.uint32)
    for sp in range(ns):
        for tp in range(nt):
            for z in range(shape[4]):
                a = np.sort(htb[sp, tp, :, :, z].ravel())
                b = np.sort(hb[ns - 1 - sp, nt - 1 - tp, :, :, z].ravel())
                assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(15, 15, 3, 3, 5), (9, 7, 3, 5, 4)])
def test_depth_planes_independent(shape):
    """Sec. 4: depth planes are independent -- permuting z commutes with the map."""
    H = rand_H(shape, 41)
    perm = np.random.default_rng(0).permutation(shape[4])
    assert same_bits(oracle.Ht_rows(np.ascontiguousarray(H[..., perm])),
                     np.ascontiguousarray(oracle.Ht_rows(H)[..., perm]))


# --------------------------------------------- brute force: dense matrix route

@pytest.mark.parametrize("shape", tiny_shapes(limit=30, seed=5))
def test_dense_transpose_equals_rowwise(shape):
    """The explicitly transposed dense matrix and the entry-by-entry read-out
    give the same H' (both float32 and float16 payloads)."""
    for dtype in (np.float32, np.float16):
        H = rand_H(shape, 51, dtype)
        assert same_bits(oracle.Ht_dense(H), oracle.Ht_rows(H))


@pytest.mark.parametrize("shape", [(15, 15, 3, 3, 2), (9, 7, 3, 5, 1), (5, 5, 5, 5, 2)])
def test_every_interior_lenslet_gives_the_same_slices(shape):
    """Lenslet periodicity (Sec. 2.1): reading H' at any lenslet of a larger
    grid whose slices stay inside the image gives the same array."""
    ns, nt, nx, ny, _ = shape
    H = rand_H(shape, 61)
    ref = oracle.Ht_rows(H)
    cr, cc = -(-((ns - 1) // 2) // nx), -(-((nt - 1) // 2) // ny)
    Lr, Lc = 2 * cr + 3, 2 * cc + 2
    for lr in range(cr, Lr - cr):
        for lc in range(cc, Lc - cc):
            assert same_bits(oracle.Ht_dense(H, grid=(Lr, Lc, lr, lc)), ref)


def test_minimal_and_degenerate_shapes():
    for shape in [(1, 1, 1, 1, 1), (1, 1, 1, 1, 7), (3, 1, 3, 1, 1), (1, 3, 1, 5, 2)]:
        H = rand_H(shape, 71)
        assert same_bits(oracle.Ht_dense(H), oracle.Ht_rows(H))
        assert same_bits(oracle.Ht_rows(oracle.Ht_rows(H)), H)


def test_Ht_at_matches_full():
    H = rand_H((15, 13, 3, 5, 3), 81)
    full = oracle.Ht_rows(H)
    idx = np.random.default_rng(1).integers(0, H.size, 500)
    assert np.array_equal(oracle.Ht_at(H, idx).view(np.uint32), full.ravel().view(np.uint32)[idx])


# ------------------------------------------------------------- projectors

def scatter_forward(H, g):
    """Image formation as described in Sec. 2.1: every voxel adds a copy of its
    pattern, scaled by its value and centred on it, to the image."""
    ns, nt, nx, ny, nz = H.shape
    _, R, C = g.shape
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    f = np.zeros((R + ns, C + nt))                       # padded canvas
    for z in range(nz):
        for P in range(R):
            for Q in range(C):
                pat = H[:, :, P % nx, Q % ny, z].astype(np.float64)
                f[P:P + ns, Q:Q + nt] += g[z, P, Q] * pat     # pixel p = P + s - hs
    return f[hs:hs + R, ht:ht + C]


@pytest.mark.parametrize("shape,R,C", [((7, 5, 3, 1, 2), 9, 8), ((5, 5, 3, 3, 1), 9, 9),
                                       ((9, 9, 3, 3, 2), 7, 10)])
def test_forward_equals_pattern_scatter(shape, R, C):
    H = lfsynth.uniform_f32(shape, 1)
    g = lfsynth.uniform_f32((shape[4], R, C), 2)
    assert np.allclose(oracle.forward(H, g), scatter_forward(H, g), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape,R,C", [((7, 5, 1, 1, 3), 12, 10), ((15, 15, 1, 1, 1), 20, 17)])
def test_one_position_cell_reduces_to_convolution(shape, R, C):
    """nx = ny = 1: the projector is an ordinary per-depth 'same' convolution and
    its adjoint the matching correlation (scipy.signal)."""
    H = lfsynth.uniform_f32(shape, 3)
    g = lfsynth.uniform_f32((shape[4], R, C), 4)
    f = lfsynth.uniform_f32((R, C), 5)
    ref_f = sum(convolve2d(g[z].astype(np.float64), H[:, :, 0, 0, z].astype(np.float64), mode="same")
                for z in range(shape[4]))
    assert np.allclose(oracle.forward(H, g), ref_f, rtol=1e-12, atol=1e-12)
    ref_b = np.stack([correlate2d(f.astype(np.float64), H[:, :, 0, 0, z].astype(np.float64), mode="same")
                      for z in range(shape[4])])
    assert np.allclose(oracle.backward(H, f), ref_b, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape,R,C", [((5, 5, 3, 3, 2), 9, 12), ((7, 9, 3, 5, 1), 8, 11)])
def test_projectors_are_the_dense_matrix(shape, R, C):
    H = lfsynth.uniform_f32(shape, 6)
    g = lfsynth.uniform_f32((shape[4], R, C), 7)
    f = lfsynth.uniform_f32((R, C), 8)
    A = oracle.A_dense(H, R, C).astype(np.float64)
    assert np.allclose(oracle.forward(H, g).ravel(), A @ g.astype(np.float64).ravel(), rtol=1e-13)
    assert np.allclose(oracle.backward(H, f).ravel(), A.T @ f.astype(np.float64).ravel(), rtol=1e-13)


@pytest.mark.parametrize("shape,R,C", [((9, 7, 3, 3, 3), 13, 14), ((15, 15, 5, 5, 2), 20, 20)])
def test_adjoint_identity_exact(shape, R, C):
    """<A g, f> = <g, A^T f>, exact in float64 on small integers."""
    H = lfsynth.small_int_f32(shape, 1, 8)
    g = lfsynth.small_int_f32((shape[4], R, C), 2, 8)
    f = lfsynth.small_int_f32((R, C), 3, 8)
    lhs = float(np.sum(oracle.forward(H, g) * f.astype(np.float64)))
    rhs = float(np.sum(g.astype(np.float64) * oracle.backward(H, f)))
    assert lhs == rhs


def backproject_with_Ht(Ht, f):
    """A^T f from H' (the form the HIP backward uses): every pixel adds its
    slice of H' -- the voxels it receives light from -- scaled by its value."""
    ns, nt, nx, ny, nz = Ht.shape
    R, C = f.shape
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    g = np.zeros((nz, R + ns, C + nt))
    for p in range(R):
        for q in range(C):
            sl = Ht[:, :, p % nx, q % ny, :].astype(np.float64)      # [s'][t'][z]
            g[:, p:p + ns, q:q + nt] += f[p, q] * np.moveaxis(sl, 2, 0)  # voxel P = p + s' - hs
    return g[:, hs:hs + R, ht:ht + C]


@pytest.mark.parametrize("shape,R,C", [((9, 7, 3, 3, 2), 12, 10), ((5, 5, 3, 5, 1), 7, 8),
                                       ((15, 15, 5, 5, 1), 10, 15)])
def test_backprojection_through_Ht_is_the_adjoint(shape, R, C):
    """The oracle's H' back-projects images exactly as A^T computed from H
    (Sec. 3: H' is the backprojection operator of Eq. 2)."""
    H = lfsynth.small_int_f32(shape, 4, 8)
    f = lfsynth.small_int_f32((R, C), 5, 8)
    assert np.array_equal(backproject_with_Ht(oracle.Ht_rows(H), f), oracle.backward(H, f))


@pytest.mark.parametrize("shape,R,C", [((5, 5, 3, 3, 2), 9, 12), ((7, 9, 3, 5, 1), 8, 11),
                                       ((9, 7, 1, 1, 3), 10, 7)])
def test_sparse_projectors_are_the_dense_matrix(shape, R, C):
    """The nonzero-entry forms (for full-size images) against the dense
    measurement matrix, on PSFs with most entries zero, and against the
    pixel/voxel forms with the sums exact (small integers): bit for bit."""
    H = lfsynth.uniform_f32(shape, 16)
    H[H < 0.7] = 0.0
    g = lfsynth.uniform_f32((shape[4], R, C), 17)
    f = lfsynth.uniform_f32((R, C), 18)
    A = oracle.A_dense(H, R, C).astype(np.float64)
    for nth in (1, 3):
        assert np.allclose(oracle.forward_sparse(H, g, nth).ravel(), A @ g.astype(np.float64).ravel(),
                           rtol=1e-13, atol=1e-13)
        assert np.allclose(oracle.backward_sparse(H, f, nth).ravel(), A.T @ f.astype(np.float64).ravel(),
                           rtol=1e-13, atol=1e-13)
    Hi = lfsynth.small_int_f32(shape, 19, 8)
    Hi[::2] = 0.0
    gi = lfsynth.small_int_f32((shape[4], R, C), 20, 8)
    fi = lfsynth.small_int_f32((R, C), 21, 8)
    assert np.array_equal(oracle.forward_sparse(Hi, gi, 2), oracle.forward(Hi, gi))
    assert np.array_equal(oracle.backward_sparse(Hi, fi, 2), oracle.backward(Hi, fi))


def test_sparse_projectors_all_zero_and_scatter():
    shape, R, C = (9, 9, 3, 3, 2), 11, 13
    g = lfsynth.uniform_f32((shape[4], R, C), 22)
    assert not oracle.forward_sparse(np.zeros(shape, np.float32), g).any()
    H = lfsynth.uniform_f32(shape, 23)
    assert np.allclose(oracle.forward_sparse(H, g), scatter_forward(H, g), rtol=1e-13, atol=1e-13)


def test_forward_at_and_backward_at_match_full():
    shape, R, C = (9, 9, 3, 3, 2), 12, 15
    H = lfsynth.uniform_f32(shape, 9)
    g = lfsynth.uniform_f32((shape[4], R, C), 10)
    f = lfsynth.uniform_f32((R, C), 11)
    full_f, full_b = oracle.forward(H, g), oracle.backward(H, f)
    pix = np.array([(0, 0), (R - 1, C - 1), (5, 7), (11, 0)])
    assert np.array_equal(oracle.forward_at(H, g, pix), full_f[pix[:, 0], pix[:, 1]])
    vox = np.array([(0, 0, 0), (1, R - 1, C - 1), (1, 4, 9)])
    assert np.array_equal(oracle.backward_at(H, f, vox), full_b[vox[:, 0], vox[:, 1], vox[:, 2]])


# ---------------------------------------------------------------- the paper's method in C

PAPER_SHAPES = [(5, 5, 3, 3, 2), (15, 15, 3, 3, 3), (7, 9, 3, 5, 2), (9, 11, 5, 3, 4), (3, 5, 5, 3, 1),
                (11, 7, 1, 1, 2), (13, 13, 5, 5, 1), (21, 17, 7, 5, 3)]


@pytest.mark.parametrize("shape", PAPER_SHAPES)
def test_paper_method_in_c_equals_the_per_axis_relations(shape):
    """oracle.paper_Ht (C, timed by the benchmark as the paper's method) writes
    exactly the entries the per-axis transcription of Eqs. 4-9 writes, with the
    same values, and leaves the others untouched."""
    H = lfsynth.bits(shape, 31, np.float32)
    ref, written, _ = paper_eqs.literal_Ht(H)
    canary = np.full(H.shape, np.float32(-7.25))
    got, cols = oracle.paper_Ht(H, out=canary.copy())
    mask = np.broadcast_to(written[..., None], H.shape)
    assert np.array_equal(got.view(np.uint32)[mask], ref.view(np.uint32)[mask])
    assert (got[~mask] == np.float32(-7.25)).all()
    assert cols == int(written.sum())


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_paper_method_in_c_equals_the_oracle_with_zero_borders(dtype):
    """On the generator's PSFs (zero on the patch border bands) the paper's
    method gives the whole of the oracle's H', for 1 and several threads."""
    H, _ = lfsynth.make_H(lfsynth.TINY, dtype)
    ref = oracle.Ht_rows(H)
    for nth in (1, 3):
        got, _ = oracle.paper_Ht(H, nthreads=nth)
        assert got.tobytes() == ref.tobytes()
