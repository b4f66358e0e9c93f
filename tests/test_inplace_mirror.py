"""The in-place H -> H' kernel's index arithmetic, on the CPU.

A NumPy mirror of k_inplace (paper_2003_09133_amd/csrc/lfbp_inplace.hip) and of
its launch arithmetic: every unit (block pair, row group) reads its rows into
two tiles before writing, units touch disjoint rows, all addresses stay inside
the array, and the rewritten array equals the oracle's H'.  Keep it in step
with the kernel."""
import numpy as np
import pytest

import lfsynth
import oracle


def inplace_mirror(H, tile_budget=40 * 1024, max_lds=160 * 1024, esize=4, group_rows=5):
    ns, nt, nx, ny, nz = H.shape
    W, NB = ny * nz, ns * nt
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    a_off, b_off = (nx - hs % nx) % nx, (ny - ht % ny) % ny
    pairs = (NB - 1) // 2
    flat = H.reshape(-1).copy()
    if pairs == 0:
        return flat.reshape(H.shape), set()
    budget = tile_budget if 2 * W * esize <= tile_budget else max_lds
    nr0 = min(nx, group_rows, budget // (2 * W * esize))
    assert nr0 > 0
    groups = -(-nx // nr0)
    nr_full = -(-nx // groups)
    assert 2 * nr_full * W * esize <= budget <= max_lds
    touched = np.zeros(flat.size, np.int64)
    E = flat.size
    for unit in range(pairs * groups):
        O, grp = divmod(unit, groups)
        Op = NB - 1 - O
        sp, tp = divmod(O, nt)
        a, b = (sp + a_off) % nx, (tp + b_off) % ny
        rotA, rotB = b * nz, ((ny - b) % ny) * nz
        x0 = grp * nr_full
        assert x0 < nx
        nr = min(nr_full, nx - x0)
        xb0 = (x0 + a) % nx
        k1 = min(nr, nx - xb0)
        gO = (O * nx + x0) * W
        gP1, gP2 = (Op * nx + xb0) * W, Op * nx * W
        segs_in = [(gO, nr * W, rotB, "B", 0), (gP1, k1 * W, rotA, "A", 0)]
        segs_out = [(gO, nr * W, "A", 0), (gP1, k1 * W, "B", 0)]
        if nr > k1:
            segs_in.append((gP2, (nr - k1) * W, rotA, "A", k1 * W))
            segs_out.append((gP2, (nr - k1) * W, "B", k1 * W))
        tiles = {"A": np.empty(nr * W, flat.dtype), "B": np.empty(nr * W, flat.dtype)}
        for g, L, rot, t, off in segs_in:            # load_segment: whole rows, rotated into the tile
            assert g >= 0 and g + L <= E and L % W == 0
            e = np.arange(L)
            r, j = e // W, e % W
            tiles[t][off + r * W + (j - rot) % W] = flat[g + e]
        for g, L, t, off in segs_out:                 # store_segment, after every load of the unit
            flat[g:g + L] = tiles[t][off:off + L]
            touched[g:g + L] += 1
    centre = (NB - 1) // 2
    assert np.all(touched[centre * nx * W:(centre + 1) * nx * W] == 0)
    rest = np.delete(touched, np.arange(centre * nx * W, (centre + 1) * nx * W))
    assert np.all(rest == 1)                        # every other element written exactly once
    return flat.reshape(H.shape), touched


@pytest.mark.parametrize("shape", [(15, 15, 3, 3, 3), (9, 7, 3, 5, 2), (3, 5, 5, 3, 1), (1, 1, 1, 1, 2),
                                   (1, 3, 1, 1, 1), (11, 7, 1, 1, 2), (13, 13, 5, 5, 1), (21, 9, 7, 3, 4),
                                   (5, 5, 9, 1, 3)])
@pytest.mark.parametrize("tile_budget", [40 * 1024, 2 * 4 * 15, 512])
def test_inplace_mirror_equals_oracle(shape, tile_budget):
    """The launch's tile budget (small budgets force many row groups per block
    pair; a row pair larger than the budget falls back to the whole LDS)."""
    H = lfsynth.bits(shape, 3, np.float32)
    out, _ = inplace_mirror(H, tile_budget)
    ref = oracle.Ht_rows(H)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    out, _ = inplace_mirror(H, tile_budget, group_rows=1 << 20)     # whole blocks where the budget allows
    ref = oracle.Ht_rows(H)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))


def test_inplace_mirror_is_an_involution():
    H = lfsynth.bits((9, 11, 3, 5, 2), 4, np.float32)
    once, _ = inplace_mirror(H, 600)
    twice, _ = inplace_mirror(once, 600)
    assert not np.array_equal(once.view(np.uint32), H.view(np.uint32))
    assert np.array_equal(twice.view(np.uint32), H.view(np.uint32))
