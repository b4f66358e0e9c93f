"""The column-major (Matlab order) H -> H' kernel's index arithmetic, on the
CPU: a NumPy mirror of k_colmajor (paper_2003_09133_amd/csrc/lfbp_colmajor.hip)
and its chunking, against the oracle's H' moved to column-major order.  Keep
it in step with the kernel."""
import numpy as np
import pytest

import lfsynth
import oracle


def to_colmajor(A):
    """Column-major storage of an [ns][nt][nx][ny][nz] array, as a flat array."""
    return np.ascontiguousarray(A.transpose(4, 3, 2, 1, 0)).ravel()


def colmajor_mirror(Hc, shape, budget, max_lds=160 * 1024, esize=4):
    ns, nt, nx, ny, nz = shape
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    a_off, b_off = (nx - hs % nx) % nx, (ny - ht % ny) % ny
    col = nx * esize
    bud = budget if col <= budget else max_lds
    S0 = min(ns, bud // col)
    assert S0 > 0
    chunks = -(-ns // S0)
    S = -(-ns // chunks)
    assert nx * S * esize <= bud
    out = np.full(Hc.size, np.nan, Hc.dtype)
    written = np.zeros(Hc.size, np.int64)
    xstride = ns * nt
    for unit in range(nt * ny * nz * chunks):
        plane, c = divmod(unit, chunks)
        q1, tp = divmod(plane, nt)
        z, yp = divmod(q1, ny)
        b = (tp + b_off) % ny
        y = (yp + b) % ny
        t = nt - 1 - tp
        s0 = c * S
        assert s0 < ns
        Sn = min(S, ns - s0)
        s_lo = ns - s0 - Sn
        in0 = (t + nt * nx * (y + ny * z)) * ns
        out0 = (tp + nt * nx * (yp + ny * z)) * ns
        i = np.arange(nx * Sn)
        x, k = i // Sn, i % Sn
        src = in0 + x * xstride + s_lo + k
        assert src.min() >= 0 and src.max() < Hc.size
        tile = Hc[src]
        xp = x
        sp = s0 + k
        xs = (xp + (sp + a_off) % nx) % nx
        dst = out0 + xp * xstride + sp
        assert dst.min() >= 0 and dst.max() < Hc.size
        out[dst] = tile[xs * Sn + (Sn - 1 - k)]
        written[dst] += 1
    assert np.all(written == 1)
    return out


@pytest.mark.parametrize("shape", [(15, 15, 3, 3, 3), (9, 7, 3, 5, 2), (3, 5, 5, 3, 1), (1, 1, 1, 1, 2),
                                   (11, 7, 1, 1, 2), (21, 9, 7, 3, 4), (5, 5, 9, 1, 3), (13, 11, 9, 5, 2)])
@pytest.mark.parametrize("budget", [32 * 1024, 40, 12])
def test_colmajor_mirror_equals_oracle(shape, budget):
    H = lfsynth.bits(shape, 5, np.float32)
    got = colmajor_mirror(to_colmajor(H), shape, budget)
    ref = to_colmajor(oracle.Ht_rows(H))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
