"""The paper's index relations between H and H' (Sec. 4, Eqs. 4-9), test-only.

Used to pin the oracle: the oracle never evaluates these relations, it reads H'
out of the transposed measurement matrix.  Everything here is 1-based, in the
paper's notation, and per axis: the relations for (s, x, s', x') involve only
ns and nx, those for (t, y, t', y') only nt and ny, and depth planes are
independent (Sec. 4), so an assignment H'(s',t',x',y',:) = H(s,t,x,y,:)
(Eq. 3) is made for every pair of valid per-axis tuples.

Per axis the loop runs over the pixel index s = 1..ns (Eqs. 8-9 are taken for
s = 1..ns) and the extended slice index m = 1..ns (the nx slices plus the
ns - nx added ones, Sec. 4 after Eq. 5).  A tuple is valid when the H'
position lies in the window 0 < x' <= nx and 0 < s' (Eqs. 6-9).
"""
from __future__ import annotations

import numpy as np


def wrap_x(alpha: int, nx: int) -> int:
    """Eq. (5): the source slice x for the extended slice alpha (1-based)."""
    if alpha > nx:
        return alpha - ((alpha - 1) // nx) * nx
    if alpha <= 0:
        return alpha + (-((alpha - 1) // nx)) * nx      # ceil((1 - alpha) / nx)
    return alpha


def axis_tuples(ns: int, nx: int):
    """All valid (s', x', s, x) tuples of one axis, 1-based."""
    off = (ns - nx) // 2                                 # floor((ns - nx) / 2)
    out = []
    for s in range(1, ns + 1):
        sp = ns - s + (ns % 2)                           # Eq. (8)
        if sp <= 0:
            continue
        for m in range(1, ns + 1):
            alpha = m - off                              # Eq. (4)
            x = wrap_x(alpha, nx)                        # Eq. (5)
            xp = s - nx + alpha + (nx - 1) // 2 - off    # Eq. (6)
            if 0 < xp <= nx:
                out.append((sp, xp, s, x))
    return out


def extended_slices(ns: int, nx: int):
    """x(m) for m = 1..ns: the sequence of slices of the extended H (Eq. 5)."""
    off = (ns - nx) // 2
    return [wrap_x(m - off, nx) for m in range(1, ns + 1)]


def literal_Ht(H: np.ndarray):
    """H' assembled from Eq. 3 with the relations of Eqs. 4-9.

    Returns (Ht, written, multiplicity): entries never assigned stay zero and
    ``written`` is False there; ``multiplicity`` counts assignments per (s',t',x',y')
    so that a test can check that no entry is assigned twice."""
    ns, nt, nx, ny, nz = H.shape
    Ht = np.zeros_like(H)
    mult = np.zeros((ns, nt, nx, ny), dtype=np.int64)
    ax1 = axis_tuples(ns, nx)
    ax2 = axis_tuples(nt, ny)
    for sp, xp, s, x in ax1:
        for tp, yp, t, y in ax2:
            Ht[sp - 1, tp - 1, xp - 1, yp - 1, :] = H[s - 1, t - 1, x - 1, y - 1, :]
            mult[sp - 1, tp - 1, xp - 1, yp - 1] += 1
    return Ht, mult > 0, mult


def unwritten_per_axis(ns: int, nx: int) -> int:
    """Number of (s', x') pairs of one axis that no tuple reaches."""
    reached = {(sp, xp) for sp, xp, _, _ in axis_tuples(ns, nx)}
    return ns * nx - len(reached)
