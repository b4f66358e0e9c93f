"""CPU mirror of the 16-column forward projection (csrc/lfbp_project.hip:
fwd16_plan, k_pack16_a, k_pack16_b, k_fwd16, k_fwd16_reduce) in NumPy: the
host plan (work items, splits, slots), every lane's record offsets and box
mask as the kernel steps through its stages, and the float64 product of the
mirrored records, reduced as the kernel's reduction does, against the
oracle's forward projection (Sec. 2.1, Eq. 1).  Also: every record read of a
live lane lies inside its block, every window position and depth chunk of a
(row tile, strip, box group) is visited exactly once over the splits, and the
steps the kernel skips (boxes masked off for a group, dropped patch rows)
would only have multiplied zeros."""
import math

import numpy as np
import pytest

import lfsynth
import oracle

KMT, BU, BV, WB, CH = 64, 3, 5, 5, 7


def geom(shape, R, C):
    ns, nt, nx, ny, nz = shape
    g = dict(ns=ns, nt=nt, nx=nx, ny=ny, nz=nz, hs=(ns - 1) // 2, ht=(nt - 1) // 2, R=R, C=C)
    g["Lr"], g["Lc"] = -(-R // nx), -(-C // ny)
    g["M"] = g["Lr"] * g["Lc"]
    g["Kr"], g["Kt"] = ns + nx - 1, nt + ny - 1
    return g


def plan16(shape, R, C, target=512):
    g = geom(shape, R, C)
    P = dict(g=g)
    nx, ny, ns, nt, hs, ht = g["nx"], g["ny"], g["ns"], g["nt"], g["hs"], g["ht"]
    P["nch"] = -(-g["nz"] // CH)
    P["nstrips"], P["nbox"] = -(-ny // BV), -(-nx // BU)
    P["ngroups"] = -(-P["nbox"] // WB)
    P["padP"], P["padQ"] = (ns - 1 - hs + nx - 1) // nx, (nt - 1 - ht + ny - 1) // ny
    P["LRp"] = g["Lr"] + P["padP"] + (hs + nx - 1) // nx
    P["LCp"] = g["Lc"] + P["padQ"] + (ht + ny - 1) // ny
    P["ncols"] = P["nstrips"] * P["nbox"] * 16
    mtiles = -(-g["M"] // KMT)
    P["mtiles"] = mtiles
    rlo, nrow, rows = {}, {}, []
    for mt in range(mtiles):
        lp_lo, lp_hi = (KMT * mt) // g["Lc"], min(g["M"] - 1, KMT * mt + KMT - 1) // g["Lc"]
        best = 0
        for h in range(P["ngroups"]):
            lo = max(-min(nx - 1, BU * WB * h + BU * WB - 1), nx * lp_lo + hs - (R - 1))
            hi = min(ns - 1 - BU * WB * h, nx * lp_hi + hs)
            rlo[mt, h], nrow[mt, h] = lo, max(0, hi - lo + 1)
            best = max(best, nrow[mt, h])
        rows.append(best)
    rows_max = max(rows)

    def window(j):
        return -min(ny - 1, BV * j + BV - 1), nt - 1 - BV * j

    def residues(j):
        c_lo, c_hi = window(j)
        out = []
        for rho in range(ny):
            tfirst = c_lo + (rho - c_lo) % ny
            out.append((tfirst, (c_hi - tfirst) // ny + 1 if tfirst <= c_hi else 0))
        return out

    def stages(mt, j, h):
        return sum(P["nch"] * ((nrow[mt, h] * nc + 3) // 4) for _, nc in residues(j))

    Tmax = max(stages(mt, 0, h) for mt in range(mtiles) for h in range(P["ngroups"]))

    def count(c, mt):
        return 1 if rows_max == 0 else max(1, -(-rows[mt] * c // rows_max))

    per = P["nstrips"] * P["ngroups"]
    cap = max(1, min(64, Tmax // 64))
    S = 1
    for c in range(2, cap + 1):
        if -(-sum(count(c, mt) for mt in range(mtiles)) * per // 4) > target:
            break
        S = c
    tab = [0]
    for mt in range(mtiles):
        tab.append(tab[-1] + count(S, mt))
    items = []
    for k in range(max(count(S, mt) for mt in range(mtiles))):
        for j in range(P["nstrips"]):
            for h in range(P["ngroups"]):
                for mt in range(mtiles):
                    cnt = count(S, mt)
                    if k >= cnt:
                        continue
                    T = stages(mt, j, h)
                    items.append(dict(mt=mt, j=j, h=h, r_lo=rlo[mt, h], nrows=nrow[mt, h], st0=T * k // cnt,
                                      st1=T * (k + 1) // cnt, slot=tab[mt] + k))
    P.update(S=S, tab=tab, items=items, residues=residues, window=window, stages=stages)
    return P


def pack_a(P, gvol):
    """A16 records [px][py][chunk][LP'][LQ'][8] (float64)."""
    g = P["g"]
    nx, ny, R, C, nz = g["nx"], g["ny"], g["R"], g["C"], g["nz"]
    A = np.zeros((nx, ny, P["nch"], P["LRp"], P["LCp"], 8))
    for px in range(nx):
        for py in range(ny):
            for LP in range(P["LRp"]):
                Pp = nx * (LP - P["padP"]) + px
                if not 0 <= Pp < R:
                    continue
                for LQ in range(P["LCp"]):
                    Q = ny * (LQ - P["padQ"]) + py
                    if 0 <= Q < C:
                        col = gvol[:, Pp, Q]
                        for c in range(P["nch"]):
                            d = col[CH * c:CH * c + CH]
                            A[px, py, c, LP, LQ, :len(d)] = d
    return A


def pack_b(P, H):
    """B16 records [s'+nx-1][t'+ny-1][chunk][strip][box][n][8] (float64)."""
    g = P["g"]
    ns, nt, nx, ny, hs, ht = g["ns"], g["nt"], g["nx"], g["ny"], g["hs"], g["ht"]
    B = np.zeros((g["Kr"], g["Kt"], P["nch"], P["nstrips"], P["nbox"], 16, 8))
    for sr in range(g["Kr"]):
        sp = sr - (nx - 1)
        for tc in range(g["Kt"]):
            tp = tc - (ny - 1)
            x, y = (hs - sp) % nx, (ht - tp) % ny
            for j in range(P["nstrips"]):
                for bi in range(P["nbox"]):
                    for n in range(15):
                        u, v = BU * bi + n // BV, BV * j + n % BV
                        if u < nx and v < ny and 0 <= sp + u < ns and 0 <= tp + v < nt:
                            col = H[sp + u, tp + v, x, y, :]
                            for c in range(P["nch"]):
                                d = col[CH * c:CH * c + CH]
                                B[sr, tc, c, j, bi, n, :len(d)] = d
    return B


def run_items(P, A, B, check_zero=True):
    """The kernel's walk for every item: partial sums per slot, and the checks."""
    g = P["g"]
    nx, ny, hs, ht, ns = g["nx"], g["ny"], g["hs"], g["ht"], g["ns"]
    Af = A.reshape(-1, 8)
    Bf = B.reshape(-1, 8)
    part = np.zeros((P["tab"][-1], KMT, P["ncols"]))
    visits = {}
    lanes_m = np.arange(64)
    for it in P["items"]:
        mt, j, h, r_lo, nrows = it["mt"], it["j"], it["h"], it["r_lo"], it["nrows"]
        res = P["residues"](j)
        # lane lenslets: rows 16 k + n of the tile
        m = KMT * mt + lanes_m
        Lp, Lq = m // g["Lc"], m % g["Lc"]
        live_m = m < g["M"]
        # decode the first stage
        rem, rho = it["st0"], 0
        while rho < ny and rem >= P["nch"] * ((nrows * res[rho][1] + 3) // 4):
            rem -= P["nch"] * ((nrows * res[rho][1] + 3) // 4)
            rho += 1
        grp, c = divmod(rem, P["nch"])
        for st in range(it["st0"], it["st1"]):
            tfirst, ncols = res[rho]
            Ppos = nrows * ncols
            pos = 4 * grp + np.arange(4)
            ok = pos < Ppos
            ri, ci = pos // max(1, ncols), pos % max(1, ncols)
            sp, tp = r_lo + ri, tfirst + ny * ci
            es, et = hs - sp + nx * P["padP"], ht - tp + ny * P["padQ"]
            qs, px, qt, py = es // nx, es % nx, et // ny, et % ny
            # box mask from the rows of the group's first and last live position
            p3 = min(4 * grp + 3, Ppos - 1)
            smin, smax = r_lo + (4 * grp) // ncols, r_lo + p3 // ncols
            mask = [WB * h + i < P["nbox"] and smin <= ns - 1 - BU * (WB * h + i) and
                    smax >= -min(nx - 1, BU * (WB * h + i) + BU - 1) for i in range(WB)]
            for q in range(4):
                if not ok[q]:
                    continue
                visits[(mt, j, h, sp[q], tp[q], c)] = visits.get((mt, j, h, sp[q], tp[q], c), 0) + 1
                # A records of the 64 lanes' lenslets at this position
                ia = (((px[q] * ny + py[q]) * P["nch"] + c) * P["LRp"] + (Lp + qs[q])) * P["LCp"] + (Lq + qt[q])
                assert (ia[live_m] >= 0).all() and (ia[live_m] < len(Af)).all()
                a = np.where(live_m[:, None], Af[np.clip(ia, 0, len(Af) - 1)], 0.0)[:, :CH]
                pidx = (sp[q] + nx - 1) * g["Kt"] + (tp[q] + ny - 1)
                for i in range(WB):
                    bi = WB * h + i
                    if bi >= P["nbox"]:
                        continue
                    ib = ((pidx * P["nch"] + c) * P["nstrips"] + j) * P["nbox"] + bi
                    assert 0 <= ib * 16 and ib * 16 + 15 < len(Bf)
                    b = Bf[ib * 16:ib * 16 + 16, :CH]
                    if not mask[i]:
                        assert not b.any(), "a masked-off box would have had nonzero B records"
                        continue
                    part[it["slot"], :, (j * P["nbox"] + bi) * 16:(j * P["nbox"] + bi) * 16 + 16] += a @ b.T
            # advance the walk
            c += 1
            if c == P["nch"]:
                c = 0
                grp += 1
                if grp >= (Ppos + 3) // 4:
                    grp = 0
                    rho += 1
                    while rho < ny and res[rho][1] == 0:
                        rho += 1
    # every (row tile, strip, group) window position and chunk once, rows outside
    # the tile's kept range only with zero A records
    for (mt, j, h), _ in {(i["mt"], i["j"], i["h"]): 0 for i in P["items"]}.items():
        it = next(i for i in P["items"] if (i["mt"], i["j"], i["h"]) == (mt, j, h))
        c_lo, c_hi = P["window"](j)
        for sp in range(it["r_lo"], it["r_lo"] + it["nrows"]):
            for tp in range(c_lo, c_hi + 1):
                for c in range(P["nch"]):
                    assert visits.get((mt, j, h, sp, tp, c)) == 1, (mt, j, h, sp, tp, c)
    return part


def reduce16(P, part):
    g = P["g"]
    f = np.zeros((g["R"], g["C"]))
    for p in range(g["R"]):
        for q in range(g["C"]):
            Lp, u, Lq, v = p // g["nx"], p % g["nx"], q // g["ny"], q % g["ny"]
            m = Lp * g["Lc"] + Lq
            mt, r = divmod(m, KMT)
            bi, j = u // BU, v // BV
            col = (j * P["nbox"] + bi) * 16 + (u - BU * bi) * BV + (v - BV * j)
            f[p, q] = part[P["tab"][mt]:P["tab"][mt + 1], r, col].sum()
    return f


def dropped_rows_have_zero_a(P, A):
    """Patch rows outside a tile's kept range: the tile's lenslets see only zero A records there."""
    g = P["g"]
    nx, hs = g["nx"], g["hs"]
    for mt in range(P["mtiles"]):
        m = np.arange(KMT * mt, min(g["M"], KMT * mt + KMT))
        Lp = m // g["Lc"]
        for h in range(P["ngroups"]):
            it = next(i for i in P["items"] if (i["mt"], i["h"]) == (mt, h))
            for sp in range(-(nx - 1), g["ns"]):
                if it["r_lo"] <= sp < it["r_lo"] + it["nrows"]:
                    continue
                src = nx * Lp + hs - sp
                assert ((src < 0) | (src >= g["R"]))[:].all() or not (
                    -min(nx - 1, BU * WB * h + BU * WB - 1) <= sp <= g["ns"] - 1 - BU * WB * h), (mt, h, sp)


CASES = [((9, 9, 3, 3, 5), 12, 12), ((15, 15, 3, 5, 9), 20, 25), ((11, 7, 5, 3, 16), 17, 13),
         ((7, 9, 1, 1, 8), 9, 11), ((9, 13, 17, 5, 3), 40, 14), ((5, 5, 3, 3, 1), 30, 31),
         ((13, 11, 9, 11, 7), 38, 47)]


@pytest.mark.parametrize("shape,R,C", CASES)
def test_fwd16_mirror_matches_oracle(shape, R, C):
    P = plan16(shape, R, C)
    H = lfsynth.uniform_f32(shape, 11).astype(np.float64)
    gvol = lfsynth.uniform_f32((shape[4], R, C), 12).astype(np.float64)
    A, B = pack_a(P, gvol), pack_b(P, H)
    part = run_items(P, A, B)
    f = reduce16(P, part)
    ref = oracle.forward(H.astype(np.float32), gvol.astype(np.float32))
    assert np.abs(f - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    dropped_rows_have_zero_a(P, A)


def test_fwd16_plan_of_the_projector_workload():
    """600 x 600 px, H[165,165,15,15,21]: 28 splits at most, 498 workgroups of four
    wavefronts (one round of 512), row tiles at the image's top and bottom edge
    with fewer splits, every wavefront's stages a contiguous run of its walk."""
    P = plan16((165, 165, 15, 15, 21), 600, 600)
    assert (P["nch"], P["nstrips"], P["nbox"], P["ngroups"], P["ncols"]) == (3, 3, 5, 1, 240)
    assert P["S"] == 28 and -(-len(P["items"]) // 4) == 498
    counts = [P["tab"][mt + 1] - P["tab"][mt] for mt in range(P["mtiles"])]
    assert counts[0] < counts[12] == 28 and counts[-1] < 28
    for key in {(i["mt"], i["j"], i["h"]) for i in P["items"]}:
        runs = sorted((i["st0"], i["st1"]) for i in P["items"] if (i["mt"], i["j"], i["h"]) == key)
        assert runs[0][0] == 0 and runs[-1][1] == P["stages"](*key)
        assert all(a[1] == b[0] for a, b in zip(runs, runs[1:]))
