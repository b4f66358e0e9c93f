"""The projector kernels' index arithmetic, on the CPU.

A mirror, in NumPy, of the address and index computations of the packing
kernels, the GEMM kernel and the reduction of paper_2003_09133_amd/csrc/
lfbp_project.hip: it checks that every global address they form lies inside
its array, that the workgroup -> tile map is a bijection, and, by running the
mirrored records through a float64 matrix product, that the formulation gives
the oracle's f = H g and g = H' f.  Keep it in step with the kernels.
"""
import functools
import itertools

import numpy as np
import pytest

import lfsynth
import oracle

kThreads, kMT, kNT, kHalf, kStageK, kRec, kRecVec, kXcds = 256, 64, 256, 11, 22, 24, 6, 8


def slot_k(q):
    h = 1 if q >= 12 else 0
    j = q - 12 * h
    return kHalf * h + j if j < kHalf else -1


SLOT_K = np.array([slot_k(q) for q in range(kRec)])


def geom(shape, R, C):
    ns, nt, nx, ny, nz = shape
    Lr, Lc = -(-R // nx), -(-C // ny)
    return dict(ns=ns, nt=nt, nx=nx, ny=ny, nz=nz, hs=(ns - 1) // 2, ht=(nt - 1) // 2, R=R, C=C, Lr=Lr, Lc=Lc,
                M=Lr * Lc, Kr=ns + nx - 1, Kc=nt + ny - 1)


def tile_of_block(b, mtiles, ntiles, splits):
    nb = mtiles * ntiles * splits
    x, q, r = b % kXcds, nb // kXcds, nb % kXcds
    L = x * q + min(x, r) + b // kXcds
    return L % mtiles, (L // mtiles) % ntiles, L // (mtiles * ntiles)


def fwd_stage(g, nzc, s):
    st, zc = divmod(s, nzc)
    sr, tc = divmod(st, g['Kc'])
    sp, tp = sr - (g['nx'] - 1), tc - (g['ny'] - 1)
    e, f = g['hs'] - sp, g['ht'] - tp
    px, py = e % g['nx'], f % g['ny']
    dP, dQ = (e - px) // g['nx'], (f - py) // g['ny']
    # the GEMM's form of the same (a_rsrc_fwd): unsigned division of a biased, never negative index
    ep = g['hs'] + g['nx'] - 1 - sr + g['nx'] * g['ns']
    fq = g['ht'] + g['ny'] - 1 - tc + g['ny'] * g['nt']
    assert 0 <= ep < 2 ** 32 and 0 <= fq < 2 ** 32
    assert (ep % g['nx'], ep // g['nx'] - g['ns']) == (px, dP) and (fq % g['ny'], fq // g['ny'] - g['nt']) == (py, dQ)
    return sp, tp, zc, px, py, dP, dQ


def class_boxes(g):
    """Box shape of the forward columns (mirror of class_boxes)."""
    nx, ny, ns, nt = g['nx'], g['ny'], g['ns'], g['nt']
    best, best_cost = None, None
    for bu in range(1, min(nx, 64) + 1):
        bv = min(ny, 64 // bu)
        nbu, nbv = -(-nx // bu), -(-ny // bv)
        waves = -(-(nbu * nbv) // 4) * 4
        if waves * 64 > 2 * nx * ny + 256 and bu != min(nx, 64):
            continue
        cost = waves * (ns + bu - 1) * (nt + bv - 1)
        if best is None or cost < best_cost or (cost == best_cost and abs(bu - bv) < abs(best[0] - best[1])):
            best, best_cost = (bu, bv, nbv, nbu * nbv), cost
    return dict(bu=best[0], bv=best[1], nbv=best[2], boxes=best[3])


def class_of_col(cb, nx, ny, n):
    """Column n -> class (u, v), or None for a padding column."""
    b, k = n >> 6, n & 63
    if b >= cb['boxes'] or k >= cb['bu'] * cb['bv']:
        return None
    bi, bj = divmod(b, cb['nbv'])
    du, dv = divmod(k, cb['bv'])
    u, v = bi * cb['bu'] + du, bj * cb['bv'] + dv
    return (u, v) if u < nx and v < ny else None


def col_of_class(cb, u, v):
    bi, bj = u // cb['bu'], v // cb['bv']
    return (bi * cb['nbv'] + bj) * 64 + (u - bi * cb['bu']) * cb['bv'] + (v - bj * cb['bv'])


def fwd_tile_rows(g, cb, mt, box):
    """(count, first) of the window rows box `box` needs for row tile mt
    (mirror of fwd_tile_rows): the rows whose patch-row shift s' = ir - u1
    puts a source row P = nx Lp + hs - s' inside the image for some lenslet
    row Lp of the tile."""
    bi = box // cb['nbv']
    u1 = min(g['nx'], (bi + 1) * cb['bu']) - 1
    Rw = g['ns'] + cb['bu'] - 1
    m_lo, m_hi = mt * kMT, min(g['M'] - 1, mt * kMT + kMT - 1)
    lp_lo, lp_hi = m_lo // g['Lc'], m_hi // g['Lc']
    ir_lo = max(0, g['nx'] * lp_lo + g['hs'] - (g['R'] - 1) + u1)
    ir_hi = min(Rw - 1, g['nx'] * lp_hi + g['hs'] + u1)
    return max(0, ir_hi - ir_lo + 1), ir_lo


def fwd_window(g, p, ntile, wave, mt=None):
    """The wavefront's stages (k_gemm, forward), in window order: the box's
    Rw x Cw = (ns + bu - 1) x (nt + bv - 1) patch shifts (only the rows row
    tile mt needs, when mt is given), depth chunk fastest; the column shifts
    by residue b modulo ny, within a residue all row shifts, each with the
    residue's column shifts b, b + ny, ... innermost."""
    cb = p['cb']
    b = ntile * (kNT // 64) + wave
    if b >= cb['boxes']:
        return []
    bi, bj = divmod(b, cb['nbv'])
    u1, v1 = min(g['nx'], (bi + 1) * cb['bu']) - 1, min(g['ny'], (bj + 1) * cb['bv']) - 1
    sr0, tc0 = g['nx'] - 1 - u1, g['ny'] - 1 - v1
    Rw, Cw = g['ns'] + cb['bu'] - 1, g['nt'] + cb['bv'] - 1
    assert sr0 >= 0 and tc0 >= 0 and sr0 + Rw <= g['Kr'] and tc0 + Cw <= g['Kc']
    if mt is not None:
        Rw, ir_lo = fwd_tile_rows(g, cb, mt, b)
        sr0 += ir_lo
        assert Rw == 0 or sr0 + Rw <= g['Kr']
    order = walk_order(Rw, Cw, g['ny'])
    return [((sr0 + ir) * g['Kc'] + tc0 + ic) * p['nzc'] + zc for ir, ic in order for zc in range(p['nzc'])]


@functools.lru_cache(maxsize=None)
def walk_order(Rw, Cw, ny):
    """Window positions (ir, ic) in walk order, checked against the kernel's
    closed form (WindowWalk, with n1 and the divisors by Rw q taken per
    wavefront)."""
    order = [(ir, b + k * ny) for b in range(min(ny, Cw)) for ir in range(Rw) for k in range((Cw - b + ny - 1) // ny)]
    assert sorted(order) == [(ir, ic) for ir in range(Rw) for ic in range(Cw)]
    q0, r0 = divmod(Cw, ny)
    q1, n1 = q0 + 1, r0 * Rw * (q0 + 1)
    for j, (ir, ic) in enumerate(order):
        first = j < n1
        jr, q = (j, q1) if first else (j - n1, q0)
        bq, rem = divmod(jr, Rw * q)
        assert (rem // q, (bq if first else r0 + bq) + (rem % q) * ny) == (ir, ic)
    return tuple(order)


def bwd_window(g, N, stages, ntile):
    """The stages of n tile ntile's wavefronts (k_gemm, backward): a contiguous run."""
    nlo = ntile * kNT
    if nlo >= N:
        return []
    nhi = min(nlo + kNT - 1, N - 1)
    cxlo, cxhi = nlo // g['nz'] // g['ny'], nhi // g['nz'] // g['ny']
    klo, khi = (g['nx'] - 1 - cxhi) * g['Kc'], (g['nx'] - 1 - cxlo + g['ns']) * g['Kc']
    base = klo // kStageK
    out = list(range(base, -(-khi // kStageK)))
    assert out[-1] < stages
    return out


def fwd_plan(g, target_blocks=512):
    """Mirror of fwd_plan: row-tile split counts in proportion to the window
    rows each tile needs, the work table (first slot per row tile, then the
    workgroups as (row tile, column tile, split))."""
    N = g['nx'] * g['ny']
    cb = class_boxes(g)
    mtiles, ntiles = -(-g['M'] // kMT), -(-(cb['boxes'] * 64) // kNT)
    nzc = -(-g['nz'] // kStageK)
    stages = g['Kr'] * g['Kc'] * nzc
    rows = [max(fwd_tile_rows(g, cb, mt, b)[0] for b in range(cb['boxes'])) for mt in range(mtiles)]
    rmax = max(rows)

    def count(c, mt):
        return 1 if rmax == 0 else max(1, -(-rows[mt] * c // rmax))

    cap = max(1, min(64, stages // 64))
    splits = 1
    for c in range(2, cap + 1):
        if sum(count(c, mt) for mt in range(mtiles)) * ntiles > target_blocks:
            break
        splits = c
    prefix = [0]
    for mt in range(mtiles):
        prefix.append(prefix[-1] + count(splits, mt))
    wgs = [(mt, nt, j) for j in range(splits) for nt in range(ntiles) for mt in range(mtiles) if j < count(splits, mt)]
    assert splits <= 64 and mtiles * ntiles < 1 << 26          # the table's (tile << 6) | split words
    assert sorted(wgs) == sorted((mt, nt, j) for mt in range(mtiles) for nt in range(ntiles)
                                 for j in range(prefix[mt + 1] - prefix[mt]))
    padP, padQ = (g['hs'] + g['nx'] - 1) // g['nx'], (g['ht'] + g['ny'] - 1) // g['ny']
    return dict(N=N, mtiles=mtiles, ntiles=ntiles, Mpad=mtiles * kMT, Npad=ntiles * kNT, nzc=nzc, stages=stages,
                splits=splits, prefix=prefix, wgs=wgs, slots=prefix[-1], padP=padP, padQ=padQ,
                LRp=g['Lr'] + 2 * padP, LCp=g['Lc'] + 2 * padQ, cb=cb)


def check_blocks(mtiles, ntiles, splits):
    seen = {tile_of_block(b, mtiles, ntiles, splits) for b in range(mtiles * ntiles * splits)}
    assert seen == set(itertools.product(range(mtiles), range(ntiles), range(splits)))


def to_blocks(rec):
    """Records [blocks][rows][24] -> the kernels' storage: per block, vector
    plane v, record, half h, 4 floats (float index ((b*3+v)*rows+r)*8+4h+c)."""
    nb, rows, _ = rec.shape
    return np.ascontiguousarray(rec.reshape(nb, rows, 2, 3, 4).transpose(0, 3, 1, 2, 4)).ravel()


def read_records(flat, base4, lane4, vstride4):
    """What the GEMM's lanes read: 16-byte vectors at base4 + lane4 + v*vstride4
    for the halves h = 0, 1 (lane4 without the half) -> records [n][24]."""
    out = np.empty(lane4.shape + (kRec,))
    for h in range(2):
        for v in range(3):
            idx4 = base4 + 2 * lane4 + h + v * vstride4
            assert idx4.min() >= 0 and (idx4.max() + 1) * 4 <= flat.size
            out[..., 12 * h + 4 * v:12 * h + 4 * v + 4] = flat[(idx4[..., None] * 4 + np.arange(4))]
    return out


def split_ranges(stages, splits):
    return [(stages * k // splits, stages * (k + 1) // splits) for k in range(splits)]


def forward_mirror(H, gvol, target_blocks=512):
    """Records and GEMM of the forward kernel; returns f (float64)."""
    ns, nt, nx, ny, nz = H.shape
    _, R, C = gvol.shape
    g = geom(H.shape, R, C)
    p = fwd_plan(g, target_blocks)
    cell = nx * ny * nz
    Hf = H.astype(np.float64).ravel()
    gT = np.ascontiguousarray(np.transpose(gvol, (1, 2, 0))).astype(np.float64).ravel()
    # k_pack_fwd_a: gS[pxy][LP][LQ][zc][slot]
    pxy, LP, LQ, zc, q = np.meshgrid(np.arange(nx * ny), np.arange(p['LRp']), np.arange(p['LCp']),
                                     np.arange(p['nzc']), np.arange(kRec), indexing='ij')
    P, Q = nx * (LP - p['padP']) + pxy // ny, ny * (LQ - p['padQ']) + pxy % ny
    k = SLOT_K[q]
    z = zc * kStageK + k
    ok = (P >= 0) & (P < R) & (Q >= 0) & (Q < C) & (k >= 0) & (z < nz)
    idx = np.where(ok, (P * C + Q) * nz + z, 0)
    assert idx.min() >= 0 and idx.max() < gT.size
    arows = p['LRp'] * p['LCp']
    # blocks (px, py, zc) of LRp*LCp records
    gS = to_blocks(np.where(ok, gT[idx], 0.0).transpose(0, 3, 1, 2, 4).reshape(nx * ny * p['nzc'], arows, kRec))
    # k_pack_fwd_b: Bp[s][n][slot]
    s_all = np.arange(p['stages'])
    sp, tp, zcs, pxs, pys, dP, dQ = (np.array(v) for v in zip(*[fwd_stage(g, p['nzc'], s) for s in s_all]))
    n = np.arange(p['Npad'])
    cls = [class_of_col(p['cb'], nx, ny, c) for c in n]
    colok = np.array([c is not None for c in cls])
    u = np.array([c[0] if c else 0 for c in cls])
    v = np.array([c[1] if c else 0 for c in cls])
    assert sorted(c for c in cls if c) == [(a, b) for a in range(nx) for b in range(ny)]   # each class once
    S, Nn, Qs = np.meshgrid(s_all, n, np.arange(kRec), indexing='ij')
    kk = SLOT_K[Qs]
    zz = zcs[S] * kStageK + kk
    su, tv = sp[S] + u[Nn], tp[S] + v[Nn]
    okb = colok[Nn] & (su >= 0) & (su < ns) & (tv >= 0) & (tv < nt) & (kk >= 0) & (zz < nz)
    idx = np.where(okb, (su * nt + tv) * cell + (pxs[S] * ny + pys[S]) * nz + zz, 0)
    assert idx.min() >= 0 and idx.max() < H.size
    Bp = to_blocks(np.where(okb, Hf[idx], 0.0))          # blocks = stages, Npad records each
    # GEMM: every workgroup's lanes and stages, from the work table
    m = np.arange(p['Mpad'])
    mc = np.minimum(m, g['M'] - 1)
    lane_a = (mc // g['Lc']) * p['LCp'] + mc % g['Lc']             # record of the lane's lenslet
    abase = ((pxs * ny + pys) * p['nzc'] + zcs) * kRecVec * arows + 2 * ((dP + p['padP']) * p['LCp'] + dQ + p['padQ'])
    lane_b = np.arange(p['Npad'])
    use = SLOT_K >= 0                                               # the MFMA steps read slots 0-10 and 12-22
    okb_s = okb.any(axis=2)                                         # [stage][column] holds a nonzero slot
    for ntile in range(p['ntiles']):
        for wave in range(kNT // 64):
            cols = np.arange(ntile * kNT + 64 * wave, ntile * kNT + 64 * wave + 64)
            win = fwd_window(g, p, ntile, wave)
            assert len(set(win)) == len(win) and all(0 <= st < p['stages'] for st in win)
            outside = np.ones(p['stages'], bool)
            outside[win] = False
            assert not okb_s[np.ix_(outside, cols)].any(), "nonzero B record outside the window"
            for mt in range(p['mtiles']):
                # the rows a row tile drops hold only zero A records for its lenslets
                rows_t = lane_a[mt * kMT:(mt + 1) * kMT]
                kept = set(fwd_window(g, p, ntile, wave, mt))
                assert kept <= set(win)
                for st in set(win) - kept:
                    assert not read_records(gS, abase[st], rows_t, 2 * arows).any(), "dropped row with nonzero A"
    partial = np.zeros((p['slots'], kMT, p['Npad']))
    for mt, ntile, j in p['wgs']:
        nsplit = p['prefix'][mt + 1] - p['prefix'][mt]
        slot = p['prefix'][mt] + j
        assert 0 <= j < nsplit and slot < p['slots']
        rows_t = lane_a[mt * kMT:(mt + 1) * kMT]
        for wave in range(kNT // 64):
            cols = np.arange(ntile * kNT + 64 * wave, ntile * kNT + 64 * wave + 64)
            win = fwd_window(g, p, ntile, wave, mt)
            b, e = len(win) * j // nsplit, len(win) * (j + 1) // nsplit
            for st in win[b:e]:
                Arec = read_records(gS, abase[st], rows_t, 2 * arows)
                Brec = read_records(Bp, st * kRecVec * p['Npad'], lane_b[cols], 2 * p['Npad'])
                partial[slot][:, cols] += Arec[:, use] @ Brec[:, use].T
    # k_fwd_reduce: a pixel's lenslet row m sums its row tile's slots
    pp, qq = np.meshgrid(np.arange(R), np.arange(C), indexing='ij')
    mm = (pp // nx) * g['Lc'] + qq // ny
    nn = np.vectorize(lambda a, b: col_of_class(p['cb'], a, b))(pp % nx, qq % ny)
    assert mm.max() < p['Mpad'] and nn.max() < p['Npad']
    tiles = np.array([partial[p['prefix'][mt]:p['prefix'][mt + 1]].sum(axis=0) for mt in range(p['mtiles'])])
    return tiles[mm // kMT, mm % kMT, nn]


def backward_mirror(Ht, f):
    """Records and GEMM of the backprojection kernel; returns g (float64)."""
    ns, nt, nx, ny, nz = Ht.shape
    R, C = f.shape
    g = geom(Ht.shape, R, C)
    N = nx * ny * nz
    mtiles, ntiles = -(-g['M'] // kMT), -(-N // kNT)
    Mpad, Npad = mtiles * kMT, ntiles * kNT
    K = g['Kr'] * g['Kc']
    stages = -(-K // kStageK)
    cell = nx * ny * nz
    Hf = Ht.astype(np.float64).ravel()
    ff = f.astype(np.float64).ravel()
    S, Qs = np.meshgrid(np.arange(stages), np.arange(kRec), indexing='ij')
    kk = SLOT_K[Qs]
    k = S * kStageK + kk
    kc = np.where(kk >= 0, k, 0)
    ri = kc // g['Kc']
    r, r2 = ri - (nx - 1), kc - ri * g['Kc'] - (ny - 1)
    kok = (kk >= 0) & (k < K)
    # k_pack_bwd_a: Ap[s][m][slot]
    m = np.arange(Mpad)
    LP, LQ = m // g['Lc'], m % g['Lc']
    P = nx * LP[None, :, None] + g['hs'] - r[:, None, :]
    Q = ny * LQ[None, :, None] + g['ht'] - r2[:, None, :]
    oka = (m[None, :, None] < g['M']) & kok[:, None, :] & (P >= 0) & (P < R) & (Q >= 0) & (Q < C)
    idx = np.where(oka, P * C + Q, 0)
    assert idx.min() >= 0 and idx.max() < R * C
    Ap = to_blocks(np.where(oka, ff[idx], 0.0))
    # k_pack_bwd_b: Bp[s][n][slot]
    n = np.arange(Npad)
    cz, z = n // nz, n % nz
    cx, cy = cz // ny, cz % ny
    x, y = (g['hs'] - r) % nx, (g['ht'] - r2) % ny
    rx, ry = r[:, None, :] + cx[None, :, None], r2[:, None, :] + cy[None, :, None]
    okb = (n[None, :, None] < N) & kok[:, None, :] & (rx >= 0) & (rx < ns) & (ry >= 0) & (ry < nt)
    idx = (rx * nt + ry) * cell + (x[:, None, :] * ny + y[:, None, :]) * nz + z[None, :, None]
    idx = np.where(okb, idx, 0)
    assert idx.min() >= 0 and idx.max() < Ht.size
    Bp = to_blocks(np.where(okb, Hf[idx], 0.0))
    check_blocks(mtiles, ntiles, 1)
    use = SLOT_K >= 0
    G = np.zeros((Mpad, Npad))
    okb_s = okb.any(axis=2)
    for ntile in range(ntiles):
        cols = np.arange(ntile * kNT, ntile * kNT + kNT)
        win = bwd_window(g, N, stages, ntile)
        outside = np.ones(stages, bool)
        outside[win] = False
        assert not okb_s[np.ix_(outside, cols)].any(), "nonzero B record outside the window"
        for s in win:
            Arec = read_records(Ap, s * kRecVec * Mpad, np.arange(Mpad), 2 * Mpad)
            Brec = read_records(Bp, s * kRecVec * Npad, cols, 2 * Npad)
            G[:, cols] += Arec[:, use] @ Brec[:, use].T
    # epilogue: (m, n) -> g[z][nx LP + cx][ny LQ + cy]
    out = np.zeros((nz, R, C))
    mm, nn = np.meshgrid(np.arange(g['M']), np.arange(N), indexing='ij')
    Pp = nx * (mm // g['Lc']) + (nn // nz) // ny
    Qq = ny * (mm % g['Lc']) + (nn // nz) % ny
    ok = (Pp < R) & (Qq < C)
    out[(nn % nz)[ok], Pp[ok], Qq[ok]] = G[:g['M'], :N][ok]
    return out


SHAPES = [((15, 15, 3, 3, 2), 12, 200), ((9, 9, 1, 1, 2), 10, 70), ((11, 9, 3, 3, 3), 9, 140),
          ((15, 15, 3, 3, 3), 21, 21), ((15, 15, 3, 3, 3), 20, 23), ((9, 7, 3, 5, 2), 12, 10),
          ((5, 5, 5, 5, 1), 7, 8), ((7, 9, 1, 1, 3), 11, 9), ((1, 1, 1, 1, 2), 4, 5), ((3, 3, 7, 7, 2), 14, 21),
          ((21, 21, 3, 3, 9), 8, 7), ((5, 5, 3, 3, 2), 9, 12), ((3, 3, 1, 1, 2), 5, 6),
          ((9, 9, 3, 3, 30), 10, 10), ((5, 5, 3, 3, 45), 6, 7), ((3, 3, 3, 3, 23), 7, 5), ((7, 5, 3, 1, 22), 9, 4),
          ((21, 21, 17, 17, 2), 40, 36), ((11, 13, 5, 7, 30), 23, 30)]


@pytest.mark.parametrize("shape,R,C", SHAPES)
def test_projector_mirror_bounds_and_values(shape, R, C):
    H = lfsynth.uniform_f32(shape, 1)
    gv = lfsynth.uniform_f32((shape[4], R, C), 2)
    f = lfsynth.uniform_f32((R, C), 3)
    ref = oracle.forward(H, gv)
    assert np.allclose(forward_mirror(H, gv), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    ref = oracle.backward(H, f)               # from H; the kernel reads H'
    got = backward_mirror(oracle.Ht_rows(H), f)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("target_blocks", [1, 16, 160, 512, 608])
def test_forward_mirror_split_counts(target_blocks):
    """Every split count covers the stages exactly once."""
    shape, R, C = (9, 7, 3, 5, 2), 12, 10
    H = lfsynth.uniform_f32(shape, 4)
    gv = lfsynth.uniform_f32((shape[4], R, C), 5)
    ref = oracle.forward(H, gv)
    assert np.allclose(forward_mirror(H, gv, target_blocks=target_blocks), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_workgroup_map_is_a_bijection():
    for mt, nt, sp in itertools.product([1, 3, 25, 26], [1, 2, 19], [1, 5, 8, 20]):
        check_blocks(mt, nt, sp)


@pytest.mark.parametrize("shape,R,C", [((165, 165, 15, 15, 21), 600, 600), ((165, 165, 15, 15, 21), 120, 120),
                                       ((45, 45, 15, 15, 5), 97, 120), ((345, 345, 15, 15, 51), 330, 345)])
def test_large_shapes_record_addresses(shape, R, C):
    """Shapes of the GPU tests and the projector workload: the lanes' record
    addresses at every forward stage stay inside the phase-split copy of g."""
    g = geom(shape, R, C)
    p = fwd_plan(g)
    arows = p['LRp'] * p['LCp']
    gS_vecs = shape[2] * shape[3] * p['nzc'] * arows * kRecVec
    mc = np.minimum(np.arange(p['Mpad']), g['M'] - 1)
    lane = 2 * ((mc // g['Lc']) * p['LCp'] + mc % g['Lc'])
    st = np.array([fwd_stage(g, p['nzc'], s) for s in range(p['stages'])])
    _, _, zc, px, py, dP, dQ = st.T
    base = ((px * shape[3] + py) * p['nzc'] + zc) * kRecVec * arows + 2 * ((dP + p['padP']) * p['LCp'] + dQ + p['padQ'])
    assert base.min() + lane.min() >= 0 and base.max() + lane.max() + 1 + 2 * 2 * arows < gS_vecs
    # the shift never carries a lane's record out of its (px, py, zc) block
    blk = ((px * shape[3] + py) * p['nzc'] + zc) * kRecVec * arows
    assert np.all(base - blk + lane.max() + 1 < 2 * arows) and np.all(base - blk + lane.min() >= 0)
    # the work table (checked in fwd_plan): every workgroup's slot inside the partial sums
    assert all(p['prefix'][mt] + j < p['slots'] for mt, _, j in p['wgs'])
    if shape == (165, 165, 15, 15, 21) and (R, C) == (600, 600):
        # the projector workload: 21 splits for the 19 row tiles that need every window row, 14, 18 and 20
        # for the three at either edge, 503 workgroups in one round of 512
        assert p['splits'] == 21 and len(p['wgs']) == 503
        counts = [p['prefix'][mt + 1] - p['prefix'][mt] for mt in range(p['mtiles'])]
        assert counts == [14, 18, 20] + [21] * 19 + [20, 18, 14]


def grad_window(g, Mg, N, mt, nt_, stages):
    """The stages of gradient tile (mt, nt_) (k_gemm, gradient with respect
    to H): none when no entry of the tile is kept (no pair 0 <= r - x < ns),
    else the run of stages over the lenslet rows LP with nx LP in
    [hs - rhi, R - 1 + hs - rlo]."""
    nx, ny, nz, ns = g['nx'], g['ny'], g['nz'], g['ns']
    m0, nlo = mt * kMT, nt_ * kNT
    rlo, rhi = m0 // g['Kc'], min(m0 + kMT - 1, Mg - 1) // g['Kc']
    nhi = min(nlo + kNT - 1, N - 1)
    xlo, xhi = nlo // nz // ny, nhi // nz // ny
    if m0 >= Mg or rhi < xlo or rlo - xhi > ns - 1:
        return []
    d, e = g['hs'] - rhi, g['R'] - 1 + g['hs'] - rlo
    lp_lo = (d + nx - 1) // nx if d > 0 else 0
    lp_hi = -1 if e < 0 else min(g['Lr'] - 1, e // nx)
    if lp_lo > lp_hi:
        return []
    base = lp_lo * g['Lc'] // kStageK
    end = -(-min(g['M'], (lp_hi + 1) * g['Lc']) // kStageK)
    assert 0 <= base <= end <= stages
    return list(range(base, end))


def grad_mirror(shape, w, gv):
    """Records, GEMM and epilogue of the gradient with respect to H."""
    ns, nt, nx, ny, nz = shape
    R, C = w.shape
    g = geom(shape, R, C)
    Mg = g['Kr'] * g['Kc']
    N = nx * ny * nz
    mtiles, ntiles = -(-Mg // kMT), -(-N // kNT)
    Mpad, Npad = mtiles * kMT, ntiles * kNT
    stages = -(-g['M'] // kStageK)
    wf, gf = w.astype(np.float64).ravel(), gv.astype(np.float64).ravel()
    S, Qs = np.meshgrid(np.arange(stages), np.arange(kRec), indexing='ij')
    kk = SLOT_K[Qs]
    k = S * kStageK + kk
    kc = np.where(kk >= 0, k, 0)
    LP, LQ = kc // g['Lc'], kc % g['Lc']
    kok = (kk >= 0) & (k < g['M'])
    # k_pack_gh_a: rows m = (r, r2)
    m = np.arange(Mpad)
    r, r2 = m // g['Kc'], m % g['Kc']
    pp = nx * LP[:, None, :] + r[None, :, None] - g['hs']
    qq = ny * LQ[:, None, :] + r2[None, :, None] - g['ht']
    oka = (m[None, :, None] < Mg) & kok[:, None, :] & (pp >= 0) & (pp < R) & (qq >= 0) & (qq < C)
    idx = np.where(oka, pp * C + qq, 0)
    assert idx.min() >= 0 and idx.max() < R * C
    Ap = to_blocks(np.where(oka, wf[idx], 0.0))
    # k_pack_gh_b: columns n = (x, y, z)
    n = np.arange(Npad)
    cz, z = n // nz, n % nz
    x, y = cz // ny, cz % ny
    P = nx * LP[:, None, :] + x[None, :, None]
    Q = ny * LQ[:, None, :] + y[None, :, None]
    okb = (n[None, :, None] < N) & kok[:, None, :] & (P < R) & (Q < C)
    idx = np.where(okb, z[None, :, None] * R * C + P * C + Q, 0)
    assert idx.min() >= 0 and idx.max() < gf.size
    Bp = to_blocks(np.where(okb, gf[idx], 0.0))
    check_blocks(mtiles, ntiles, 1)
    use = SLOT_K >= 0
    E = np.zeros((Mpad, Npad))
    for mt in range(mtiles):
        for nt_ in range(ntiles):
            m0, nlo = mt * kMT, nt_ * kNT
            rows, cols = np.arange(m0, m0 + kMT), np.arange(nlo, nlo + kNT)
            win = grad_window(g, Mg, N, mt, nt_, stages)
            # the stages outside the window hold only zero A records for the tile's rows (a tile
            # with no kept entry computes nothing, and none of its entries is kept below)
            rlo, rhi = m0 // g['Kc'], min(m0 + kMT - 1, Mg - 1) // g['Kc']
            xlo, xhi = nlo // nz // ny, min(nlo + kNT - 1, N - 1) // nz // ny
            if not (m0 >= Mg or rhi < xlo or rlo - xhi > ns - 1):
                for st in sorted(set(range(stages)) - set(win)):
                    assert not read_records(Ap, st * kRecVec * Mpad, rows, 2 * Mpad).any(), "skipped stage with nonzero A"
            for st in win:
                Arec = read_records(Ap, st * kRecVec * Mpad, rows, 2 * Mpad)
                Brec = read_records(Bp, st * kRecVec * Npad, cols, 2 * Npad)
                E[m0:m0 + kMT, nlo:nlo + kNT] += Arec[:, use] @ Brec[:, use].T
    # epilogue: (m, n) -> dH[r - x][r2 - y][x][y][z] when inside the patch
    dH = np.full(shape, np.nan)
    mm, nn = np.meshgrid(np.arange(Mg), np.arange(N), indexing='ij')
    rr, rr2 = mm // g['Kc'], mm % g['Kc']
    xx, yy, zz = (nn // nz) // ny, (nn // nz) % ny, nn % nz
    sp, tp = rr - xx, rr2 - yy
    ok = (sp >= 0) & (sp < ns) & (tp >= 0) & (tp < nt)
    flat = (((sp * nt + tp) * nx + xx) * ny + yy) * nz + zz
    assert len(np.unique(flat[ok])) == ok.sum() == np.prod(shape)     # every entry exactly once
    dH.reshape(-1)[flat[ok]] = E[:Mg, :N][ok]
    return dH


@pytest.mark.parametrize("shape,R,C", [((9, 9, 3, 3, 2), 90, 60), ((15, 15, 1, 1, 2), 40, 50),
                                       ((15, 15, 3, 3, 3), 21, 21), ((9, 7, 3, 5, 2), 12, 10), ((5, 5, 5, 5, 1), 7, 8),
                                       ((7, 9, 1, 1, 3), 11, 9), ((21, 21, 17, 17, 2), 40, 36),
                                       ((3, 3, 7, 7, 2), 14, 21), ((9, 9, 3, 3, 30), 10, 10)])
def test_grad_psf_mirror(shape, R, C):
    w = lfsynth.uniform_f32((R, C), 11)
    gv = lfsynth.uniform_f32((shape[4], R, C), 12)
    ref = oracle.grad_psf(shape, w, gv)
    got = grad_mirror(shape, w, gv)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
