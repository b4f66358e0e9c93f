"""Address bounds of the projector kernels, on the CPU.

A mirror, in NumPy, of the index arithmetic of the operand loaders and result
writes of k_fwd_gemm / k_fwd_reduce / k_bwd_gemm (paper_2003_09133_amd/csrc/
lfbp_project.hip): for every lane and every stage of the listed shapes, every
global address the kernels form must lie inside its array.  Keep it in step
with the kernels' loaders.  The forward loaders read 16-byte vectors that
may extend past the run they serve: each must be aligned and share its 16-byte
line with an element of its array, for every alignment of the array, and the
scatter of the vectors into LDS must write every (depth, row/column) slot of
the stage exactly once, from the element the GEMM formulation names.
"""
import itertools

import numpy as np
import pytest

kThreads, kMT, kNT, kFwdZC, kBwdKC = 256, 64, 256, 22, 16
kFwdVPR = (kFwdZC + 3 + 3) // 4
kFwdBSlots = kNT * kFwdVPR // kThreads
kFwdASlots = (kMT * kFwdVPR + kThreads - 1) // kThreads
def geom(shape, R, C):
    ns, nt, nx, ny, nz = shape
    return dict(ns=ns, nt=nt, nx=nx, ny=ny, nz=nz, hs=(ns-1)//2, ht=(nt-1)//2, R=R, C=C,
                Lr=-(-R//nx), Lc=-(-C//ny), M=(-(-R//nx))*(-(-C//ny)), Kr=ns+nx-1, Kc=nt+ny-1)
def imod(a, n): return a % n
def vec_ok(start, size, phase):
    """A 16-byte vector read at element `start` of an fp32 array whose first
    element sits at word `phase` of a 16-byte line: it must be aligned and
    share its line with at least one element of the array (so it stays on a
    page the array occupies)."""
    return (np.all((start + phase) % 4 == 0) and start.max() <= size - 1 and (start + 3).min() >= 0)
def check_fwd(shape, R, C, cus=256, stage_sample=None, phases=(0, 1, 2, 3)):
    g = geom(shape, R, C); ns, nt, nx, ny, nz = shape
    E = ns*nt*nx*ny*nz; N = nx*ny
    mtiles, ntiles = -(-g['M']//kMT), -(-N//kNT)
    nzc = -(-nz//kFwdZC); stages = g['Kr']*g['Kc']*nzc
    want = (2*cus)//(mtiles*ntiles); splits = max(1, min(want, 64, max(1, stages//8)))
    Mpad, Npad = mtiles*kMT, ntiles*kNT
    gT_size = nz*R*C; part_size = splits*Mpad*Npad
    tid = np.arange(kThreads)
    cell = nx*ny*nz
    st_list = range(stages) if stage_sample is None else stage_sample(stages)
    for mt, nt_ in itertools.product(range(mtiles), range(ntiles)):
        m0, n0 = mt*kMT, nt_*kNT
        for stage in st_list:
            st, zc = divmod(stage, nzc); sr, tc = divmod(st, g['Kc']); sp, tp = sr-(nx-1), tc-(ny-1)
            z0 = zc*kFwdZC; zn = min(kFwdZC, nz-z0); x, y = imod(g['hs']-sp, nx), imod(g['ht']-tp, ny)
            sbase = (sp*nt + tp)*cell + (x*ny + y)*nz + z0
            for phase in phases:
                # B: slot e = tid + 256 j -> column nl = e // VPR, vector k = e % VPR
                cover = np.zeros((kNT, kFwdZC), np.int64)
                for j in range(kFwdBSlots):
                    e = tid + j*kThreads; nl, k = e // kFwdVPR, e % kFwdVPR; n = n0 + nl
                    u, v = n // ny, n % ny
                    valid = (n < N) & (sp+u >= 0) & (sp+u < ns) & (tp+v >= 0) & (tp+v < nt)
                    rs = sbase + (u*nt + v)*cell
                    lead = np.where(valid, (rs + phase) & 3, 0)
                    vb = np.where(valid, rs - lead, -phase)
                    kmax = (lead + zn - 1) >> 2
                    kk = np.minimum(k, kmax)
                    assert vec_ok(vb + 4*kk, E, phase), ("B", shape, R, C, stage, phase, j)
                    # the vector holds the run's depths at the positions the store takes them from
                    src = vb + 4*kk
                    for q in range(4):
                        z = 4*k + q - lead
                        inr = (z >= 0) & (z < kFwdZC)
                        live = inr & valid & (z < zn)
                        assert np.all(src[live] + q == rs[live] + z[live])
                        np.add.at(cover, (nl[inr], z[inr]), 1)
                assert np.all(cover == 1), ("B cover", shape, stage)
                # A: 448 slots over 2 per thread
                cover = np.zeros((kMT, kFwdZC), np.int64)
                for j in range(kFwdASlots):
                    e = tid + j*kThreads; ml, k = e // kFwdVPR, e % kFwdVPR; m = m0 + ml
                    Lp, Lq = m // g['Lc'], m % g['Lc']
                    P, Q = nx*Lp + g['hs'] - sp, ny*Lq + g['ht'] - tp
                    valid = (ml < kMT) & (m < g['M']) & (P >= 0) & (P < R) & (Q >= 0) & (Q < C)
                    rs = (P*C + Q)*nz + z0
                    lead = np.where(valid, (rs + phase) & 3, 0)
                    vb = np.where(valid, rs - lead, -phase)
                    kmax = (lead + zn - 1) >> 2
                    kk = np.minimum(k, kmax)
                    assert vec_ok(vb + 4*kk, gT_size, phase), ("A", shape, R, C, stage, phase, j)
                    src = vb + 4*kk
                    for q in range(4):
                        z = 4*k + q - lead
                        inr = (z >= 0) & (z < kFwdZC) & (ml < kMT)
                        live = inr & valid & (z < zn)
                        assert np.all(src[live] + q == rs[live] + z[live])
                        np.add.at(cover, (ml[inr], z[inr]), 1)
                assert np.all(cover == 1), ("A cover", shape, stage)
        # partial writes
        for split in [0, splits-1]:
            li, lk = tid & 31, (tid & 63) >> 5; wave = tid >> 6
            for i, j, r in itertools.product(range(2), range(2), range(16)):
                mm = m0 + 32*i + 8*(r >> 2) + 4*lk + (r & 3); nn = n0 + wave*64 + 32*j + li
                off = (split*Mpad + mm)*Npad + nn
                assert off.min() >= 0 and off.max() < part_size
    # reduce reads
    p = np.arange(R)[:, None]; q = np.arange(C)[None, :]
    mm = (p//nx)*g['Lc'] + q//ny; nn = (p % nx)*ny + q % ny
    assert mm.max() < Mpad and nn.max() < Npad
    return stages, splits
def check_bwd(shape, R, C, kk_sample=None):
    g = geom(shape, R, C); ns, nt, nx, ny, nz = shape
    E = ns*nt*nx*ny*nz; N = nx*ny*nz; K = g['Kr']*g['Kc']; cell = nx*ny*nz
    mtiles, ntiles = -(-g['M']//kMT), -(-N//kNT)
    tid = np.arange(kThreads); stages = -(-K//kBwdKC)
    st_list = range(stages) if kk_sample is None else kk_sample(stages)
    for mt, nt_ in itertools.product(range(mtiles), range(ntiles)):
        m0, n0 = mt*kMT, nt_*kNT
        n = n0 + tid; c = n//nz; cx = np.where(n < N, c//ny, 0); cy = np.where(n < N, c % ny, 0); z = n % nz
        hoff = np.where(n < N, (cx*nt + cy)*cell + z, -1)
        m = m0 + (tid >> 2); P0 = np.where(m < g['M'], nx*(m//g['Lc']) + g['hs'], 0); Q0 = np.where(m < g['M'], ny*(m % g['Lc']) + g['ht'], 0)
        for s in st_list:
            k0 = s*kBwdKC
            for j in range(4):
                k = k0 + 4*(tid & 3) + j
                ri, r2i = k // g['Kc'], k % g['Kc']
                p, q = P0 - (ri-(nx-1)), Q0 - (r2i-(ny-1))
                ok = (m < g['M']) & (k < K) & (p >= 0) & (p < R) & (q >= 0) & (q < C)
                idx = np.where(ok, p*C + q, 0)
                assert idx.min() >= 0 and idx.max() < R*C
            for kk in range(kBwdKC):
                k = k0 + kk; ri, r2i = k // g['Kc'], k % g['Kc']; r, r2 = ri-(nx-1), r2i-(ny-1)
                x, y = imod(g['hs']-r, nx), imod(g['ht']-r2, ny)
                valid = (hoff >= 0) & (k < K) & (r+cx >= 0) & (r+cx < ns) & (r2+cy >= 0) & (r2+cy < nt)
                base = (r*nt + r2)*cell + (x*ny + y)*nz
                idx = np.where(valid, base + hoff, 0)
                assert idx.min() >= 0 and idx.max() < E, ("Ht", shape, s, kk)
        # output writes
        li, lk = tid & 31, (tid & 63) >> 5; wave = tid >> 6
        for j in range(2):
            nn = n0 + wave*64 + 32*j + li
            c = nn // nz; zz = nn % nz; ccx, ccy = c//ny, c % ny
            for i, r in itertools.product(range(2), range(16)):
                mm = m0 + 32*i + 8*(r >> 2) + 4*lk + (r & 3)
                Pp = nx*(mm//g['Lc']) + ccx; Qq = ny*(mm % g['Lc']) + ccy
                ok = (nn < N) & (mm < g['M']) & (Pp < R) & (Qq < C)
                off = np.where(ok, zz*R*C + Pp*C + Qq, 0)
                assert off.min() >= 0 and off.max() < nz*R*C
    return stages

SHAPES = [((15, 15, 3, 3, 3), 21, 21), ((15, 15, 3, 3, 3), 20, 23), ((9, 7, 3, 5, 2), 12, 10),
          ((5, 5, 5, 5, 1), 7, 8), ((7, 9, 1, 1, 3), 11, 9), ((1, 1, 1, 1, 2), 4, 5), ((3, 3, 7, 7, 2), 14, 21),
          ((21, 21, 3, 3, 9), 8, 7), ((5, 5, 3, 3, 2), 9, 12), ((3, 3, 1, 1, 2), 5, 6),
          ((9, 9, 3, 3, 30), 10, 10), ((5, 5, 3, 3, 45), 6, 7)]


@pytest.mark.parametrize("shape,R,C", SHAPES)
def test_projector_addresses_in_bounds(shape, R, C):
    check_fwd(shape, R, C)
    check_bwd(shape, R, C)


def test_projector_addresses_in_bounds_full_size_edges():
    edge = lambda n: sorted(set([0, 1, 2, n // 2, n - 3, n - 2, n - 1]) & set(range(n)))
    check_fwd((165, 165, 15, 15, 21), 600, 600, stage_sample=edge)
    check_bwd((165, 165, 15, 15, 21), 600, 600, kk_sample=edge)


def test_projector_addresses_in_bounds_gpu_test_shapes():
    """The larger shapes the GPU tests run, at edge and randomly sampled stages."""
    rng = np.random.default_rng(0)
    pick = lambda n: sorted(set([0, 1, n // 2, n - 2, n - 1]) | set(rng.integers(0, n, 40).tolist()))
    for shape, R, C in [((45, 45, 15, 15, 5), 120, 105), ((45, 45, 15, 15, 5), 97, 120),
                        ((165, 165, 15, 15, 21), 120, 120), ((33, 25, 11, 5, 4), 55, 40)]:
        check_fwd(shape, R, C, stage_sample=pick)
        check_bwd(shape, R, C, kk_sample=pick)
