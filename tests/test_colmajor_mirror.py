"""The column-major (Matlab order) H -> H' kernel's index arithmetic, on the
CPU: a NumPy mirror of k_colmajor and its launch arithmetic
(paper_2003_09133_amd/csrc/lfbp_colmajor.hip) against the oracle's H' moved
to column-major order.  Every 16-byte vector read lies inside the array or
takes the element path, every tile slot written lies inside its row's pitch,
every element read from the tile was loaded, and every output element is
written exactly once.  Keep it in step with the kernel."""
import numpy as np
import pytest

import lfsynth
import oracle


def to_colmajor(A):
    """Column-major storage of an [ns][nt][nx][ny][nz] array, as a flat array."""
    return np.ascontiguousarray(A.transpose(4, 3, 2, 1, 0)).ravel()


def row_table_bytes(nx, VE):
    return ((nx + VE - 1) * 4 + 15) // 16 * 16


def launch_params(shape, esize, max_lds=160 * 1024, tile_budget=96 * 1024):
    ns, nt, nx, ny, nz = shape
    VE = 16 // esize
    vec_col = nx * 16
    table = row_table_bytes(nx, VE)
    small = min(tile_budget, max_lds)
    budget = small if vec_col * 4 + table <= small else max_lds
    assert budget >= table + vec_col
    pmax = ((budget - table) // vec_col) * VE
    S0 = min(ns, pmax - (VE - 1))
    chunks = -(-ns // S0)
    S = -(-ns // chunks)
    P = (S + 2 * VE - 2) // VE * VE
    assert nx * P * esize + table <= max(budget, tile_budget) and nx * P * esize + table <= max_lds
    return VE, S, chunks, P


THREADS = 256


def colmajor_mirror(Hc, shape, phase_in=0, phase_out=0, **kw):
    """Hc: flat column-major H.  phase_*: misalignment (in elements) of the
    arrays' first element against 16 bytes, as the kernel sees it."""
    ns, nt, nx, ny, nz = shape
    esize = Hc.dtype.itemsize
    VE, S, chunks, P = launch_params(shape, esize, **kw)
    VR = P // VE
    E = Hc.size
    hs, ht = (ns - 1) // 2, (nt - 1) // 2
    a_off, b_off = (nx - hs % nx) % nx, (ny - ht % ny) % ny
    xstride = ns * nt
    assert nx * xstride < 2**31
    xsm = xstride % VE
    dq_load, dr_load = THREADS // VR, THREADS % VR
    Sl = ns - (chunks - 1) * S
    NFs, st = [], []
    for Sn_ in (S, Sl):
        NF_ = (Sn_ - (VE - 1)) // VE if Sn_ >= VE - 1 else 0
        nf1 = max(NF_, 1)
        dr_ = THREADS % nf1
        NFs.append(NF_)
        st.append((THREADS // nf1, dr_, dr_ * VE % nx, NF_ * VE % nx))
    out = np.zeros(E, Hc.dtype)
    written = np.zeros(E, np.int64)
    tid = np.arange(THREADS)
    for unit in range(nt * ny * nz * chunks):
        plane, c = divmod(unit, chunks)
        q1, tp = divmod(plane, nt)
        z, yp = divmod(q1, ny)
        y = (yp + (tp + b_off) % ny) % ny
        t = nt - 1 - tp
        s0 = c * S
        assert s0 < ns
        Sn = min(S, ns - s0)
        s_lo = ns - s0 - Sn
        in0 = (t + nt * nx * (y + ny * z)) * ns
        out0 = (tp + nt * nx * (yp + ny * z)) * ns
        total = nx * VR
        cin = (in0 + s_lo + phase_in) % VE
        tile = np.full(nx * P, -1, np.int64)          # which element of H each slot holds
        g_first, g_last = in0 + s_lo, in0 + (nx - 1) * xstride + s_lo
        if g_first >= VE and g_last + P <= E:
            # fast path: per-thread stepping of (x, v, xoff); batches of 4
            x, v = tid // VR, tid % VR
            xoff = x * xstride
            j = tid.copy()
            while np.any(j < total):
                m = (cin + x * xsm) & (VE - 1)
                live = (j < total) & (v * VE < m + Sn)
                off = np.where(live, xoff + VE - m + v * VE, VE - cin)
                assert np.all(off >= 0) and np.all(off + VE <= 2**32)
                vg = g_first - VE + off                          # element index of the vector
                assert np.all((vg + phase_in) % VE == 0) and vg.min() >= 0 and vg.max() + VE <= E
                assert np.array_equal(x[live], (j // VR)[live]) and np.array_equal(v[live], (j % VR)[live])
                slot = x * P + v * VE
                for q in range(VE):
                    tile[slot[live] + q] = vg[live] + q
                v = v + dr_load
                x = x + dq_load
                xoff = xoff + dq_load * xstride
                carry = v >= VR
                v = np.where(carry, v - VR, v)
                x = x + carry
                xoff = xoff + carry * xstride
                j = j + THREADS
        else:
            for jj in range(total):
                x, v = divmod(jj, VR)
                m = (cin + x * xsm) & (VE - 1)
                if v * VE >= m + Sn:
                    continue
                vg = in0 + x * xstride + s_lo - m + v * VE
                for q in range(VE):
                    i = vg + q
                    tile[x * P + v * VE + q] = i if 0 <= i < E else -2
        # row table
        i = np.arange(nx + VE - 1)
        xr = i % nx
        rt = xr * P + ((cin + xr * xsm) & (VE - 1)) + Sn - 1 - i
        last = int(Sn != S)
        NF = NFs[last]
        dq, dr, du, dnf = st[last]
        cout = (out0 + s0 + phase_out) % VE
        ob = out0 + s0
        nvec = nx * NF

        def put(dst, idx, ok):
            src = tile[idx[ok]]
            assert np.all(src >= 0), "tile slot read before it was loaded"
            out[dst[ok]] = Hc[src]
            np.add.at(written, dst[ok], 1)

        if nvec:
            xp, f = tid // NF, tid % NF
            xoff = xp * xstride
            u = (s0 + a_off + f * VE) % nx
            j = tid.copy()
            while np.any(j < nvec):
                ok = j < nvec
                assert np.array_equal(xp[ok], (j // NF)[ok]) and np.array_equal(f[ok], (j % NF)[ok])
                mo = (cout + xp * xsm) & (VE - 1)
                kA = (VE - mo) & (VE - 1)
                k0 = kA + f * VE
                x0 = (xp + u) % nx
                x0 = (x0 + kA) % nx
                assert np.array_equal(x0[ok], ((xp + (s0 + k0 + a_off) % nx) % nx)[ok])
                C = x0 - k0
                dst0 = ob + xoff + k0
                assert np.all(((dst0 + phase_out) % VE == 0)[ok]) and np.all((k0 + VE <= Sn)[ok])
                for q in range(VE):
                    put(dst0 + q, rt[np.where(ok, x0 + q, 0)] + C, ok)
                f = f + dr
                xp = xp + dq
                xoff = xoff + dq * xstride
                u = u + du
                u = np.where(u >= nx, u - nx, u)
                carry = f >= NF
                f = np.where(carry, f - NF, f)
                xp = xp + carry
                xoff = xoff + carry * xstride
                u = np.where(carry, np.where(u >= dnf, u - dnf, u + nx - dnf), u)
                j = j + THREADS
        L = Sn - NF * VE
        jj = np.arange(nx * L)
        xp, ii = jj // L, jj % L
        mo = (cout + xp * xsm) & (VE - 1)
        kA = (VE - mo) & (VE - 1)
        kk = np.where(ii < kA, ii, ii + NF * VE)
        x = (xp + (s0 + kk + a_off) % nx) % nx
        put(ob + xp * xstride + kk, rt[x] + x - kk, np.ones(jj.size, bool))
    assert np.all(written == 1)
    return out


SHAPES = [(15, 15, 3, 3, 3), (9, 7, 3, 5, 2), (3, 5, 5, 3, 1), (1, 1, 1, 1, 2), (11, 7, 1, 1, 2),
          (21, 9, 7, 3, 4), (5, 5, 9, 1, 3), (13, 11, 9, 5, 2), (33, 3, 17, 1, 1), (1, 1, 5, 3, 2)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("budget", [96 * 1024, 0])
def test_colmajor_mirror_equals_oracle(shape, dtype, budget):
    """budget 0: the smallest tile budget of the launch rule (one vector of
    each row per chunk beyond the slack), which forces many chunks."""
    H = lfsynth.bits(shape, 5, dtype)
    kw = {} if budget else {"tile_budget": 1, "max_lds": shape[2] * 16 * 2 + row_table_bytes(shape[2], 16 // H.itemsize)}
    ref = to_colmajor(oracle.Ht_rows(H))
    for ph in ((0, 0), (1, 3), (3, 2)):
        got = colmajor_mirror(to_colmajor(H), shape, *ph, **kw)
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), ph


def test_wide_cells_take_the_whole_lds():
    """nx = 2047: four vectors of every row exceed 96 KB; the tile grows to
    the device's LDS with a ragged last chunk."""
    VE, S, chunks, P = launch_params((35, 1, 2047, 1, 1), 4)
    assert 4 * 2047 * 16 > 96 * 1024 and chunks > 1 and 35 % S != 0
    H = lfsynth.bits((35, 1, 2047, 1, 1), 6, np.float32)
    got = colmajor_mirror(to_colmajor(H), H.shape)
    assert np.array_equal(got.view(np.uint32), to_colmajor(oracle.Ht_rows(H)).view(np.uint32))


@pytest.mark.parametrize("units", [1, 7, 8, 9, 16, 1001, 10769, 344542])
def test_xcd_order_is_a_permutation(units):
    """unit_of_block: each XCD (workgroup index mod 8) takes a contiguous run
    of units; together the workgroups cover every unit exactly once."""
    bid = np.arange(units)
    x, q, r = bid % 8, units // 8, units % 8
    unit = x * q + np.minimum(x, r) + bid // 8
    assert np.array_equal(np.sort(unit), bid)


@pytest.mark.parametrize("units", [1, 8, 2**24 - 1, 2**24, 2**24 + 5, 21_000_000, 2**31 - 1])
def test_launch_grid_covers_every_unit(units):
    """launch_colmajor and launch_inplace: one workgroup per unit, on a second
    grid dimension of 2^16-wide rows past 2^24 units, so that the work-items
    of each dimension (256 threads per workgroup) fit 32 bits; workgroups of
    the last row past the last unit return at once, and the others, in
    dispatch order b = x + y * 2^16, map one to one onto the units."""
    if units < 2**24:
        gx, gy = units, 1
    else:
        gx, gy = 1 << 16, (units + 0xFFFF) >> 16
    assert gx * 256 < 2**32 and gy <= 32768
    assert gx * gy >= units > gx * (gy - 1)
    b = np.arange(min(units, 4096))                      # a prefix: the map is the same formula throughout
    x, q, r = b % 8, units // 8, units % 8
    unit = x * q + np.minimum(x, r) + b // 8
    assert unit.max() < units and np.unique(unit).size == b.size

