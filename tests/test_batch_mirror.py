"""NumPy mirror of the batched launch's slot arithmetic (csrc/lfbp_gather.hip
batch_slot, csrc/lfbp_internal.h xcd_share/xcd_first, csrc/lfbp_api.cpp
layout_batch), on the CPU: over the slots b < nslots of a launch, every unit
of every problem is visited exactly once; in the XCD schedule each XCD's share
of a problem is one contiguous run of its units and the XCD walks differ in
length by at most one unit per problem; in the linear schedule slot b is unit
b of the problems laid end to end."""
import numpy as np
import pytest

XCDS = 8


def share(n, x):
    return n // XCDS + (1 if x < n % XCDS else 0)


def first(n, x):
    return x * (n // XCDS) + min(x, n % XCDS)


def layout(nunits):
    """Per-XCD prefix sums of the walks, as the host builds them."""
    xstart = np.zeros((XCDS, len(nunits) + 1), dtype=np.int64)
    for x in range(XCDS):
        for p, n in enumerate(nunits):
            xstart[x, p + 1] = xstart[x, p] + share(n, x)
    return xstart


def layout_linear(nunits):
    """Prefix sums of the one linear walk (row 0 of the table; other rows unused)."""
    xstart = np.zeros((XCDS, len(nunits) + 1), dtype=np.int64)
    xstart[0, 1:] = np.cumsum(nunits)
    return xstart


def slot_inline(nunits, xstart, b, linear=False):
    """The branch-free scalar count used when the descriptors and the prefix
    table travel in the kernel arguments."""
    x, l = (0, b) if linear else (b % XCDS, b // XCDS)
    if l >= xstart[x, -1]:
        return None
    xs = xstart[x]
    p = sum(1 for i in range(1, 16) if i < len(nunits) and xs[i] <= l)
    return p, (0 if linear else first(nunits[p], x)) + (l - xs[p])


def slot_table(nunits, xstart, b, linear=False):
    """The bisection used with a device descriptor table."""
    x, l = (0, b) if linear else (b % XCDS, b // XCDS)
    if l >= xstart[x, -1]:
        return None
    lo, hi = 0, len(nunits)
    while hi - lo > 1:
        mid = (lo + hi) >> 1
        if xstart[x, mid] <= l:
            lo = mid
        else:
            hi = mid
    return lo, (0 if linear else first(nunits[lo], x)) + (l - xstart[x, lo])


@pytest.mark.parametrize("seed", range(12))
def test_slots_cover_every_unit_once(seed):
    rng = np.random.default_rng(seed)
    count = int(rng.integers(1, 40))
    nunits = [int(v) for v in rng.choice([1, 2, 3, 7, 8, 9, 15, 16, 17, 100, 1001],
                                         size=count)]
    nunits.sort(reverse=True)
    xstart = layout(nunits)
    xtotal = xstart[:, -1]
    slots = int(xtotal.max())
    assert xtotal.max() - xtotal.min() <= count
    seen = {p: np.zeros(n, dtype=np.int64) for p, n in enumerate(nunits)}
    for b in range(XCDS * slots):
        got = slot_table(nunits, xstart, b)
        if count <= 16:
            assert got == slot_inline(nunits, xstart, b)
        if got is None:
            continue
        p, u = got
        assert 0 <= u < nunits[p]
        seen[p][u] += 1
        # an XCD's units of one problem form one contiguous run
        x = b % XCDS
        assert first(nunits[p], x) <= u < first(nunits[p], x) + share(nunits[p], x)
    for p, c in seen.items():
        assert (c == 1).all(), (p, c)


def test_shares_partition_each_problem():
    for n in range(0, 70):
        runs = [(first(n, x), first(n, x) + share(n, x)) for x in range(XCDS)]
        assert runs[0][0] == 0 and runs[-1][1] == n
        assert all(runs[i][1] == runs[i + 1][0] for i in range(XCDS - 1))
        assert max(share(n, x) for x in range(XCDS)) - min(share(n, x) for x in range(XCDS)) <= 1


@pytest.mark.parametrize("seed", range(8))
def test_linear_slots_are_the_units_end_to_end(seed):
    rng = np.random.default_rng(100 + seed)
    count = int(rng.integers(1, 40))
    nunits = sorted((int(v) for v in rng.choice([1, 2, 3, 7, 9, 16, 17, 100, 1001], size=count)), reverse=True)
    xstart = layout_linear(nunits)
    order = [(p, u) for p, n in enumerate(nunits) for u in range(n)]
    nslots = int(xstart[0, -1])
    assert nslots == len(order)
    for b in range(nslots + 9):                      # slots past the end are holes
        got = slot_table(nunits, xstart, b, linear=True)
        if count <= 16:
            assert got == slot_inline(nunits, xstart, b, linear=True)
        assert got == (order[b] if b < nslots else None)
