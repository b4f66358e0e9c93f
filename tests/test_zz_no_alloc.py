"""lfbp_compute_Ht_batched_noalloc (the batched H' build whose descriptor table
lives in the library's fixed device scratch) through the C ABI, against
lfbp_compute_Ht_batched bit for bit: two calls in a row on one stream, the
second with a smaller batch, both past the 16 problems that travel in the
kernel arguments; a small batch; and the limit."""
import ctypes

import numpy as np
import pytest
import torch

import lfsynth
from gpu_util import DEV, to_dev
from paper_2003_09133_amd import _abi

pytestmark = pytest.mark.gpu


def shapes(seed, n):
    rng = np.random.default_rng(seed)
    odd = lambda lo, hi: int(rng.integers(lo, hi + 1)) | 1
    return [(odd(1, 61), odd(1, 61), odd(1, 13), odd(1, 13), int(rng.integers(1, 30))) for _ in range(n)]


def table(Hs, outs):
    return (_abi.Problem * len(Hs))(*[_abi.Problem(h.data_ptr(), o.data_ptr(), _abi.Shape.of(h.shape))
                                      for h, o in zip(Hs, outs)])


def run(fn, Hs, dtype):
    outs = [torch.full_like(h, float("nan")) for h in Hs]
    st = fn(table(Hs, outs), len(Hs), dtype, torch.cuda.current_stream().cuda_stream)
    assert st == _abi.OK, _abi.STATUS_NAMES.get(st, st)
    return outs


def same_bits(a, b):
    it = torch.int32 if a.element_size() == 4 else torch.int16
    return torch.equal(a.view(it), b.view(it))


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_noalloc_equals_batched_twice_second_smaller(dtype):
    L = _abi.lib()
    dt = _abi.F32 if dtype == np.float32 else _abi.F16
    first = [to_dev(lfsynth.bits(s, 5 * i + 1, dtype)) for i, s in enumerate(shapes(61, 40))]
    second = [to_dev(lfsynth.bits(s, 7 * i + 2, dtype)) for i, s in enumerate(shapes(62, 21))]
    for Hs in (first, second):
        print(f"noalloc batch of {len(Hs)} problems, {np.dtype(dtype).name}", flush=True)
        got = run(L.lfbp_compute_Ht_batched_noalloc, Hs, dt)
        ref = run(L.lfbp_compute_Ht_batched, Hs, dt)
        torch.cuda.synchronize()
        for i, (g, r) in enumerate(zip(got, ref)):
            assert same_bits(g, r), f"problem {i} of {len(Hs)}, shape {tuple(Hs[i].shape)}"
    L.lfbp_release_plans()


def test_noalloc_small_batch_and_limit():
    L = _abi.lib()
    Hs = [to_dev(lfsynth.bits(s, i + 9, np.float32)) for i, s in enumerate(shapes(63, 5))]
    got = run(L.lfbp_compute_Ht_batched_noalloc, Hs, _abi.F32)
    ref = run(L.lfbp_compute_Ht_batched, Hs, _abi.F32)
    torch.cuda.synchronize()
    assert all(same_bits(g, r) for g, r in zip(got, ref))
    # one problem more than the scratch holds: refused before anything runs
    n = _abi.NOALLOC_MAX_PROBLEMS + 1
    h = torch.empty((3, 3, 1, 1, 1), device=DEV)
    outs = torch.empty((n, 3, 3, 1, 1, 1), device=DEV)
    probs = (_abi.Problem * n)(*[_abi.Problem(h.data_ptr(), outs[i].data_ptr(), _abi.Shape.of(h.shape))
                                 for i in range(n)])
    assert L.lfbp_compute_Ht_batched_noalloc(probs, n, _abi.F32, None) == _abi.ESCRATCH
    L.lfbp_release_plans()
