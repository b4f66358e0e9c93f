"""In-place H -> H' (lfbp_compute_Ht_inplace) against the out-of-place kernels
and the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import lfsynth
import oracle
import paper_2003_09133_amd as lf
from gpu_util import DEV, assert_same_bits, gpu_equal_bits, to_dev

pytestmark = pytest.mark.gpu


def random_shapes(seed, n):
    rng = np.random.default_rng(seed)
    odd = lambda lo, hi: int(rng.integers(lo, hi + 1)) | 1
    return [(odd(1, 41), odd(1, 41), odd(1, 13), odd(1, 13), int(rng.integers(1, 24))) for _ in range(n)]


SHAPES = [(15, 15, 3, 3, 3), (1, 1, 1, 1, 1), (1, 3, 1, 1, 2), (3, 5, 5, 3, 1), (11, 7, 1, 1, 2),
          (21, 9, 7, 3, 4), (5, 5, 9, 1, 3), (15, 15, 15, 15, 200)] + random_shapes(5, 10)


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("shape", SHAPES)
def test_inplace_equals_oracle_and_involution(shape, dtype):
    H = lfsynth.bits(shape, 17, dtype)
    d = to_dev(H)
    lf.compute_Ht_inplace(d)
    torch.cuda.synchronize()
    assert_same_bits(d.cpu().numpy(), oracle.Ht_rows(H), f"{shape} {dtype.__name__}")
    lf.compute_Ht_inplace(d)
    torch.cuda.synchronize()
    assert_same_bits(d.cpu().numpy(), H, f"{shape} twice")


def test_inplace_microscope_equals_oracle():
    """The microscope PSF (random bit payloads), whole array: in place against
    the oracle, and against the out-of-place kernel."""
    w = lfsynth.MICROSCOPE
    H = lfsynth.bits(w.shape, w.seed, np.float32)
    d = to_dev(H)
    ref = lf.compute_Ht(d)
    lf.compute_Ht_inplace(d)
    assert_same_bits(d.cpu().numpy(), oracle.Ht_rows(H), "microscope in place")
    assert gpu_equal_bits(d, ref)


def test_inplace_camera_f16_equals_oracle():
    """The camera PSF in float16 (random bit payloads): in place against the
    oracle at 3 million sampled elements and at whole x-rows of the first,
    middle and last blocks, then against the out-of-place kernel everywhere;
    a second call restores H."""
    from gpu_util import sample_indices
    w = lfsynth.CAMERA
    H = lfsynth.bits(w.shape, w.seed, np.float16)
    d = to_dev(H)
    ref = lf.compute_Ht(d)
    lf.compute_Ht_inplace(d)
    ns, nt, nx, ny, nz = w.shape
    W = ny * nz
    rows = [0, nx - 1, (ns * nt // 2) * nx + 3, ns * nt * nx - 1]
    idx = np.concatenate([sample_indices(H.size, 3_000_000, 41)] +
                         [np.arange(r * W, (r + 1) * W, dtype=np.int64) for r in rows])
    got = d.view(-1)[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    assert_same_bits(got, oracle.Ht_at(H, idx), "camera f16 in place, sampled")
    assert gpu_equal_bits(d, ref)
    del ref
    lf.compute_Ht_inplace(d)
    assert gpu_equal_bits(d, to_dev(H))


def test_inplace_on_a_view_and_stream_order():
    """A PSF array inside a larger buffer (unaligned start) with canaries
    around it; queued after a plain build on the same stream."""
    shape = (9, 11, 5, 3, 7)
    n = int(np.prod(shape))
    H = lfsynth.bits(shape, 23, np.float32)
    buf = torch.full((n + 7,), -1.0, device=DEV)
    view = buf[3:3 + n].view(shape)
    view.copy_(torch.from_numpy(H))
    out = lf.compute_Ht(view)
    lf.compute_Ht_inplace(view)
    torch.cuda.synchronize()
    assert gpu_equal_bits(out, view)                  # bit patterns (the payloads include NaNs)
    assert torch.all(buf[:3] == -1.0) and torch.all(buf[3 + n:] == -1.0)


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("offset", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("shape", [(11, 7, 1, 1, 2), (5, 5, 9, 1, 3), (9, 7, 3, 5, 2), (7, 9, 3, 1, 1)])
def test_inplace_unaligned_views(shape, offset, dtype):
    """Arrays starting `offset` elements into a buffer (every position of the
    first element in a 16-byte vector), rows shorter than a vector among
    them: equal to the oracle, canaries untouched."""
    n = int(np.prod(shape))
    H = lfsynth.bits(shape, 29, dtype)
    tdt = torch.float32 if dtype == np.float32 else torch.float16
    buf = torch.full((n + 16,), -1.0, device=DEV, dtype=tdt)
    view = buf[offset:offset + n].view(shape)
    view.copy_(torch.from_numpy(H))
    lf.compute_Ht_inplace(view)
    torch.cuda.synchronize()
    assert_same_bits(view.cpu().numpy(), oracle.Ht_rows(H), f"{shape} offset {offset} {dtype.__name__}")
    assert torch.all(buf[:offset] == -1.0) and torch.all(buf[offset + n:] == -1.0)
