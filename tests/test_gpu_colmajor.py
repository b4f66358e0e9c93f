"""H' of column-major (Matlab order) arrays on the GPU against the CPU
oracle, bit for bit: the oracle's H' of the same array, moved to column-major
order on the host, for small shapes with ragged tails, the chunked and
whole-LDS paths, the Table 1 sizes of Sec. 5 (sampled for the two largest),
and both element sizes."""
import numpy as np
import pytest
import torch

import lfsynth
import oracle
import paper_2003_09133_amd as lf
from gpu_util import DEV, assert_same_bits, gpu_equal_bits, sample_indices

pytestmark = pytest.mark.gpu


def to_dev_colmajor(H: np.ndarray) -> torch.Tensor:
    """H [ns][nt][nx][ny][nz] stored column-major on the GPU (a view of a
    contiguous [nz][ny][nx][nt][ns] tensor)."""
    store = np.ascontiguousarray(H.transpose(4, 3, 2, 1, 0))
    return torch.from_numpy(store).to(DEV).permute(4, 3, 2, 1, 0)


def storage(t: torch.Tensor) -> torch.Tensor:
    """The flat column-major storage of a column-major tensor."""
    return t.permute(4, 3, 2, 1, 0).reshape(-1)


def ref_colmajor(H: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(oracle.Ht_rows(H).transpose(4, 3, 2, 1, 0)).ravel()


SMALL = [(1, 1, 1, 1, 1), (3, 3, 1, 1, 1), (15, 15, 3, 3, 3), (9, 7, 3, 5, 2), (3, 5, 5, 3, 1),
         (11, 7, 1, 1, 2), (21, 9, 7, 3, 4), (5, 5, 9, 1, 3), (13, 11, 9, 5, 2), (33, 65, 17, 3, 1),
         (65, 3, 1, 1, 7), (299, 3, 3, 1, 2)]


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("shape", SMALL)
def test_small_shapes(shape, dtype):
    H = lfsynth.bits(shape, 11, dtype)
    out = lf.compute_Ht_colmajor(to_dev_colmajor(H))
    torch.cuda.synchronize()
    assert_same_bits(storage(out).cpu().numpy(), ref_colmajor(H), f"colmajor {shape}")


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("shape", [(35, 3, 1537, 1, 1), (13, 1, 2047, 1, 2), (301, 3, 257, 1, 2)])
def test_columns_wider_than_the_tile_budget(shape, dtype):
    """Cells of more than 1500 rows: four 16-byte vectors of every row
    exceed 96 KB, so tiles take up to the device's whole LDS, a few s
    positions each, with a ragged last chunk; and 257 rows of 301 positions,
    which the 96 KB tile budget splits into chunks."""
    H = lfsynth.bits(shape, 12, dtype)
    out = lf.compute_Ht_colmajor(to_dev_colmajor(H))
    torch.cuda.synchronize()
    assert_same_bits(storage(out).cpu().numpy(), ref_colmajor(H), f"colmajor {shape}")


def test_cells_wider_than_2048_rows_are_refused():
    H = torch.zeros((1, 3, 2049, 1, 3), device=DEV, dtype=torch.float16).permute(4, 3, 2, 1, 0)
    assert H.shape == (3, 1, 2049, 3, 1)
    with pytest.raises(lf.LfbpError):
        lf.compute_Ht_colmajor(H)


def test_unaligned_views():
    """Arrays whose first element is not 16-byte aligned: the vector loads
    and stores shift, the first and last vectors take the element path."""
    shape = (21, 9, 7, 3, 4)
    H = lfsynth.bits(shape, 14, np.float32)
    n = H.size
    store = torch.from_numpy(np.ascontiguousarray(H.transpose(4, 3, 2, 1, 0)).ravel()).to(DEV)
    for off_in, off_out in ((1, 3), (2, 0), (3, 1)):
        big = torch.zeros(n + 8, device=DEV, dtype=torch.float32)
        big[off_in:off_in + n] = store
        dst = torch.full((n + 8,), 7.0, device=DEV, dtype=torch.float32)
        src = big[off_in:off_in + n].view(tuple(reversed(shape))).permute(4, 3, 2, 1, 0)
        out = dst[off_out:off_out + n].view(tuple(reversed(shape))).permute(4, 3, 2, 1, 0)
        lf.compute_Ht_colmajor(src, out=out)
        torch.cuda.synchronize()
        d = dst.cpu().numpy()
        assert_same_bits(d[off_out:off_out + n], ref_colmajor(H), f"offsets {off_in} {off_out}")
        assert np.all(d[:off_out] == 7.0) and np.all(d[off_out + n:] == 7.0)


def test_agrees_with_row_major_and_is_an_involution():
    H = lfsynth.bits((91, 91, 15, 15, 11), 13, np.float32)
    dc = to_dev_colmajor(H)
    out = lf.compute_Ht_colmajor(dc)
    rows = lf.compute_Ht(torch.from_numpy(H).to(DEV))
    back = lf.compute_Ht_colmajor(out, out=torch.empty_like(out))
    torch.cuda.synchronize()
    assert gpu_equal_bits(out.contiguous(), rows)
    assert gpu_equal_bits(storage(back), storage(dc))


def test_rejects_row_major_tensors():
    H = torch.zeros((3, 3, 3, 3, 2), device=DEV)
    with pytest.raises(ValueError):
        lf.compute_Ht_colmajor(H)


@pytest.mark.parametrize("i", range(len(lfsynth.TABLE1_SHAPES)))
def test_table1_sizes(i):
    """Every size of Table 1 (11 depths): the whole array for the nine
    smaller ones, 2M sampled elements plus two whole (t', y', z) planes for
    the two largest (1 GB and 7.5 GB in float32)."""
    w = lfsynth.table1_workload(i)
    dtype = np.float16 if i % 2 else np.float32
    H = lfsynth.bits(w.shape, 40 + i, dtype)
    print(f"\n{w.name} {w.shape} {np.dtype(dtype).name}", flush=True)
    if i < 9:
        out = lf.compute_Ht_colmajor(to_dev_colmajor(H))
        torch.cuda.synchronize()
        assert_same_bits(storage(out).cpu().numpy(), ref_colmajor(H), w.name)
        return
    dH = torch.from_numpy(H).to(DEV)
    dc = dH.permute(4, 3, 2, 1, 0).contiguous().permute(4, 3, 2, 1, 0)   # column-major copy
    del dH
    out = lf.compute_Ht_colmajor(dc)
    torch.cuda.synchronize()
    flat = storage(out)
    idx = sample_indices(H.size, 2_000_000, 3)                 # row-major logical indices
    col = np.ravel_multi_index(np.unravel_index(idx, w.shape), w.shape, order="F")
    got = flat[torch.from_numpy(col).to(DEV)].cpu().numpy()
    assert_same_bits(got, oracle.Ht_at(H, idx), f"{w.name} sampled")
    ns, nt, nx, ny, nz = w.shape
    plane = ns * nt * nx                                       # one (y', z) slab of the storage
    for yz in (0, ny * nz - 1):
        s_idx = np.arange(yz * plane, (yz + 1) * plane, dtype=np.int64)
        ridx = np.ravel_multi_index(np.unravel_index(s_idx, w.shape, order="F"), w.shape)
        assert_same_bits(flat[yz * plane:(yz + 1) * plane].cpu().numpy(), oracle.Ht_at(H, ridx),
                         f"{w.name} slab {yz}")
