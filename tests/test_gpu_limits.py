"""Launch-size limits of the H' kernels on the GPU, against the oracle: grids
whose work-items would pass the 32-bit dispatch size (the out-of-place
gather capped and striding over its units, the column-major and in-place
kernels on a second grid dimension), on thin PSF arrays with many small
work units."""
import numpy as np
import pytest
import torch

import lfsynth
import oracle
import paper_2003_09133_amd as lf
from gpu_util import DEV, gpu_equal_bits

pytestmark = pytest.mark.gpu


def test_gather_grid_capped_at_the_dispatch_size():
    """One x-row per 64-thread workgroup on 69 M x-rows: 69 M workgroups
    would be 4.4e9 work-items; the grid is capped and strides."""
    shape = (1001, 1001, 69, 1, 1)
    assert shape[0] * shape[1] * shape[2] * 64 > 2**32
    H = lfsynth.bits(shape, 21, np.float32)
    dH = torch.from_numpy(H).to(DEV)
    cfg = {"variant": lf.GATHER_DIRECT, "block_threads": 64, "rows_in_flight": 1}
    out = lf.compute_Ht(dH, config=cfg)
    ref = torch.from_numpy(oracle.Ht_rows(H)).to(DEV)
    torch.cuda.synchronize()
    assert gpu_equal_bits(out, ref)


def test_colmajor_past_2_24_units():
    """21 M planes of a thin column-major array: one workgroup each, on a
    two-dimensional grid."""
    shape = (3, 2049, 3, 2049, 5)
    assert shape[1] * shape[3] * shape[4] >= 2**24
    H = lfsynth.bits(shape, 22, np.float16)
    dH = torch.from_numpy(H).to(DEV)
    dc = dH.permute(4, 3, 2, 1, 0).contiguous().permute(4, 3, 2, 1, 0)   # column-major copy
    out = lf.compute_Ht_colmajor(dc)
    ref = torch.from_numpy(oracle.Ht_rows(H)).to(DEV)
    torch.cuda.synchronize()
    assert gpu_equal_bits(out.contiguous(), ref)


def test_inplace_past_2_24_units():
    """25 M row-group pairs (4097 x 4097 blocks of 15 one-element rows)."""
    shape = (4097, 4097, 15, 1, 1)
    H = lfsynth.bits(shape, 23, np.float16)
    dH = torch.from_numpy(H).to(DEV)
    lf.compute_Ht_inplace(dH)
    ref = torch.from_numpy(oracle.Ht_rows(H)).to(DEV)
    torch.cuda.synchronize()
    assert gpu_equal_bits(dH, ref)
    lf.compute_Ht_inplace(dH)                                  # the map is its own inverse
    torch.cuda.synchronize()
    assert gpu_equal_bits(dH, torch.from_numpy(H).to(DEV))
