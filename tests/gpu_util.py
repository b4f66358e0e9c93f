"""Helpers of the GPU tests (no computation of H' here)."""
from __future__ import annotations

import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def bits_of(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint16)


def assert_same_bits(got: np.ndarray, ref: np.ndarray, what: str = ""):
    assert got.shape == ref.shape and got.dtype == ref.dtype, (got.shape, ref.shape, got.dtype, ref.dtype)
    g, r = bits_of(got).ravel(), bits_of(ref).ravel()
    if not np.array_equal(g, r):
        bad = np.flatnonzero(g != r)
        idx = np.unravel_index(bad[:5], got.shape)
        raise AssertionError(f"{what}: {bad.size} of {g.size} elements differ; first at "
                             f"{list(zip(*[i.tolist() for i in idx]))}: got {g[bad[:5]]}, want {r[bad[:5]]}")


def gpu_equal_bits(a: torch.Tensor, b: torch.Tensor) -> bool:
    """Bitwise equality of two device tensors of one dtype (as integers)."""
    it = torch.int32 if a.element_size() == 4 else torch.int16
    return bool(torch.equal(a.view(it), b.view(it)))


def gpu_rel_l2(a: torch.Tensor, b: torch.Tensor) -> float:
    """Relative L2 distance of two device tensors, in float64."""
    a, b = a.double(), b.double()
    return float((a - b).norm() / b.norm())


# The prepared operator's forward (16-column class boxes) and the per-call
# forward (64-column boxes) sum in different orders in float32, and each adds
# its float32 partial sums in float64: they agree far inside the 1e-5 bound
# both keep against the float64 oracle.
SAME_SUM_TOL = 1e-6


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k flat indices in [0, n): both ends, then random."""
    rng = np.random.default_rng(seed)
    ends = np.array([0, 1, 2, n - 3, n - 2, n - 1], dtype=np.int64).clip(0, n - 1)
    return np.unique(np.concatenate([ends, rng.integers(0, n, k, dtype=np.int64)]))
