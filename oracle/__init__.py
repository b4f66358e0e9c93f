"""CPU oracle for the backprojection array H' and the light-field projectors.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the benchmark's ``cpu_baseline`` leg, never by the product package.

H' is computed from its plain definition -- the transposed measurement matrix
A of the forward model f = H g (Sec. 2.1, Eq. 1; Sec. 3, Fig. 6 discussion) --
in C (``lfbp_oracle.c``); the projectors evaluate A g and A^T f in float64 from
H.  Every function here is pinned by the CPU tests to values and properties
the paper fixes (see tests/test_oracle_pins.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblfbp_oracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    global _lib
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           os.path.join(_HERE, "lfbp_oracle.c"), os.path.join(_HERE, "lfbp_paper.c"), "-o", _SO + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    _lib = None
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        for name, args in {
            "oracle_A_dense": [vp, i32, vp, i64, i64, vp],
            "oracle_Ht_dense": [vp, i32, vp, vp],
            "oracle_Ht_dense_grid": [vp, i32, vp, i64, i64, i64, i64, vp],
            "oracle_Ht_rows": [vp, i32, vp, vp, i32],
            "oracle_Ht_at": [vp, i32, vp, vp, i64, vp, i32],
            "oracle_forward": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_forward_at": [vp, vp, vp, i64, i64, vp, i64, vp, i32],
            "oracle_backward": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_backward_at": [vp, vp, vp, i64, i64, vp, i64, vp, i32],
            "oracle_forward_d": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_forward_sparse": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_backward_sparse": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_backward_d": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_grad_psf": [vp, vp, vp, i64, i64, vp, i32],
            "oracle_grad_psf_at": [vp, vp, vp, i64, i64, vp, i64, vp, i32],
            "paper_Ht": [vp, i32, vp, vp, i32, vp],
        }.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = i32
        _lib = lib
    return _lib


def _dims(H: np.ndarray) -> np.ndarray:
    if H.ndim != 5:
        raise ValueError("H must be 5-D [ns][nt][nx][ny][nz]")
    return np.asarray(H.shape, dtype=np.int64)


def _payload(H: np.ndarray) -> np.ndarray:
    H = np.ascontiguousarray(H)
    if H.dtype.itemsize not in (2, 4):
        raise ValueError("element size must be 2 or 4 bytes")
    return H


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def A_dense(H: np.ndarray, R: int, C: int) -> np.ndarray:
    """Dense measurement matrix [R*C, nz*R*C] on an R x C image, entries are H
    payloads (same dtype as H) or zero."""
    H = _payload(H)
    nz = H.shape[4]
    A = np.empty((R * C, nz * R * C), dtype=H.dtype)
    _check(_load().oracle_A_dense(H.ctypes.data, H.dtype.itemsize, _dims(H).ctypes.data, R, C,
                                  A.ctypes.data), "oracle_A_dense")
    return A


def Ht_dense(H: np.ndarray, grid=None) -> np.ndarray:
    """H' from the explicitly transposed dense measurement matrix.  ``grid`` =
    (Lr, Lc, lr, lc) reads the slices of lenslet (lr, lc) of an Lr x Lc grid;
    default: the smallest grid, central lenslet."""
    H = _payload(H)
    out = np.empty_like(H)
    Lr, Lc, lr, lc = grid if grid is not None else (0, 0, 0, 0)
    _check(_load().oracle_Ht_dense_grid(H.ctypes.data, H.dtype.itemsize, _dims(H).ctypes.data,
                                        Lr, Lc, lr, lc, out.ctypes.data), "oracle_Ht_dense")
    return out


def Ht_rows(H: np.ndarray, nthreads: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """H' by evaluating the needed entries of A one at a time (no dense A)."""
    H = _payload(H)
    if out is None:
        out = np.empty_like(H)
    _check(_load().oracle_Ht_rows(H.ctypes.data, H.dtype.itemsize, _dims(H).ctypes.data,
                                  out.ctypes.data, nthreads), "oracle_Ht_rows")
    return out


def Ht_at(H: np.ndarray, flat_idx: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Selected elements of H' (flat row-major indices)."""
    H = _payload(H)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.shape, dtype=H.dtype)
    _check(_load().oracle_Ht_at(H.ctypes.data, H.dtype.itemsize, _dims(H).ctypes.data,
                                idx.ctypes.data, idx.size, out.ctypes.data, nthreads), "oracle_Ht_at")
    return out


def paper_Ht(H: np.ndarray, nthreads: int = 0, out: np.ndarray | None = None):
    """H' by the paper's own method (Sec. 4: Eq. 3 with the relations of
    Eqs. 4-9, looped as in Fig. 10), for timing "the paper's method on this
    host".  Entries the relations do not reach keep the value they had in
    ``out`` (zeros when ``out`` is None).  Returns ``(Ht, depth_columns_written)``."""
    H = _payload(H)
    if out is None:
        out = np.zeros_like(H)
    assert out.shape == H.shape and out.dtype == H.dtype and out.flags.c_contiguous
    cols = ctypes.c_int64(0)
    _check(_load().paper_Ht(H.ctypes.data, H.dtype.itemsize, _dims(H).ctypes.data, out.ctypes.data, nthreads,
                            ctypes.byref(cols)), "paper_Ht")
    return out, cols.value


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def forward(H: np.ndarray, g: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """f = A g in float64; H float32 [ns][nt][nx][ny][nz], g float32 [nz][R][C]."""
    H, g = _f32(H), _f32(g)
    nz, R, C = g.shape
    assert nz == H.shape[4]
    f = np.empty((R, C), dtype=np.float64)
    _check(_load().oracle_forward(H.ctypes.data, _dims(H).ctypes.data, g.ctypes.data, R, C,
                                  f.ctypes.data, nthreads), "oracle_forward")
    return f


def forward_at(H: np.ndarray, g: np.ndarray, pixels: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """f = A g at the listed pixels (array of (p, q) pairs), float64."""
    H, g = _f32(H), _f32(g)
    nz, R, C = g.shape
    pix = np.ascontiguousarray(pixels, dtype=np.int64).reshape(-1, 2)
    out = np.empty(len(pix), dtype=np.float64)
    _check(_load().oracle_forward_at(H.ctypes.data, _dims(H).ctypes.data, g.ctypes.data, R, C,
                                     pix.ctypes.data, len(pix), out.ctypes.data, nthreads),
           "oracle_forward_at")
    return out


def backward(H: np.ndarray, f: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """A^T f in float64, computed from H (not from H'); f float32 [R][C]."""
    H, f = _f32(H), _f32(f)
    R, C = f.shape
    g = np.empty((H.shape[4], R, C), dtype=np.float64)
    _check(_load().oracle_backward(H.ctypes.data, _dims(H).ctypes.data, f.ctypes.data, R, C,
                                   g.ctypes.data, nthreads), "oracle_backward")
    return g


def backward_at(H: np.ndarray, f: np.ndarray, voxels: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """A^T f at the listed voxels (array of (z, P, Q) triples), float64."""
    H, f = _f32(H), _f32(f)
    R, C = f.shape
    vox = np.ascontiguousarray(voxels, dtype=np.int64).reshape(-1, 3)
    out = np.empty(len(vox), dtype=np.float64)
    _check(_load().oracle_backward_at(H.ctypes.data, _dims(H).ctypes.data, f.ctypes.data, R, C,
                                      vox.ctypes.data, len(vox), out.ctypes.data, nthreads),
           "oracle_backward_at")
    return out


def forward_sparse(H: np.ndarray, g: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """f = A g in float64, summed over the nonzero entries of H only (the same
    entries of A read from the H side; cost scales with the nonzeros)."""
    H, g = _f32(H), _f32(g)
    nz, R, C = g.shape
    assert nz == H.shape[4]
    f = np.empty((R, C), dtype=np.float64)
    _check(_load().oracle_forward_sparse(H.ctypes.data, _dims(H).ctypes.data, g.ctypes.data, R, C,
                                         f.ctypes.data, nthreads), "oracle_forward_sparse")
    return f


def backward_sparse(H: np.ndarray, f: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """A^T f in float64 from H, summed over the nonzero entries of H only."""
    H, f = _f32(H), _f32(f)
    R, C = f.shape
    g = np.empty((H.shape[4], R, C), dtype=np.float64)
    _check(_load().oracle_backward_sparse(H.ctypes.data, _dims(H).ctypes.data, f.ctypes.data, R, C,
                                          g.ctypes.data, nthreads), "oracle_backward_sparse")
    return g


def forward64(H: np.ndarray, g: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """f = A g with a float64 volume g [nz][R][C]; float64."""
    H, g = _f32(H), np.ascontiguousarray(g, dtype=np.float64)
    nz, R, C = g.shape
    assert nz == H.shape[4]
    f = np.empty((R, C), dtype=np.float64)
    _check(_load().oracle_forward_d(H.ctypes.data, _dims(H).ctypes.data, g.ctypes.data, R, C,
                                    f.ctypes.data, nthreads), "oracle_forward_d")
    return f


def backward64(H: np.ndarray, f: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """A^T f with a float64 image f [R][C], computed from H; float64."""
    H, f = _f32(H), np.ascontiguousarray(f, dtype=np.float64)
    R, C = f.shape
    g = np.empty((H.shape[4], R, C), dtype=np.float64)
    _check(_load().oracle_backward_d(H.ctypes.data, _dims(H).ctypes.data, f.ctypes.data, R, C,
                                     g.ctypes.data, nthreads), "oracle_backward_d")
    return g


def rl_norm(H: np.ndarray, R: int, C: int, nthreads: int = 0) -> np.ndarray:
    """A^T 1: the normaliser of the Richardson-Lucy update (Eq. 2), float64."""
    return backward64(H, np.ones((R, C)), nthreads)


def rl_step(H: np.ndarray, f: np.ndarray, g: np.ndarray, norm: np.ndarray | None = None,
            nthreads: int = 0) -> np.ndarray:
    """One Richardson-Lucy update (Eq. 2) in float64, from H (never H'):

        g_new = g / (A^T 1) * A^T ( f / (A g) ),

    elementwise.  Readings: where (A g)[p][q] is 0 the quotient is 0; where
    A^T 1 is 0 (a voxel seen by no pixel of the image) g_new is 0."""
    R, C = f.shape
    norm = rl_norm(H, R, C, nthreads) if norm is None else np.asarray(norm, dtype=np.float64)
    fp = forward64(H, g, nthreads)
    ratio = np.zeros_like(fp)
    np.divide(np.asarray(f, dtype=np.float64), fp, out=ratio, where=fp > 0)
    bp = backward64(H, ratio, nthreads)
    out = np.zeros_like(bp)
    np.divide(np.asarray(g, dtype=np.float64) * bp, norm, out=out, where=norm > 0)
    return out


def grad_psf(shape, w: np.ndarray, g: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """d<w, A g>/dH, float64 [ns][nt][nx][ny][nz], from the definition of A."""
    w, g = _f32(w), _f32(g)
    R, C = w.shape
    dims = np.array(shape, dtype=np.int64)
    assert g.shape == (shape[4], R, C)
    out = np.empty(tuple(shape), dtype=np.float64)
    _check(_load().oracle_grad_psf(dims.ctypes.data, w.ctypes.data, g.ctypes.data, R, C, out.ctypes.data,
                                   nthreads), "oracle_grad_psf")
    return out


def grad_psf_at(shape, w: np.ndarray, g: np.ndarray, flat_idx: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """d<w, A g>/dH at the listed flat indices of H, float64."""
    w, g = _f32(w), _f32(g)
    R, C = w.shape
    dims = np.array(shape, dtype=np.int64)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.float64)
    _check(_load().oracle_grad_psf_at(dims.ctypes.data, w.ctypes.data, g.ctypes.data, R, C, idx.ctypes.data,
                                      idx.size, out.ctypes.data, nthreads), "oracle_grad_psf_at")
    return out
