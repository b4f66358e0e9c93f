"""Seeded synthetic inputs for light-field PSF arrays.

Inputs only: nothing here re-arranges H, projects a volume or back-projects an
image.  Both the HIP library's tests and the CPU oracle's tests take their data
from this module.  The C core (``lfsynth.c``) is built by ``build()`` into
``liblfsynth.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .workloads import (BATCHED_SETS, CAMERA, MICROSCOPE, PROJECTOR, SMALL_SETS, TINY,
                        TABLE1_SHAPES, Workload, batched_set, small_set, table1_workload)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblfsynth.so")
_lib = None

__all__ = ["build", "gauss_f32", "bits_u32", "bits_u16", "bits", "uniform_f32",
           "small_int_f32", "poisson_counts", "word", "Workload", "TINY", "MICROSCOPE", "CAMERA",
           "PROJECTOR", "BATCHED_SETS", "SMALL_SETS", "TABLE1_SHAPES", "batched_set", "small_set", "table1_workload", "make_H"]


def build(verbose: bool = False) -> str:
    """Compile lfsynth.c with gcc and OpenMP into liblfsynth.so."""
    global _lib
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           os.path.join(_HERE, "lfsynth.c"), "-o", _SO + ".tmp", "-lm"]
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
        i64, u64, dbl, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        vp = ctypes.c_void_p
        lib.lfsynth_gauss_f32.restype = i64
        lib.lfsynth_gauss_f32.argtypes = [i64] * 5 + [dbl, dbl, dbl, u64, dbl, vp,
                                                      ctypes.POINTER(dbl), i32]
        lib.lfsynth_bits_u32.argtypes = [i64, u64, vp, i32]
        lib.lfsynth_bits_u16.argtypes = [i64, u64, vp, i32]
        lib.lfsynth_uniform_f32.argtypes = [i64, u64, vp, i32]
        lib.lfsynth_small_int_f32.argtypes = [i64, u64, ctypes.c_int32, vp, i32]
        lib.lfsynth_word.restype = u64
        lib.lfsynth_word.argtypes = [u64, u64]
        _lib = lib
    return _lib


def word(seed: int, idx: int) -> int:
    """The 64-bit SplitMix64 word number ``idx`` of stream ``seed``."""
    return int(_load().lfsynth_word(seed, idx))


def gauss_f32(shape, sig0: float, slope: float, zc: float, seed: int,
              thr: float = 0.05, nthreads: int = 0, out: np.ndarray | None = None):
    """Gaussian-envelope PSF patterns times uniform noise; entries below
    ``thr * max`` are zeroed.  Returns ``(H, zero_fraction, vmax)``."""
    ns, nt, nx, ny, nz = (int(v) for v in shape)
    if out is None:
        out = np.empty((ns, nt, nx, ny, nz), dtype=np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.size == ns * nt * nx * ny * nz
    vmax = ctypes.c_double(0.0)
    zeros = _load().lfsynth_gauss_f32(ns, nt, nx, ny, nz, float(sig0), float(slope), float(zc),
                                      int(seed), float(thr), out.ctypes.data, ctypes.byref(vmax),
                                      int(nthreads))
    return out, zeros / max(out.size, 1), vmax.value


def bits_u32(shape, seed: int, nthreads: int = 0) -> np.ndarray:
    """Random 32-bit payloads (with NaN, inf, -0 and denormal patterns mixed in)."""
    out = np.empty(shape, dtype=np.uint32)
    _load().lfsynth_bits_u32(out.size, int(seed), out.ctypes.data, int(nthreads))
    return out


def bits_u16(shape, seed: int, nthreads: int = 0) -> np.ndarray:
    """Random 16-bit payloads (with NaN, inf, -0 and denormal patterns mixed in)."""
    out = np.empty(shape, dtype=np.uint16)
    _load().lfsynth_bits_u16(out.size, int(seed), out.ctypes.data, int(nthreads))
    return out


def bits(shape, seed: int, dtype, nthreads: int = 0) -> np.ndarray:
    """Random payloads viewed as ``dtype`` (float32 or float16)."""
    dtype = np.dtype(dtype)
    if dtype.itemsize == 4:
        return bits_u32(shape, seed, nthreads).view(dtype)
    if dtype.itemsize == 2:
        return bits_u16(shape, seed, nthreads).view(dtype)
    raise ValueError(f"unsupported element size {dtype.itemsize}")


def uniform_f32(shape, seed: int, nthreads: int = 0) -> np.ndarray:
    out = np.empty(shape, dtype=np.float32)
    _load().lfsynth_uniform_f32(out.size, int(seed), out.ctypes.data, int(nthreads))
    return out


def small_int_f32(shape, seed: int, k: int, nthreads: int = 0) -> np.ndarray:
    """Integers 0..k-1 stored as float32: sums of products are exact in float64."""
    out = np.empty(shape, dtype=np.float32)
    _load().lfsynth_small_int_f32(out.size, int(seed), int(k), out.ctypes.data, int(nthreads))
    return out


def poisson_counts(mean: np.ndarray, seed: int) -> np.ndarray:
    """Photon counts: one Poisson draw per element with the given means
    (numpy's seeded PCG64 generator), as float32.  The shot noise of a
    light-field image f = Poisson(H g) is what the Richardson-Lucy update of
    Eq. 2 is the maximum-likelihood iteration for."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.asarray(mean, dtype=np.float64)).astype(np.float32)


def make_H(w: Workload, dtype=np.float32, nthreads: int = 0, out: np.ndarray | None = None):
    """The PSF array of workload ``w``: float32 generator output, rounded to
    nearest-even when float16 storage is asked for.  Returns ``(H, zero_fraction)``."""
    H, zf, _ = gauss_f32(w.shape, w.sig0, w.slope, w.zc, w.seed, nthreads=nthreads,
                         out=out if np.dtype(dtype) == np.float32 else None)
    if np.dtype(dtype) == np.float16:
        H = H.astype(np.float16)
    return H, zf
