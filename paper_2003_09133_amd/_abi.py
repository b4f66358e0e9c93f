"""ctypes view of liblfbp.so (the C ABI of include/lfbp.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LFBP_LIB", os.path.join(HERE, "liblfbp.so"))

OK, EINVAL, ESHAPE, EDTYPE, EALIAS, EDEVICE, ENOMEM, EALIGN, ECAPTURE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
NOALLOC_MAX_PROBLEMS = 1024
F32, F16 = 0, 1
GATHER_AUTO, GATHER_DIRECT, GATHER_STAGED, GATHER_WIDE = 0, 1, 2, 3

STATUS_NAMES = {OK: "LFBP_OK", EINVAL: "LFBP_EINVAL", ESHAPE: "LFBP_ESHAPE", EDTYPE: "LFBP_EDTYPE",
                EALIAS: "LFBP_EALIAS", EDEVICE: "LFBP_EDEVICE", ENOMEM: "LFBP_ENOMEM", EALIGN: "LFBP_EALIGN",
                ECAPTURE: "LFBP_ECAPTURE", ESCRATCH: "LFBP_ESCRATCH"}


class Shape(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int64), ("nt", ctypes.c_int64), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]

    @classmethod
    def of(cls, dims):
        return cls(*(int(v) for v in dims))


class Problem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_void_p), ("Ht", ctypes.c_void_p), ("shape", Shape)]


class GatherConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("rows_in_flight", ctypes.c_int32), ("tile_bytes", ctypes.c_int32),
                ("vec_per_thread", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("waves_per_eu", ctypes.c_int32), ("schedule", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LfbpError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({status_string(status)})")


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"liblfbp.so not found at {LIB_PATH}: build it first "
                              f"(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        st = ctypes.c_int
        sig = {
            "lfbp_compute_Ht": (st, [vp, vp, Shape, i32, vp]),
            "lfbp_compute_Ht_config": (st, [vp, vp, Shape, i32, ctypes.POINTER(GatherConfig), vp]),
            "lfbp_compute_Ht_inplace": (st, [vp, Shape, i32, vp]),
            "lfbp_compute_Ht_colmajor": (st, [vp, vp, Shape, i32, vp]),
            "lfbp_default_config": (st, [Shape, i32, ctypes.POINTER(GatherConfig)]),
            "lfbp_compute_Ht_batched": (st, [ctypes.POINTER(Problem), i32, i32, vp]),
            "lfbp_compute_Ht_batched_noalloc": (st, [ctypes.POINTER(Problem), i32, i32, vp]),
            "lfbp_compute_Ht_batched_config": (st, [ctypes.POINTER(Problem), i32, i32,
                                                    ctypes.POINTER(GatherConfig), i32, vp]),
            "lfbp_forward": (st, [vp, Shape, vp, i64, i64, vp, vp]),
            "lfbp_forward_ws": (st, [vp, Shape, vp, i64, i64, vp, vp, i64, vp]),
            "lfbp_forward_workspace_size": (i64, [Shape, i64, i64]),
            "lfbp_backward": (st, [vp, Shape, vp, i64, i64, vp, vp]),
            "lfbp_backward_ws": (st, [vp, Shape, vp, i64, i64, vp, vp, i64, vp]),
            "lfbp_backward_workspace_size": (i64, [Shape, i64, i64]),
            "lfbp_rl_step": (st, [vp, vp, Shape, vp, i64, i64, vp, vp, vp, vp]),
            "lfbp_rl_step_ws": (st, [vp, vp, Shape, vp, i64, i64, vp, vp, vp, vp, i64, vp]),
            "lfbp_rl_workspace_size": (i64, [Shape, i64, i64]),
            "lfbp_rl_norm_ws": (st, [vp, Shape, i64, i64, vp, vp, i64, vp]),
            "lfbp_grad_psf": (st, [vp, vp, Shape, i64, i64, vp, vp]),
            "lfbp_grad_psf_ws": (st, [vp, vp, Shape, i64, i64, vp, vp, i64, vp]),
            "lfbp_operator_size": (i64, [Shape, i64, i64]),
            "lfbp_operator_workspace_size": (i64, [Shape, i64, i64]),
            "lfbp_operator_prepare": (st, [vp, vp, Shape, i64, i64, vp, i64, vp]),
            "lfbp_forward_op": (st, [vp, i64, Shape, vp, i64, i64, vp, vp, i64, vp]),
            "lfbp_backward_op": (st, [vp, i64, Shape, vp, i64, i64, vp, vp, i64, vp]),
            "lfbp_rl_step_op": (st, [vp, i64, Shape, vp, i64, i64, vp, vp, vp, vp, i64, vp]),
            "lfbp_rl_norm_op": (st, [vp, i64, Shape, i64, i64, vp, vp, i64, vp]),
            "lfbp_grad_psf_workspace_size": (i64, [Shape, i64, i64]),
            "lfbp_status_string": (ctypes.c_char_p, [st]),
            "lfbp_release_plans": (None, []),
            "lfbp_plan_count": (ctypes.c_int32, []),
            "lfbp_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().lfbp_status_string(status).decode()
    except ImportError:
        return STATUS_NAMES.get(status, str(status))


def check(status: int, what: str):
    if status != OK:
        raise LfbpError(status, what)
