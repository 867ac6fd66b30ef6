"""ctypes declarations of ``libvbcsr.so`` (argument marshalling only).

The shared library is built in-tree by :mod:`paper_2609_04397_amd.build`.
Loading fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvbcsr.so")

VBCSR_OK = 0
VBCSR_EINVAL = -1
VBCSR_ESHAPE = -2
VBCSR_EDUP = -3
VBCSR_ENOMEM = -4
VBCSR_EHIP = -5
VBCSR_EUNSUPPORTED = -6
NOALLOC_SCRATCH_BYTES = 32 << 20  # VBCSR_NOALLOC_SCRATCH_BYTES
CODE_NAMES = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "EDUP", -4: "ENOMEM", -5: "EHIP",
              -6: "EUNSUPPORTED"}

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
PATH = {"auto": 0, "vec": 1, "mfma": 2}
ORDER = {"auto": 0, "atom": 1, "rcm": 2, "cluster": 3}
DAMPING = {"none": 0, "jackson": 1}
PHASE = {"R": 0, "R+tau": 1}

# Every symbol declared in include/vbcsr.h, with (restype, argtypes).
_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_int = ctypes.c_int


class PlanOpts(ctypes.Structure):
    _fields_ = [("rows_per_wg", ctypes.c_int32), ("nrhs_tile", ctypes.c_int32),
                ("path", ctypes.c_int32), ("row_order", ctypes.c_int32)]


class SpgemmStats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("kept_symbolic", ctypes.c_int64),
                ("nnzb", ctypes.c_int64), ("products", ctypes.c_int64),
                ("flops", ctypes.c_double), ("ms_norms", ctypes.c_double),
                ("ms_symbolic", ctypes.c_double), ("ms_numeric", ctypes.c_double),
                ("ms_filter", ctypes.c_double), ("ms_build", ctypes.c_double)]


SIGNATURES = {
    "vbcsr_create": (_int, [ctypes.POINTER(_p), _i32, _p, _p, _p, _p, _i64, _int,
                            ctypes.POINTER(PlanOpts), _p]),
    "vbcsr_create_local": (_int, [ctypes.POINTER(_p), _i32, _i32, _p, _p, _p, _p, _i64, _int,
                                  ctypes.POINTER(PlanOpts), _p]),
    "vbcsr_shape": (_int, [_p, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                           ctypes.POINTER(_i64)]),
    "vbcsr_halo_create": (_int, [ctypes.POINTER(_p), _i32, _p, _p, _p, _p, _i32, _i32]),
    "vbcsr_halo_info": (_int, [_p, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                               ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "vbcsr_halo_graph": (_int, [_p, _p, _p, _p, _p]),
    "vbcsr_halo_local_values": (_int, [_p, _p, _p]),
    "vbcsr_halo_lists": (_int, [_p, _p, _p, _p, _p, _p, _p]),
    "vbcsr_halo_destroy": (None, [_p]),
    "vbcsr_halo_pack": (_int, [_p, _i64, _i64, _p, _i64, _i32, _i32, _p, _i64, _p]),
    "vbcsr_halo_reduce": (_int, [_p, _i64, _i64, _p, _p, _p, _i64, _p, _i64, _i64, _i32, _i32, _p]),
    "vbcsr_set_values": (_int, [_p, _p, _int, _int, _p]),
    "vbcsr_spmm": (_int, [_p, _p, _i64, _p, _i64, _i32, _f64, _f64, _p]),
    "vbcsr_spmm_t": (_int, [_p, _p, _i64, _p, _i64, _i32, _f64, _f64, _p]),
    "vbcsr_sddmm": (_int, [_p, _p, _i64, _p, _i64, _i32, _p, _p]),
    "vbcsr_page_size": (_int, [_p, ctypes.POINTER(_i64)]),
    "vbcsr_get_pages": (_int, [_p, _p, _p]),
    "vbcsr_use_pages": (_int, [_p, _p]),
    "vbcsr_refresh_transposed": (_int, [_p, _p]),
    "vbcsr_sddmm_pages": (_int, [_p, _p, _i64, _p, _i64, _i32, _p, _p]),
    "vbcsr_cheb_workspace_bytes": (_int, [_p, _i32, _i32, ctypes.POINTER(_i64)]),
    "vbcsr_cheb_moments": (_int, [_p, _p, _i64, _i32, _i32, _p, _p, _i64, _p]),
    "vbcsr_cheb_moments_doubled": (_int, [_p, _p, _i64, _i32, _i32, _p, _p, _i64, _p]),
    "vbcsr_cheb_step": (_int, [_p, _p, _i64, _p, _i64, _p, _i64, _i32, _p, _p, _i64, _p]),
    "vbcsr_cheb_step_noalloc": (_int, [_p, _p, _i64, _p, _i64, _p, _i64, _i32, _p, _p]),
    "vbcsr_info": (_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                          ctypes.POINTER(_i32)]),
    "vbcsr_plan_host": (_int, [_i32, _p, _p, _p, _i64, ctypes.POINTER(_i32), _p, _i32, _p, _p,
                               ctypes.POINTER(_i64), ctypes.POINTER(PlanOpts)]),
    "vbcsr_get_structure": (_int, [_p, _p, _p, _p]),
    "vbcsr_get_values": (_int, [_p, _p, _int, _p]),
    "vbcsr_spgemm": (_int, [ctypes.POINTER(_p), _p, _p, _f64, ctypes.POINTER(PlanOpts),
                            ctypes.POINTER(SpgemmStats), _p]),
    "vbcsr_kpm_dos": (_int, [_p, _i32, _i32, _p, _i64, _p, _p, _p]),
    "vbcsr_kpm_threshold": (_int, [_i32, _i64, _f64, ctypes.POINTER(_f64)]),
    "vbcsr_kpm_gap": (_int, [_p, _p, _i64, _f64, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
    "vbcsr_zmat_create": (_int, [ctypes.POINTER(_p), _i32, _p, _p, _p, _p, _i32, _p, _p, _p, _i64,
                                 _int, ctypes.POINTER(PlanOpts), _p]),
    "vbcsr_zmat_sample": (_int, [_p, _p, _i32, _p]),
    "vbcsr_zmat_spmm": (_int, [_p, _p, _i64, _p, _i64, _i32, _p, _p, _i32, _p]),
    "vbcsr_zmat_info": (_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                               ctypes.POINTER(_i64)]),
    "vbcsr_zmat_get_structure": (_int, [_p, _p, _p]),
    "vbcsr_zmat_get_values": (_int, [_p, _p, _p]),
    "vbcsr_zmat_destroy": (None, [_p]),
    "vbcsr_destroy": (None, [_p]),
    "vbcsr_last_error": (ctypes.c_char_p, []),
}

_lib = None


class VbcsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (CODE_NAMES.get(code, "?"), code, msg))
        self.code = code


def load():
    """Load ``libvbcsr.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvbcsr.so is not built (%s); run python -m "
                          "paper_2609_04397_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != VBCSR_OK:
        msg = load().vbcsr_last_error()
        raise VbcsrError(rc, msg.decode() if msg else "")
