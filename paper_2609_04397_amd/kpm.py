"""Kernel polynomial method after the moments (marshalling only): density of
states on the device, the resolution-tied threshold and the gap (host code
of the library).  Paper, section 5."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def dos(mu, x, damping: str = "jackson", work=None):
    """Density of states at the points ``x`` (device FP64 tensor, |x| < 1)
    from moments ``mu`` (device FP64, normalised per state)."""
    for name, t in (("mu", mu), ("x", x)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
            raise TypeError("%s must be a CUDA float64 tensor" % name)
    mu = mu.contiguous()
    x = x.contiguous()
    rho = torch.empty_like(x)
    wp = ctypes.c_void_p(work.data_ptr()) if work is not None else None
    if work is not None and work.numel() * work.element_size() < 8 * mu.numel():
        raise ValueError("work needs %d bytes" % (8 * mu.numel()))
    check(_lib.load().vbcsr_kpm_dos(ctypes.c_void_p(mu.data_ptr()), mu.numel(),
                                    _lib.DAMPING[damping], ctypes.c_void_p(x.data_ptr()),
                                    x.numel(), ctypes.c_void_p(rho.data_ptr()), wp, _stream()))
    return rho


def threshold(n_moments: int, n_states: int, fraction: float = 0.1) -> float:
    t = ctypes.c_double()
    check(_lib.load().vbcsr_kpm_threshold(int(n_moments), int(n_states), float(fraction),
                                          ctypes.byref(t)))
    return t.value


def gap(x, rho, thr: float):
    """(lo, hi) bounding the widest below-threshold run (host arrays), or None."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    check(_lib.load().vbcsr_kpm_gap(x.ctypes.data, rho.ctypes.data, x.size, float(thr),
                                    ctypes.byref(lo), ctypes.byref(hi)))
    return None if np.isnan(lo.value) else (lo.value, hi.value)
