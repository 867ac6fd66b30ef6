"""Reciprocal-space operators (marshalling only): ``KMatrix`` wraps one
``vbcsr_zmat`` handle (paper, section 3.3, equation 4).  Sampling and the
complex products run in the HIP kernels behind the C ABI."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

_CT = {"fp64": torch.complex128, "fp32": torch.complex64}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class KMatrix:
    """Periodic operator from image blocks; ``sample(k)`` assembles O(k)."""

    def __init__(self, block_sizes, row_ptr, col_idx, image, shifts, values=None, tau=None,
                 prec: str = "fp64", row_order: str = "auto"):
        if prec not in _CT:
            raise ValueError("prec must be fp64 or fp32")
        self.prec, self.dtype = prec, _CT[prec]
        b, rp, ci = _np(block_sizes, np.int32), _np(row_ptr, np.int64), _np(col_idx, np.int32)
        im, sh = _np(image, np.int32), _np(shifts, np.int32).reshape(-1, 3)
        self.n = int(b.size)
        rows = np.repeat(np.arange(self.n), np.diff(rp))
        nnz = int((b[rows].astype(np.int64) * b[ci].astype(np.int64)).sum()) if ci.size else 0
        v = _np(values, np.float64) if values is not None else None
        t = _np(tau, np.float64).reshape(-1, 3) if tau is not None else None
        opts = _lib.PlanOpts(0, 0, 0, _lib.ORDER[row_order])
        h = ctypes.c_void_p()
        check(_lib.load().vbcsr_zmat_create(
            ctypes.byref(h), self.n, b.ctypes.data, rp.ctypes.data,
            ci.ctypes.data if ci.size else None, im.ctypes.data if im.size else None,
            sh.shape[0], sh.ctypes.data, t.ctypes.data if t is not None else None,
            v.ctypes.data if v is not None else None, nnz, _lib.PREC[prec], ctypes.byref(opts),
            _stream()))
        self._h = h
        n_rows, nkb, nkv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(_lib.load().vbcsr_zmat_info(h, ctypes.byref(n_rows), ctypes.byref(nkb),
                                          ctypes.byref(nkv)))
        self.N, self.nnzb_k, self.n_values_k = n_rows.value, nkb.value, nkv.value
        self.block_sizes = b

    @classmethod
    def from_images(cls, Z, **kw):
        return cls(Z.b, Z.row_ptr, Z.col_idx, Z.image, Z.shifts, Z.values, Z.tau, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().vbcsr_zmat_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sample(self, k, convention: str = "R"):
        kk = _np(k, np.float64)
        check(_lib.load().vbcsr_zmat_sample(self._h, kk.ctypes.data, _lib.PHASE[convention],
                                            _stream()))
        return self

    def spmm(self, X, Y=None, alpha=1.0, beta=0.0, adjoint=False):
        if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == self.dtype):
            raise TypeError("X must be a CUDA %s tensor" % self.dtype)
        if X.dim() == 1:
            X = X.unsqueeze(1)
        X = X.contiguous()
        nrhs = X.shape[1]
        if Y is None:
            Y = torch.empty_like(X)
            beta = 0.0
        a = _np([complex(alpha).real, complex(alpha).imag], np.float64)
        bb = _np([complex(beta).real, complex(beta).imag], np.float64)
        check(_lib.load().vbcsr_zmat_spmm(self._h, ctypes.c_void_p(X.data_ptr()), X.stride(0),
                                          ctypes.c_void_p(Y.data_ptr()), Y.stride(0), nrhs,
                                          a.ctypes.data, bb.ctypes.data, 1 if adjoint else 0,
                                          _stream()))
        return Y

    def structure(self):
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(max(self.nnzb_k, 1), np.int32)
        check(_lib.load().vbcsr_zmat_get_structure(self._h, rp.ctypes.data, ci.ctypes.data))
        return rp, ci[:self.nnzb_k]

    def values(self):
        out = torch.empty(self.n_values_k, dtype=self.dtype, device="cuda")
        check(_lib.load().vbcsr_zmat_get_values(self._h, ctypes.c_void_p(out.data_ptr()),
                                                _stream()))
        return out
