"""Reciprocal-space sampling of a periodic operator -- TEST INFRASTRUCTURE.

Written from the definition (section 3.3, equation 4):
    O(k) = sum_R exp(-2 pi i k.R) O(R)                        ("R")
and the alternative convention that multiplies block (i, j) by the phase of
R + tau_j - tau_i                                             ("R+tau").
Every block is multiplied by its phase, the real and imaginary parts are
expanded to scalar CSR by the oracle's own expansion (duplicate (i, j) from
several images stay separate entries, so products sum them), and products
use the oracle's FP64 scalar-CSR kernels:
    (Re + i Im)(Xr + i Xi)   = (Re Xr - Im Xi) + i (Re Xi + Im Xr)
    (Re + i Im)^H (Xr + i Xi) = (Re^T Xr + Im^T Xi) + i (Re^T Xi - Im^T Xr)
(the adjoint of equation 1 with the conjugate transpose).
"""
from __future__ import annotations

import numpy as np

import oracle


def phases(Z, k, convention: str = "R") -> np.ndarray:
    """exp(-2 pi i k . d) of every block, d = R or R + tau_j - tau_i."""
    k = np.asarray(k, dtype=np.float64)
    d = Z.shifts[Z.image].astype(np.float64)
    if convention == "R+tau":
        rows = np.repeat(np.arange(Z.n), np.diff(Z.row_ptr))
        d = d + Z.tau[Z.col_idx] - Z.tau[rows]
    elif convention != "R":
        raise ValueError(convention)
    return np.exp(-2j * np.pi * (d @ k))


class KOperator:
    """O(k) as two real scalar-CSR parts over the same entries."""

    def __init__(self, Z, k, convention="R"):
        ph = np.repeat(phases(Z, k, convention), Z.block_sizes)
        cv = Z.values * ph
        self.re = oracle.expand(Z.b, Z.row_ptr, Z.col_idx, np.ascontiguousarray(cv.real))
        self.im = oracle.expand(Z.b, Z.row_ptr, Z.col_idx, np.ascontiguousarray(cv.imag))
        self.N = self.re.N

    def spmm(self, X):
        X = np.asarray(X, dtype=np.complex128)
        Xr, Xi = np.ascontiguousarray(X.real), np.ascontiguousarray(X.imag)
        m = oracle.csr_spmm
        return (m(self.re, Xr) - m(self.im, Xi)) + 1j * (m(self.re, Xi) + m(self.im, Xr))

    def spmm_h(self, X):
        X = np.asarray(X, dtype=np.complex128)
        Xr, Xi = np.ascontiguousarray(X.real), np.ascontiguousarray(X.imag)
        ret, imt = oracle.transpose(self.re), oracle.transpose(self.im)
        m = oracle.csr_spmm
        return (m(ret, Xr) + m(imt, Xi)) + 1j * (m(ret, Xi) - m(imt, Xr))

    def abs_scale(self, X, adjoint=False):
        """|O(k)| |X| (elementwise moduli): scale of the rounding error."""
        A = oracle.ScalarCSR(self.N, self.re.rp, self.re.ci, np.hypot(self.re.va, self.im.va))
        if adjoint:
            A = oracle.transpose(A)
        return oracle.csr_spmm(A, np.abs(np.asarray(X)))
