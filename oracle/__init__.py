"""FP64 CPU oracle for the variable-block sparse products -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It is a plain scalar-CSR implementation in C
(``oracle.c``, built with gcc, no fast-math) behind ctypes; it shares no code
with the device library.

Every function follows one definition from the paper:

* :func:`expand`      block semantics (section 2.1): block ``(i, j)`` is a dense
  ``b_i x b_j`` matrix at rows ``off_i..``, columns ``off_j..``;
* :func:`spmm`        forward product ``Y_i += sum_j A_ij X_j`` (section 3.2);
* :func:`spmm_t`      adjoint product ``Y_j += A_ij^T X_i`` (equation 1, real);
* :func:`sddmm`       block-sampled ``dA_ij = dY_i X_j^T`` (the gradient of
  ``sum(Y * G)`` with respect to the stored blocks);
* :func:`cheb_moments` Chebyshev moments ``mu_k = <R, T_k(A) R>`` of the
  kernel polynomial method (section 5), FP64 throughout;
* :func:`spgemm`      thresholded block product ``C_ij = sum_k A_ik B_kj``
  (section 3.2, equation 2): symbolic stage with the block-norm bound of
  equation 3, numeric stage, a closing filter on the computed block norms.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_expand.argtypes = [ctypes.c_int32, _i32p, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p]
    lib.oracle_expand.restype = None
    lib.oracle_csr_spmm.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_double, ctypes.c_double, _f64p,
                                    ctypes.c_int64]
    lib.oracle_csr_spmm.restype = None
    lib.oracle_csr_transpose.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p]
    lib.oracle_csr_transpose.restype = None
    lib.oracle_sddmm.argtypes = [ctypes.c_int32, _i32p, _i64p, _i32p, _f64p, ctypes.c_int64, _f64p,
                                 ctypes.c_int64, ctypes.c_int32, _f64p]
    lib.oracle_sddmm.restype = None
    lib.oracle_cheb.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64,
                                ctypes.c_int32, ctypes.c_int32, _f64p]
    lib.oracle_cheb.restype = ctypes.c_int
    lib.oracle_seq_norms.argtypes = [ctypes.c_int64, _i64p, _f64p, _f64p]
    lib.oracle_seq_norms.restype = None
    lib.oracle_spgemm_symbolic.argtypes = [ctypes.c_int32, _i64p, _i32p, _f64p, _i64p, _i32p,
                                           _f64p, ctypes.c_double, _i64p, ctypes.c_int64, _i64p,
                                           _i32p, _f64p, ctypes.c_int64]
    lib.oracle_spgemm_symbolic.restype = ctypes.c_int64
    lib.oracle_spgemm_numeric.argtypes = [ctypes.c_int32, _i32p, _i64p, _i32p, _f64p, _i64p,
                                          _i32p, _f64p, _i64p, ctypes.c_int64, _i64p, _i32p,
                                          _f64p]
    lib.oracle_spgemm_numeric.restype = None
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


class ScalarCSR:
    """Scalar-expanded operator: ``rp`` int64 [N+1], ``ci`` int32, ``va`` float64."""

    def __init__(self, N, rp, ci, va):
        self.N, self.rp, self.ci, self.va = N, rp, ci, va

    @property
    def nnz(self):
        return int(self.rp[-1])

    def abs(self) -> "ScalarCSR":
        return ScalarCSR(self.N, self.rp, self.ci, np.abs(self.va))

    def with_values(self, va) -> "ScalarCSR":
        return ScalarCSR(self.N, self.rp, self.ci, np.ascontiguousarray(va, dtype=np.float64))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def expand(b, row_ptr, col_idx, values) -> ScalarCSR:
    """Expand every block into scalar CSR entries (block semantics, section 2.1)."""
    b = _c(b, np.int32)
    row_ptr = _c(row_ptr, np.int64)
    col_idx = _c(col_idx, np.int32)
    values = _c(values, np.float64)
    n = b.shape[0]
    off = np.concatenate([[0], np.cumsum(b.astype(np.int64))])
    N = int(off[-1])
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    nnz = int((b[rows].astype(np.int64) * b[col_idx].astype(np.int64)).sum())
    if values.shape[0] != nnz:
        raise ValueError("values length %d != sum of block sizes %d" % (values.shape[0], nnz))
    rp = np.empty(N + 1, dtype=np.int64)
    ci = np.empty(max(nnz, 1), dtype=np.int32)
    va = np.empty(max(nnz, 1), dtype=np.float64)
    _load().oracle_expand(n, b, row_ptr, col_idx, values if nnz else np.zeros(1), rp, ci, va)
    return ScalarCSR(N, rp, ci[:nnz] if nnz else ci, va[:nnz] if nnz else va)


def expand_op(op, values=None) -> ScalarCSR:
    return expand(op.b, op.row_ptr, op.col_idx, op.values if values is None else values)


def csr_spmm(A: ScalarCSR, X, alpha=1.0, beta=0.0, Y=None) -> np.ndarray:
    """``alpha * A X + beta * Y`` on a scalar-CSR operator."""
    X = _c(X, np.float64)
    if X.ndim == 1:
        X = X[:, None]
    nrhs = X.shape[1]
    if Y is None:
        Y = np.zeros((A.N, nrhs))
        beta = 0.0
    else:
        Y = np.array(Y, dtype=np.float64, order="C", copy=True)
    _load().oracle_csr_spmm(A.N, A.rp, A.ci, A.va, X, nrhs, nrhs, float(alpha), float(beta),
                            Y, nrhs)
    return Y


def transpose(A: ScalarCSR) -> ScalarCSR:
    """Scalar transpose (stable counting sort)."""
    rpt = np.empty(A.N + 1, dtype=np.int64)
    nnz = A.nnz
    cit = np.empty(max(nnz, 1), dtype=np.int32)
    vat = np.empty(max(nnz, 1), dtype=np.float64)
    _load().oracle_csr_transpose(A.N, A.rp, A.ci, A.va, rpt, cit, vat)
    return ScalarCSR(A.N, rpt, cit[:nnz] if nnz else cit, vat[:nnz] if nnz else vat)


def spmm(op, X, alpha=1.0, beta=0.0, Y=None, values=None) -> np.ndarray:
    """``alpha * A X + beta * Y`` for a block operator (forward, section 3.2)."""
    return csr_spmm(expand_op(op, values), X, alpha, beta, Y)


def spmm_t(op, X, alpha=1.0, beta=0.0, Y=None, values=None) -> np.ndarray:
    """``alpha * A^T X + beta * Y`` (equation 1 with the real adjoint)."""
    return csr_spmm(transpose(expand_op(op, values)), X, alpha, beta, Y)


def sddmm(op, dY, X) -> np.ndarray:
    """``dA_ij = dY_i X_j^T`` on the stored blocks, graph order."""
    dY = _c(dY, np.float64)
    X = _c(X, np.float64)
    nnz = op.nnz
    out = np.empty(max(nnz, 1))
    _load().oracle_sddmm(op.n, _c(op.b, np.int32), _c(op.row_ptr, np.int64),
                         _c(op.col_idx, np.int32), dY, dY.shape[1], X, X.shape[1], X.shape[1], out)
    return out[:nnz]


def cheb_moments(op_or_csr, R, degree: int) -> np.ndarray:
    """Chebyshev moments ``mu[k, c] = <R_c, T_k(A) R_c>``, ``k = 0..degree``."""
    A = op_or_csr if isinstance(op_or_csr, ScalarCSR) else expand_op(op_or_csr)
    R = _c(R, np.float64)
    nrhs = R.shape[1]
    mu = np.empty((degree + 1, nrhs))
    rc = _load().oracle_cheb(A.N, A.rp, A.ci, A.va, R, nrhs, nrhs, int(degree), mu)
    if rc != 0:
        raise MemoryError("oracle_cheb: allocation failed")
    return mu


def abs_product(op, X, values=None, transpose_op=False) -> np.ndarray:
    """``|A| |X|``: the scale of the componentwise error bound."""
    A = expand_op(op, values).abs()
    if transpose_op:
        A = transpose(A)
    return csr_spmm(A, np.abs(X))


def seq_norms(sizes, values) -> np.ndarray:
    """Frobenius norms of blocks stored back to back (``sizes[t]`` values each)."""
    sizes = _c(sizes, np.int64)
    out = np.empty(max(sizes.shape[0], 1))
    _load().oracle_seq_norms(sizes.shape[0], sizes, _c(values, np.float64) if values.size
                             else np.zeros(1), out)
    return out[:sizes.shape[0]]


def block_norms(op, values=None) -> np.ndarray:
    """Frobenius norm of every stored block of ``op``, graph order."""
    r = np.repeat(np.arange(op.b.shape[0]), np.diff(op.row_ptr))
    sizes = op.b[r].astype(np.int64) * op.b[op.col_idx].astype(np.int64)
    return seq_norms(sizes, op.values if values is None else values)


def spgemm(A, B, eps: float = 0.0, rows=None) -> dict:
    """Thresholded block product ``C = A B`` (section 3.2, equations 2 and 3).

    ``A`` and ``B`` are operators over the same atoms.  For the block rows
    ``rows`` (all by default) returns a dict with

    * ``sym_rp``, ``sym_col``, ``bound``: the symbolic pattern, i.e. the
      candidates (i, j) with ``U_ij = sum_k ||A_ik|| ||B_kj|| >= eps``
      (row-pointer over ``rows``, ascending columns, the bound of each);
    * ``sym_values``: the numeric blocks of that pattern, row-major, back to
      back in pattern order;
    * ``rp``, ``col``, ``values``, ``norms``: the result after the final
      filter, which keeps the blocks whose Frobenius norm is at least ``eps``.
    """
    if not np.array_equal(np.asarray(A.b), np.asarray(B.b)):
        raise ValueError("A and B must share the atoms (block sizes)")
    b = _c(A.b, np.int32)
    n = b.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else _c(rows, np.int64)
    arp, aci = _c(A.row_ptr, np.int64), _c(A.col_idx, np.int32)
    brp, bci = _c(B.row_ptr, np.int64), _c(B.col_idx, np.int32)
    an, bn = block_norms(A), block_norms(B)
    blen = np.diff(brp)
    cap = 1
    for i in rows:
        cap += int(blen[aci[arp[i]:arp[i + 1]]].sum())
    cnt = np.zeros(max(rows.shape[0], 1), dtype=np.int64)
    col = np.empty(cap, dtype=np.int32)
    bound = np.empty(cap)
    tot = _load().oracle_spgemm_symbolic(n, arp, aci, an if an.size else np.zeros(1), brp, bci,
                                         bn if bn.size else np.zeros(1), float(eps), rows,
                                         rows.shape[0], cnt, col, bound, cap)
    if tot < 0:
        raise RuntimeError("oracle_spgemm_symbolic: capacity exceeded")
    sym_rp = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(cnt[:rows.shape[0]], out=sym_rp[1:])
    sym_col = col[:tot].copy()
    bound = bound[:tot].copy()
    rowb = np.repeat(b[rows].astype(np.int64), np.diff(sym_rp))
    sizes = rowb * b[sym_col].astype(np.int64)
    vals = np.empty(max(int(sizes.sum()), 1))
    _load().oracle_spgemm_numeric(n, b, arp, aci, _c(A.values, np.float64), brp, bci,
                                  _c(B.values, np.float64), rows, rows.shape[0], sym_rp,
                                  sym_col if tot else np.zeros(1, np.int32), vals)
    vals = vals[:int(sizes.sum())]
    norms = seq_norms(sizes, vals)
    keep = ~(norms < eps)
    base = np.zeros(tot + 1, dtype=np.int64)
    np.cumsum(sizes, out=base[1:])
    kept_vals = np.concatenate([vals[base[t]:base[t + 1]] for t in np.nonzero(keep)[0]]) \
        if keep.any() else np.zeros(0)
    t_row = np.repeat(np.arange(rows.shape[0]), np.diff(sym_rp))
    rp = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(t_row[keep], minlength=rows.shape[0]), out=rp[1:])
    return {"rows": rows, "sym_rp": sym_rp, "sym_col": sym_col, "bound": bound,
            "sym_values": vals, "rp": rp, "col": sym_col[keep].copy(), "values": kept_vals,
            "norms": norms[keep].copy()}
