"""Python front end of the variable-block library (marshalling only).

``Matrix`` wraps one ``vbcsr_mat`` handle.  Every product runs in the HIP
kernels behind the C ABI; torch supplies device memory and the current
stream, nothing else.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

_TORCH_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.float32}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Matrix:
    """A device operator with dense ``b_i x b_j`` blocks (paper, section 2.1).

    ``block_sizes`` [n], ``row_ptr`` [n+1] and ``col_idx`` [nnzb] describe the
    block graph; ``values`` (graph order, each block row-major) may be a host
    array, a device tensor or ``None`` (zeros).  ``prec`` is ``"fp64"``,
    ``"fp32"`` or ``"bf16x3"``.
    """

    _stamps = 0  # bumped by every value upload; lets autograd detect repacks

    def __init__(self, block_sizes, row_ptr, col_idx, values=None, prec: str = "fp64",
                 path: str = "auto", nrhs_tile: int = 0, row_order: str = "auto",
                 n_ghost: int = 0):
        """``n_ghost > 0`` builds a rank-local operator (section 3.1): the
        first ``len(row_ptr) - 1`` atoms are owned (block rows), the last
        ``n_ghost`` are ghosts (columns only); see ``vbcsr_create_local``."""
        lib = _lib.load()
        if prec not in _lib.PREC:
            raise ValueError("prec must be one of %s" % list(_lib.PREC))
        self.prec = prec
        self.dtype = _TORCH_DTYPE[prec]
        self.device = torch.device("cuda", torch.cuda.current_device())
        b = _np(block_sizes, np.int32)
        rp = _np(row_ptr, np.int64)
        ci = _np(col_idx, np.int32)
        self.block_sizes, self.row_ptr, self.col_idx = b, rp, ci
        self.n = int(b.shape[0])
        n_rows = int(rp.shape[0]) - 1
        if n_ghost < 0 or (n_ghost == 0 and n_rows != self.n) or \
                (n_ghost > 0 and n_rows + n_ghost != self.n):
            raise ValueError("row_ptr needs n_atoms + 1 entries (square) or "
                             "n_atoms - n_ghost + 1 (rank-local)")
        nnz = int((b[np.repeat(np.arange(n_rows), np.diff(rp))].astype(np.int64)
                   * b[ci].astype(np.int64)).sum()) if ci.size else 0
        self.n_values = nnz
        self.N = int(b.astype(np.int64).sum())
        self.n_rows = n_rows
        self.N_rows = int(b[:n_rows].astype(np.int64).sum())
        opts = _lib.PlanOpts(0, int(nrhs_tile), _lib.PATH[path], _lib.ORDER[row_order])
        host_vals = None
        dev_vals = None
        if isinstance(values, torch.Tensor) and values.is_cuda:
            dev_vals = values
        elif values is not None:
            host_vals = _np(values.cpu().numpy() if isinstance(values, torch.Tensor) else values,
                            np.float64)
        h = ctypes.c_void_p()
        if n_ghost > 0:
            check(lib.vbcsr_create_local(ctypes.byref(h), n_rows, int(n_ghost), b.ctypes.data,
                                         rp.ctypes.data, ci.ctypes.data if ci.size else None,
                                         host_vals.ctypes.data if host_vals is not None else None,
                                         nnz, _lib.PREC[prec], ctypes.byref(opts), _stream()))
        else:
            check(lib.vbcsr_create(ctypes.byref(h), self.n, b.ctypes.data, rp.ctypes.data,
                                   ci.ctypes.data if ci.size else None,
                                   host_vals.ctypes.data if host_vals is not None else None,
                                   nnz, _lib.PREC[prec], ctypes.byref(opts), _stream()))
        self._h = h
        Matrix._stamps += 1
        self._stamp = Matrix._stamps
        if dev_vals is not None:
            self.set_values(dev_vals)

    @classmethod
    def _adopt(cls, h, n_atoms: int, prec: str = "fp64"):
        """Wrap a handle the library created (the block product's result)."""
        self = cls.__new__(cls)
        self._h = h
        self.prec, self.dtype = prec, _TORCH_DTYPE[prec]
        self.device = torch.device("cuda", torch.cuda.current_device())
        inf = self.info()
        self.n, self.N, self.n_values = int(n_atoms), inf["N"], inf["n_values"]
        self.n_rows, self.N_rows = self.n, self.N
        b = np.empty(self.n, np.int32)
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(max(inf["nnzb"], 1), np.int32)
        check(_lib.load().vbcsr_get_structure(self._h, b.ctypes.data, rp.ctypes.data,
                                              ci.ctypes.data))
        self.block_sizes, self.row_ptr, self.col_idx = b, rp, ci[:inf["nnzb"]]
        Matrix._stamps += 1
        self._stamp = Matrix._stamps
        return self

    @classmethod
    def from_operator(cls, op, prec="fp64", values=None, **kw):
        """Build from a ``workloads.Operator``-like object (b, row_ptr, col_idx, values)."""
        return cls(op.b, op.row_ptr, op.col_idx, op.values if values is None else values,
                   prec=prec, **kw)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().vbcsr_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _vec(self, X, name, rows=None):
        rows = self.N if rows is None else rows
        if not isinstance(X, torch.Tensor) or not X.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % name)
        if X.dtype != self.dtype:
            raise TypeError("%s must be %s for a %s matrix" % (name, self.dtype, self.prec))
        if X.dim() == 1:
            X = X.unsqueeze(1)
        if X.dim() != 2 or X.shape[0] != rows:
            raise ValueError("%s must have %d rows" % (name, rows))
        if X.stride(1) != 1:
            X = X.contiguous()
        return X

    def info(self):
        n_rows, nnzb, nval = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        nsh = ctypes.c_int32()
        check(_lib.load().vbcsr_info(self._h, ctypes.byref(n_rows), ctypes.byref(nnzb),
                                     ctypes.byref(nval), ctypes.byref(nsh)))
        return {"N": n_rows.value, "nnzb": nnzb.value, "n_values": nval.value,
                "n_shapes": nsh.value}

    def values(self):
        """Block values in graph order (each block row-major), a device tensor."""
        out = torch.empty(self.n_values, dtype=self.dtype, device=self.device)
        check(_lib.load().vbcsr_get_values(self._h, _ptr(out), 0 if self.prec == "fp64" else 1,
                                           _stream()))
        return out

    def spgemm(self, B: "Matrix", eps: float = 0.0, path: str = "auto", nrhs_tile: int = 0,
               row_order: str = "auto"):
        """Thresholded block product ``C = A B`` (section 3.2, equations 2 and 3).

        Returns ``(C, stats)``: C is a new FP64 ``Matrix`` over the same atoms;
        ``stats`` holds the counts and phase times of the call."""
        opts = _lib.PlanOpts(0, int(nrhs_tile), _lib.PATH[path], _lib.ORDER[row_order])
        st = _lib.SpgemmStats()
        h = ctypes.c_void_p()
        check(_lib.load().vbcsr_spgemm(ctypes.byref(h), self._h, B._h, float(eps),
                                       ctypes.byref(opts), ctypes.byref(st), _stream()))
        return Matrix._adopt(h, self.n), {f: getattr(st, f) for f, _ in _lib.SpgemmStats._fields_}

    # -- values -------------------------------------------------------------
    def set_values(self, values):
        """Replace all values (graph order); a device tensor is packed by a kernel."""
        lib = _lib.load()
        if isinstance(values, torch.Tensor) and values.is_cuda:
            v = values.detach()
            if v.dtype not in (torch.float64, torch.float32):
                raise TypeError("values must be float64 or float32")
            v = v.contiguous()
            if v.numel() != self.n_values:
                raise ValueError("expected %d values" % self.n_values)
            check(lib.vbcsr_set_values(self._h, _ptr(v), 1, 0 if v.dtype == torch.float64 else 1,
                                       _stream()))
            self._keepalive = v
        else:
            v = _np(values.cpu().numpy() if isinstance(values, torch.Tensor) else values, np.float64)
            if v.size != self.n_values:
                raise ValueError("expected %d values" % self.n_values)
            check(lib.vbcsr_set_values(self._h, v.ctypes.data, 0, 0, _stream()))
        self._pages = None  # the library returned to the handle's own pages
        Matrix._stamps += 1
        self._stamp = Matrix._stamps

    # -- products -------------------------------------------------------------
    def spmm(self, X, Y=None, alpha=1.0, beta=0.0, transpose=False):
        """``Y <- alpha * op(A) X + beta * Y`` with op = identity or transpose
        (a rank-local operator maps N columns to N_rows rows)."""
        xr, yr = (self.N_rows, self.N) if transpose else (self.N, self.N_rows)
        X = self._vec(X, "X", xr)
        nrhs = X.shape[1]
        if Y is None:
            Y = torch.empty((yr, nrhs), dtype=self.dtype, device=X.device)
            beta = 0.0
        else:
            if not (isinstance(Y, torch.Tensor) and Y.is_cuda and Y.dtype == self.dtype
                    and Y.dim() == 2 and Y.shape == (yr, nrhs) and Y.stride(1) == 1):
                raise ValueError("Y must be a row-major (%d, nrhs) CUDA tensor of the matrix dtype"
                                 % yr)
        fn = _lib.load().vbcsr_spmm_t if transpose else _lib.load().vbcsr_spmm
        check(fn(self._h, _ptr(X), X.stride(0) if xr else nrhs, _ptr(Y),
                 Y.stride(0) if yr else nrhs, nrhs, float(alpha), float(beta), _stream()))
        return Y

    def spmm_t(self, X, Y=None, alpha=1.0, beta=0.0):
        return self.spmm(X, Y, alpha, beta, transpose=True)

    def __matmul__(self, X):
        return self.spmm(X)

    @property
    def T(self):
        return _Transposed(self)

    def sddmm(self, dY, X, out=None):
        """``dA_ij = dY_i X_j^T`` on the stored blocks (graph order)."""
        dY = self._vec(dY, "dY", self.N_rows)
        X = self._vec(X, "X")
        if dY.shape[1] != X.shape[1]:
            raise ValueError("dY and X need the same number of columns")
        if out is None:
            out = torch.empty(self.n_values, dtype=self.dtype, device=X.device)
        check(_lib.load().vbcsr_sddmm(self._h, _ptr(dY), dY.stride(0) if self.N_rows else dY.shape[1],
                                      _ptr(X), X.stride(0) if self.N else X.shape[1], X.shape[1],
                                      _ptr(out), _stream()))
        return out

    # -- values in the forward-page layout -----------------------------------
    @property
    def page_size(self):
        """Entries of a page-layout value buffer (values at their forward-page
        positions, zero alignment gaps and slack)."""
        n = ctypes.c_int64()
        check(_lib.load().vbcsr_page_size(self._h, ctypes.byref(n)))
        return n.value

    def _pages_arg(self, pages, name):
        if not (isinstance(pages, torch.Tensor) and pages.is_cuda and pages.device == self.device
                and pages.dtype == self.dtype and pages.dim() == 1 and pages.is_contiguous()
                and pages.numel() == self.page_size):
            raise ValueError("%s must be a contiguous %s tensor of %d entries on %s"
                             % (name, self.dtype, self.page_size, self.device))
        return pages

    def get_pages(self):
        """The current forward values in the page layout (a new device tensor)."""
        out = torch.empty(self.page_size, dtype=self.dtype, device=self.device)
        check(_lib.load().vbcsr_get_pages(self._h, _ptr(out), _stream()))
        return out

    def use_pages(self, pages):
        """Forward products read their values from ``pages`` (kept, not copied);
        ``None`` returns to the handle's own pages.  The transposed pages are
        stale until ``refresh_transposed``."""
        if pages is not None:
            self._pages_arg(pages, "pages")
        check(_lib.load().vbcsr_use_pages(self._h, None if pages is None else _ptr(pages)))
        self._pages = pages

    def refresh_transposed(self):
        """Rebuild the transposed pages from the current forward values."""
        check(_lib.load().vbcsr_refresh_transposed(self._h, _stream()))

    def sddmm_pages(self, dY, X, out=None):
        """``sddmm`` written in the page layout (zeros in the gaps)."""
        dY = self._vec(dY, "dY", self.N_rows)
        X = self._vec(X, "X")
        if dY.shape[1] != X.shape[1]:
            raise ValueError("dY and X need the same number of columns")
        if out is None:
            out = torch.empty(self.page_size, dtype=self.dtype, device=X.device)
        self._pages_arg(out, "out")
        check(_lib.load().vbcsr_sddmm_pages(self._h, _ptr(dY),
                                            dY.stride(0) if self.N_rows else dY.shape[1], _ptr(X),
                                            X.stride(0) if self.N else X.shape[1], X.shape[1],
                                            _ptr(out), _stream()))
        return out

    def cheb_workspace_bytes(self, nrhs, degree):
        b = ctypes.c_int64()
        check(_lib.load().vbcsr_cheb_workspace_bytes(self._h, int(nrhs), int(degree),
                                                     ctypes.byref(b)))
        return b.value

    def cheb_moments(self, R, degree: int, workspace=None, doubled: bool = False):
        """Chebyshev moments ``mu[k, c] = <R_c, T_k(A) R_c>`` (FP64, host array).
        ``doubled`` uses half the products (symmetric A only)."""
        R = self._vec(R, "R")
        nrhs = R.shape[1]
        mu = np.empty((degree + 1, nrhs), dtype=np.float64)
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        fn = _lib.load().vbcsr_cheb_moments_doubled if doubled else _lib.load().vbcsr_cheb_moments
        check(fn(self._h, _ptr(R), R.stride(0) if self.N else nrhs, nrhs, int(degree),
                 mu.ctypes.data, ws_ptr, ws_bytes, _stream()))
        return mu


    def cheb_step(self, Tk, Tprev, R, mu, workspace):
        """``Tprev <- 2 A Tk - Tprev`` and ``mu[c] = <R_c, Tprev_c>`` (device, FP64)."""
        Tk = self._vec(Tk, "Tk")
        nrhs = Tk.shape[1]
        if not (Tprev.is_cuda and Tprev.dtype == self.dtype and Tprev.shape == Tk.shape
                and Tprev.stride(1) == 1):
            raise ValueError("Tprev must match Tk")
        R = self._vec(R, "R")
        if mu.dtype != torch.float64 or mu.numel() < nrhs or not mu.is_cuda:
            raise ValueError("mu must be a CUDA float64 tensor of nrhs entries")
        check(_lib.load().vbcsr_cheb_step(self._h, _ptr(Tk), Tk.stride(0), _ptr(Tprev),
                                          Tprev.stride(0), _ptr(R), R.stride(0), nrhs, _ptr(mu),
                                          _ptr(workspace),
                                          workspace.numel() * workspace.element_size(),
                                          _stream()))
        return Tprev


class _Transposed:
    def __init__(self, A):
        self.A = A

    def __matmul__(self, X):
        return self.A.spmm(X, transpose=True)


class _SpmmFunction(torch.autograd.Function):
    """``Y = A(values) X`` with the hand-written backward:
    ``dX = A^T dY`` (transposed product) and ``dA_ij = dY_i X_j^T`` on the
    stored blocks (block-sampled product).  The forward always packs
    ``values`` into the handle; the backward packs them again only if another
    forward replaced them in between."""

    @staticmethod
    def forward(ctx, values, X, A):
        A.set_values(values)
        Y = A.spmm(X)
        ctx.A = A
        ctx.stamp = A._stamp
        ctx.save_for_backward(values, X)
        return Y

    @staticmethod
    def backward(ctx, G):
        values, X = ctx.saved_tensors
        A = ctx.A
        G = G.contiguous()
        if A._stamp != ctx.stamp:
            A.set_values(values)
        dV = A.sddmm(G, X) if ctx.needs_input_grad[0] else None
        dX = A.spmm_t(G) if ctx.needs_input_grad[1] else None
        if dV is not None and dV.dtype != values.dtype:
            dV = dV.to(values.dtype)
        return dV, dX, None


def spmm(values, X, A: Matrix):
    """Differentiable ``A(values) @ X`` (values in graph order)."""
    return _SpmmFunction.apply(values, X, A)


class _SpmmPagesFunction(torch.autograd.Function):
    """``Y = A(pages) X`` with the parameter in the forward-page layout
    (``Matrix.get_pages``): the forward reads ``pages`` in place, with no
    packing; the backward writes the gradient in the same layout
    (block-sampled product at the pages' positions, zero gaps) and rebuilds
    the transposed pages from ``pages`` only when ``dX`` is needed."""

    @staticmethod
    def forward(ctx, pages, X, A):
        A.use_pages(pages)
        Y = A.spmm(X)
        ctx.A = A
        ctx.save_for_backward(pages, X)
        return Y

    @staticmethod
    def backward(ctx, G):
        pages, X = ctx.saved_tensors
        A = ctx.A
        G = G.contiguous()
        A.use_pages(pages)   # another forward may have pointed the handle elsewhere
        dP = A.sddmm_pages(G, X) if ctx.needs_input_grad[0] else None
        dX = None
        if ctx.needs_input_grad[1]:
            A.refresh_transposed()
            dX = A.spmm_t(G)
        return dP, dX, None


def spmm_pages(pages, X, A: Matrix):
    """Differentiable ``A(pages) @ X`` with the values held in the operator's
    forward-page layout (``A.page_size`` entries, zero gaps)."""
    return _SpmmPagesFunction.apply(pages, X, A)
