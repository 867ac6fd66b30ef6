"""Rank-local operators and their halo exchange lists (marshalling only).

``Halo`` wraps one ``vbcsr_halo`` plan: one rank's share of a distributed
block graph (paper, section 3.1: owned atoms, ghosts ordered by owner rank
then global id) with the send, receive and reduction lists of the forward
halo fetch and the adjoint's return of ghost contributions (section 3.2).
The plan is host code of the library; packing send buffers and adding
returned contributions run in its kernels.  Moving the buffers between ranks
is the caller's: device copies when the ranks share one GPU.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .matrix import Matrix, _ptr, _stream


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Halo:
    """The plan of rank ``rank`` of ``n_ranks`` for the global block graph
    (``block_sizes``, ``row_ptr``, ``col_idx``) with atom owners ``owner``."""

    def __init__(self, block_sizes, row_ptr, col_idx, owner, rank: int, n_ranks: int):
        lib = _lib.load()
        b = _np(block_sizes, np.int32)
        rp = _np(row_ptr, np.int64)
        ci = _np(col_idx, np.int32)
        own = _np(owner, np.int32)
        h = ctypes.c_void_p()
        check(lib.vbcsr_halo_create(ctypes.byref(h), int(b.shape[0]), b.ctypes.data, rp.ctypes.data,
                                    ci.ctypes.data if ci.size else None, own.ctypes.data,
                                    int(rank), int(n_ranks)))
        self._h = h
        self.rank, self.n_ranks = int(rank), int(n_ranks)
        no, ng = ctypes.c_int32(), ctypes.c_int32()
        nb, nv, ns, nr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib.vbcsr_halo_info(h, ctypes.byref(no), ctypes.byref(ng), ctypes.byref(nb),
                                  ctypes.byref(nv), ctypes.byref(ns), ctypes.byref(nr)))
        self.n_owned, self.n_ghost = no.value, ng.value
        self.nnzb, self.n_values = nb.value, nv.value
        nl = self.n_owned + self.n_ghost
        self.gid = np.empty(nl, np.int32)
        self.block_sizes = np.empty(nl, np.int32)
        self.row_ptr = np.empty(self.n_owned + 1, np.int64)
        self.col_idx = np.empty(max(self.nnzb, 1), np.int32)
        check(lib.vbcsr_halo_graph(h, self.gid.ctypes.data, self.block_sizes.ctypes.data,
                                   self.row_ptr.ctypes.data, self.col_idx.ctypes.data))
        self.col_idx = self.col_idx[:self.nnzb]
        self.send_ptr = np.empty(self.n_ranks + 1, np.int64)
        self.send_rows = np.empty(max(ns.value, 1), np.int32)
        self.recv_ptr = np.empty(self.n_ranks + 1, np.int64)
        self.red_rows = np.empty(max(nr.value, 1), np.int32)
        self.red_ptr = np.empty(nr.value + 1, np.int64)
        self.red_pos = np.empty(max(ns.value, 1), np.int64)
        check(lib.vbcsr_halo_lists(h, self.send_ptr.ctypes.data, self.send_rows.ctypes.data,
                                   self.recv_ptr.ctypes.data, self.red_rows.ctypes.data,
                                   self.red_ptr.ctypes.data, self.red_pos.ctypes.data))
        self.send_rows = self.send_rows[:ns.value]
        self.red_rows = self.red_rows[:nr.value]
        self.red_pos = self.red_pos[:ns.value]
        off = np.zeros(nl + 1, np.int64)
        np.cumsum(self.block_sizes, out=off[1:])
        self.off = off
        self.N_rows = int(off[self.n_owned])   # owned scalar rows
        self.N = int(off[nl])                  # owned + ghost scalar rows
        self._dev = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().vbcsr_halo_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def local_values(self, global_values) -> np.ndarray:
        """The owned rows' block values, local graph order (host)."""
        gv = _np(global_values, np.float64)
        out = np.empty(max(self.n_values, 1))
        check(_lib.load().vbcsr_halo_local_values(self._h, gv.ctypes.data, out.ctypes.data))
        return out[:self.n_values]

    def matrix(self, values=None, prec: str = "fp64", **kw) -> Matrix:
        """The rank-local operator (``vbcsr_create_local``) with ``values`` in
        local graph order (``local_values``)."""
        return Matrix(self.block_sizes, self.row_ptr, self.col_idx, values, prec=prec,
                      n_ghost=self.n_ghost, **kw)

    def _lists(self):
        if self._dev is None:
            d = torch.device("cuda", torch.cuda.current_device())
            t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(d, dt)
            self._dev = {"send_rows": t(self.send_rows, torch.int32),
                         "red_rows": t(self.red_rows, torch.int32),
                         "red_ptr": t(self.red_ptr, torch.int64),
                         "red_pos": t(self.red_pos, torch.int64)}
        return self._dev

    @property
    def n_send_rows(self):
        return int(self.send_rows.shape[0])

    def send_range(self, s):
        return int(self.send_ptr[s]), int(self.send_ptr[s + 1])

    def ghost_range(self, s):
        """Local scalar rows of the ghosts owned by rank ``s``."""
        return self.N_rows + int(self.recv_ptr[s]), self.N_rows + int(self.recv_ptr[s + 1])

    def pack(self, X, buf=None):
        """Send buffer ``buf[t] = X[send_rows[t]]`` (``X``: this rank's
        vector, at least its owned rows) on the device."""
        L = self._lists()
        nrhs = X.shape[1]
        if buf is None:
            buf = torch.empty((self.n_send_rows, nrhs), dtype=X.dtype, device=X.device)
        dt = {torch.float64: 0, torch.float32: 1}[X.dtype]
        check(_lib.load().vbcsr_halo_pack(_ptr(X), X.shape[0], X.stride(0), _ptr(L["send_rows"]),
                                          self.n_send_rows, nrhs, dt, _ptr(buf),
                                          buf.stride(0) if self.n_send_rows else nrhs, _stream()))
        return buf

    def reduce(self, Y, buf):
        """Add the returned contributions ``buf`` (the layout of this rank's
        send buffer) to their owned rows of ``Y``."""
        L = self._lists()
        nrhs = Y.shape[1]
        dt = {torch.float64: 0, torch.float32: 1}[Y.dtype]
        check(_lib.load().vbcsr_halo_reduce(_ptr(Y), Y.shape[0], Y.stride(0), _ptr(L["red_rows"]),
                                            _ptr(L["red_ptr"]), _ptr(L["red_pos"]),
                                            int(self.red_rows.shape[0]), _ptr(buf),
                                            int(buf.shape[0]),
                                            buf.stride(0) if buf.shape[0] else nrhs, nrhs, dt,
                                            _stream()))
        return Y
