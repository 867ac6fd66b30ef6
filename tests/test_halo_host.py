"""Host-side halo plans of rank-local operators (no GPU).

The 2x2x2 spatial split of a periodic lattice into 8 ranks: ghost ordering
(owner rank, then global id), local graphs, and the exchange lists checked
against each other across ranks; then the forward product and the adjoint
with its ghost reduction are assembled on the CPU, with the oracle applied
to every rank's local operator (ghost rows empty), and compared with the
oracle's product of the whole operator.
"""
import ctypes

import numpy as np
import pytest

import oracle
from workloads import make_config
from workloads.core import Operator

from paper_2609_04397_amd import _lib
from paper_2609_04397_amd.halo import Halo


def lattice_owner(m, parts=2):
    """Atom x + m y + m^2 z of an m^3 lattice -> rank of its (parts^3) sub-cube."""
    a = np.arange(m ** 3)
    x, y, z = a % m, (a // m) % m, a // (m * m)
    w = m // parts
    return ((x // w) + parts * (y // w) + parts * parts * (z // w)).astype(np.int32)


@pytest.fixture(scope="module")
def split():
    op, vec = make_config("C2", scale=(8 / 32) ** 3, nrhs=3)   # 8^3 lattice, b = 13
    owner = lattice_owner(8)
    halos = [Halo(op.b, op.row_ptr, op.col_idx, owner, r, 8) for r in range(8)]
    return op, vec, owner, halos


def global_scalar_rows(op, H, local_rows):
    """Global scalar rows of local scalar rows of rank plan H."""
    goff = op.off
    atom = np.searchsorted(H.off, local_rows, side="right") - 1
    return goff[H.gid[atom]] + (local_rows - H.off[atom])


def test_owned_and_ghost_order(split):
    op, _, owner, halos = split
    for r, H in enumerate(halos):
        own = H.gid[:H.n_owned]
        gh = H.gid[H.n_owned:]
        assert np.array_equal(own, np.nonzero(owner == r)[0])
        assert np.all(owner[gh] != r)
        keys = owner[gh].astype(np.int64) * op.n + gh
        assert np.all(np.diff(keys) > 0)                 # (owner, global id) ascending
        # the ghosts are exactly the foreign columns of the owned rows
        cols = np.unique(np.concatenate([op.col_idx[op.row_ptr[i]:op.row_ptr[i + 1]] for i in own]))
        assert np.array_equal(np.sort(gh), cols[owner[cols] != r])
        # couplings reach the 1st and 2nd shells (face and edge neighbours):
        # a rank's sub-cube borders the 3 face- and 3 edge-adjacent ones,
        # not the one across the corner
        assert np.count_nonzero(np.diff(H.recv_ptr)) == 6
        assert H.recv_ptr[7 - r + 1] == H.recv_ptr[7 - r]


def test_local_graph_and_values(split):
    op, _, _, halos = split
    base = op.block_base
    for H in halos:
        assert np.array_equal(H.block_sizes, op.b[H.gid])
        vals = H.local_values(op.values)
        at = 0
        for u in range(H.n_owned):
            i = H.gid[u]
            loc = H.col_idx[H.row_ptr[u]:H.row_ptr[u + 1]]
            assert np.array_equal(H.gid[loc], op.col_idx[op.row_ptr[i]:op.row_ptr[i + 1]])
            g0, g1 = base[op.row_ptr[i]], base[op.row_ptr[i + 1]]
            assert np.array_equal(vals[at:at + g1 - g0], op.values[g0:g1])
            at += g1 - g0
        assert at == H.n_values


def test_send_lists_match_the_receivers_ghost_rows(split):
    op, _, _, halos = split
    for r, Hr in enumerate(halos):
        for s, Hs in enumerate(halos):
            a, b = Hr.send_range(s)
            lo, hi = Hs.ghost_range(r)
            sent = global_scalar_rows(op, Hr, Hr.send_rows[a:b].astype(np.int64))
            ghost = global_scalar_rows(op, Hs, np.arange(lo, hi))
            assert np.array_equal(sent, ghost), (r, s)
            if r == s:
                assert a == b


def test_reduction_map(split):
    _, _, _, halos = split
    for H in halos:
        assert np.all(np.diff(H.red_rows) > 0)
        assert np.all(H.red_rows < H.N_rows)
        assert np.array_equal(np.sort(H.red_pos), np.arange(H.n_send_rows))
        for u in range(H.red_rows.shape[0]):
            pos = H.red_pos[H.red_ptr[u]:H.red_ptr[u + 1]]
            assert np.all(np.diff(pos) > 0)
            assert np.all(H.send_rows[pos] == H.red_rows[u])


def _square_local(H, op):
    """The local operator as a square one over owned + ghost atoms (ghost rows empty)."""
    rp = np.concatenate([H.row_ptr, np.full(H.n_ghost, H.row_ptr[-1])])
    return Operator("local", H.block_sizes, rp, H.col_idx, H.local_values(op.values),
                    np.zeros(H.nnzb))


def test_exchange_assembles_the_global_products_on_cpu(split):
    """Forward: send buffers copied into the receivers' ghost rows, then the
    local products; adjoint: local transposed products, ghost rows returned
    to their owners and added through the reduction map."""
    op, vec, owner, halos = split
    X = vec["X"]
    goff = op.off
    own_rows = [global_scalar_rows(op, H, np.arange(H.N_rows)) for H in halos]
    # forward
    Xext = []
    for H, rows in zip(halos, own_rows):
        E = np.zeros((H.N, X.shape[1]))
        E[:H.N_rows] = X[rows]
        Xext.append(E)
    for r, Hr in enumerate(halos):
        buf = Xext[r][Hr.send_rows]
        for s, Hs in enumerate(halos):
            a, b = Hr.send_range(s)
            lo, hi = Hs.ghost_range(r)
            Xext[s][lo:hi] = buf[a:b]
    Y = np.zeros_like(X)
    for H, rows, E in zip(halos, own_rows, Xext):
        Y[rows] = oracle.spmm(_square_local(H, op), E)[:H.N_rows]
    ref = oracle.spmm(op, X)
    assert np.max(np.abs(Y - ref) / oracle.abs_product(op, X)) <= 1e-14
    # adjoint
    G = np.random.default_rng(3).standard_normal(X.shape)
    Yt = [oracle.spmm_t(_square_local(H, op), np.vstack([G[rows], np.zeros((H.N - H.N_rows, 3))]))
          for H, rows in zip(halos, own_rows)]
    recv = [np.zeros((H.n_send_rows, 3)) for H in halos]
    for r, Hr in enumerate(halos):
        for s, Hs in enumerate(halos):
            lo, hi = Hr.ghost_range(s)
            a, b = Hs.send_range(r)
            recv[s][a:b] = Yt[r][lo:hi]
    Z = np.zeros_like(G)
    for H, rows, Yl, buf in zip(halos, own_rows, Yt, recv):
        out = Yl[:H.N_rows].copy()
        for u, row in enumerate(H.red_rows):
            for e in range(H.red_ptr[u], H.red_ptr[u + 1]):
                out[row] += buf[H.red_pos[e]]
        Z[rows] = out
    ref = oracle.spmm_t(op, G)
    assert np.max(np.abs(Z - ref) / oracle.abs_product(op, G, transpose_op=True)) <= 1e-14


def test_plan_errors():
    lib = _lib.load()
    b = np.array([2, 3], np.int32)
    rp = np.array([0, 2, 3], np.int64)
    ci = np.array([0, 1, 1], np.int32)
    own = np.array([0, 1], np.int32)
    h = ctypes.c_void_p()
    call = lambda o, r, n: lib.vbcsr_halo_create(ctypes.byref(h), 2, b.ctypes.data, rp.ctypes.data,
                                                  ci.ctypes.data, o.ctypes.data, r, n)
    assert call(own, 2, 2) == _lib.VBCSR_EINVAL                       # rank >= n_ranks
    assert call(np.array([0, 5], np.int32), 0, 2) == _lib.VBCSR_EINVAL  # owner out of range
    ci_dup = np.array([0, 0, 1], np.int32)
    assert lib.vbcsr_halo_create(ctypes.byref(h), 2, b.ctypes.data, rp.ctypes.data,
                                 ci_dup.ctypes.data, own.ctypes.data, 0, 2) == _lib.VBCSR_EDUP
    assert call(own, 0, 2) == _lib.VBCSR_OK
    lib.vbcsr_halo_destroy(h)
