"""Pins of the CPU oracle against facts fixed independently of it.

Each test checks the oracle against something other than itself: a dense
numpy product, SciPy's BSR and CSR kernels (the uniform-block and scalar
special cases of the block model), adjoint identities, symmetry, closed forms
of the Chebyshev recurrence, exactness of central differences for a bilinear
loss, and a hand-derived worked example.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from metrics import rel_f, comp, load_golden
from workloads import random_pattern, sc_lattice, make_config
from workloads.core import Operator

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_of(op, values=None):
    """Dense matrix assembled block by block with numpy slicing."""
    v = op.values if values is None else values
    off = op.off
    D = np.zeros((op.N, op.N))
    base = op.block_base
    rows = op.block_rows
    for k in range(op.nnzb):
        i, j = int(rows[k]), int(op.col_idx[k])
        bi, bj = int(op.b[i]), int(op.b[j])
        D[off[i]:off[i] + bi, off[j]:off[j] + bj] += v[base[k]:base[k + 1]].reshape(bi, bj)
    return D


def test_golden_two_atom_example():
    g = load_golden(os.path.join(GOLDEN, "two_atom_example.txt"))
    b = np.array(g["block_sizes"], dtype=np.int32)
    rp = np.array(g["row_ptr"], dtype=np.int64)
    ci = np.array(g["col_idx"], dtype=np.int32)
    v = np.array(g["values"])
    nrhs = int(g["nrhs"][0])
    X = np.array(g["X"]).reshape(-1, nrhs)
    op = Operator("golden", b, rp, ci, v, np.zeros(ci.shape[0]))
    assert np.array_equal(oracle.spmm(op, X), np.array(g["AX"]).reshape(-1, nrhs))
    assert np.array_equal(oracle.spmm_t(op, X), np.array(g["AtX"]).reshape(-1, nrhs))
    dY = np.array(g["dY"]).reshape(-1, nrhs)
    assert np.array_equal(oracle.sddmm(op, dY, X), np.array(g["sddmm"]))


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31 - 1), n=st.integers(1, 24),
       density=st.floats(0.05, 0.6), empty=st.integers(0, 3), unsorted=st.booleans(),
       nrhs=st.integers(1, 5))
def test_forward_matches_dense(seed, n, density, empty, unsorted, nrhs):
    op = random_pattern(seed, n, bset=(1, 2, 3, 4, 5, 9, 13), density=density,
                        empty_rows=empty, unsorted=unsorted)
    rng = np.random.default_rng(seed + 1)
    X = rng.standard_normal((op.N, nrhs))
    D = dense_of(op)
    ref = D @ X
    Y = oracle.spmm(op, X)
    assert comp(Y, ref, np.abs(D) @ np.abs(X)) <= 1e-14
    Yt = oracle.spmm_t(op, X)
    assert comp(Yt, D.T @ X, np.abs(D.T) @ np.abs(X)) <= 1e-14


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (2.5, 0.0), (-0.5, 1.0), (2.0, -1.0), (0.0, 3.0)])
def test_alpha_beta(alpha, beta):
    op = random_pattern(7, 20, density=0.3, empty_rows=2)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((op.N, 3))
    Y0 = rng.standard_normal((op.N, 3))
    D = dense_of(op)
    ref = alpha * (D @ X) + beta * Y0
    Y = oracle.spmm(op, X, alpha=alpha, beta=beta, Y=Y0)
    scale = abs(alpha) * (np.abs(D) @ np.abs(X)) + abs(beta) * np.abs(Y0)
    assert comp(Y, ref, scale) <= 1e-14


def test_beta_zero_ignores_nan():
    op = random_pattern(3, 10, density=0.3)
    X = np.ones((op.N, 2))
    Y0 = np.full((op.N, 2), np.nan)
    Y = oracle.spmm(op, X, beta=0.0, Y=Y0)
    assert np.all(np.isfinite(Y))


@pytest.mark.parametrize("bsize,m", [(13, 3), (13, 4), (3, 5)])
def test_uniform_blocks_match_scipy_bsr(bsize, m):
    op = sc_lattice(m, bsize, seed=11)
    data = op.values.reshape(op.nnzb, bsize, bsize)
    A = sp.bsr_matrix((data, op.col_idx, op.row_ptr), shape=(op.N, op.N))
    X = np.random.default_rng(12).standard_normal((op.N, 4))
    ref = A @ X
    scale = abs(A) @ np.abs(X)
    assert comp(oracle.spmm(op, X), ref, scale) <= 1e-14
    assert comp(oracle.spmm_t(op, X), A.T @ X, abs(A.T) @ np.abs(X)) <= 1e-14


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_scalar_blocks_match_scipy_csr(seed):
    op = random_pattern(seed, 200, bset=(1,), density=0.05, empty_rows=5, unsorted=True)
    A = sp.csr_matrix((op.values, op.col_idx, op.row_ptr), shape=(op.N, op.N))
    X = np.random.default_rng(seed).standard_normal((op.N, 3))
    assert comp(oracle.spmm(op, X), A @ X, abs(A) @ np.abs(X)) <= 1e-14


def test_expansion_structure():
    op = random_pattern(5, 30, density=0.2, empty_rows=3, unsorted=True)
    A = oracle.expand_op(op)
    assert A.rp[0] == 0 and np.all(np.diff(A.rp) >= 0)
    assert A.nnz == op.nnz
    assert np.allclose(np.sort(A.va), np.sort(op.values))
    D = dense_of(op)
    Ad = sp.csr_matrix((A.va, A.ci, A.rp), shape=(op.N, op.N)).toarray()
    assert np.array_equal(Ad, D)


@pytest.mark.parametrize("seed", [21, 22])
def test_adjoint_dot_identity(seed):
    op = random_pattern(seed, 40, density=0.2, empty_rows=2, unsorted=True)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((op.N, 4))
    W = rng.standard_normal((op.N, 4))
    lhs = np.sum(oracle.spmm(op, X) * W)
    rhs = np.sum(X * oracle.spmm_t(op, W))
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(oracle.abs_product(op, X)) * np.abs(W)).sum()


@pytest.mark.parametrize("name,scale", [("C1", 0.2), ("C3", 0.003), ("FD50", 1.0), ("C5", 0.003)])
def test_symmetric_operator_transpose_equals_forward(name, scale):
    op, vec = make_config(name, scale=scale, nrhs=3)
    X = vec["X"]
    Y = oracle.spmm(op, X)
    Yt = oracle.spmm_t(op, X)
    assert comp(Yt, Y, oracle.abs_product(op, X)) <= 1e-14


def test_identity_operator_is_bitwise_identity():
    b = np.array([1, 4, 9, 13, 2], dtype=np.int32)
    n = b.size
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    vals = np.concatenate([np.eye(int(x)).ravel() for x in b])
    op = Operator("eye", b, rp, ci, vals, np.zeros(n))
    X = np.random.default_rng(0).standard_normal((op.N, 7))
    assert np.array_equal(oracle.spmm(op, X), X)
    assert np.array_equal(oracle.spmm_t(op, X), X)


def test_block_diagonal_is_independent_dense_products():
    rng = np.random.default_rng(4)
    b = np.array([3, 1, 5, 2], dtype=np.int32)
    n = b.size
    blocks = [rng.standard_normal((int(x), int(x))) for x in b]
    op = Operator("bdiag", b, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                  np.concatenate([m.ravel() for m in blocks]), np.zeros(n))
    X = rng.standard_normal((op.N, 2))
    off = op.off
    Y = oracle.spmm(op, X)
    for i, m in enumerate(blocks):
        ref = m @ X[off[i]:off[i + 1]]
        assert comp(Y[off[i]:off[i + 1]], ref, np.abs(m) @ np.abs(X[off[i]:off[i + 1]])) <= 1e-15


def test_sddmm_brute_force():
    op = random_pattern(9, 8, bset=(1, 2, 3), density=0.5, unsorted=True)
    rng = np.random.default_rng(10)
    dY = rng.standard_normal((op.N, 3))
    X = rng.standard_normal((op.N, 3))
    got = oracle.sddmm(op, dY, X)
    off, base, rows = op.off, op.block_base, op.block_rows
    for k in range(op.nnzb):
        i, j = int(rows[k]), int(op.col_idx[k])
        for p in range(op.b[i]):
            for q in range(op.b[j]):
                want = sum(dY[off[i] + p, c] * X[off[j] + q, c] for c in range(3))
                assert abs(got[base[k] + p * op.b[j] + q] - want) <= 1e-14 * (1 + abs(want))


def test_sddmm_is_adjoint_of_value_map():
    """sum_k <dA_k, E_k> == <G, A(E) X> for any values E on the pattern."""
    op = random_pattern(12, 30, density=0.25, empty_rows=2, unsorted=True)
    rng = np.random.default_rng(13)
    G = rng.standard_normal((op.N, 4))
    X = rng.standard_normal((op.N, 4))
    E = rng.standard_normal(op.nnz)
    lhs = np.dot(oracle.sddmm(op, G, X), E)
    rhs = np.sum(G * oracle.spmm(op, X, values=E))
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


def test_gradient_central_differences_are_exact():
    """L(V, X) = sum((A(V) X) * G) is bilinear, so central differences are
    exact up to rounding for any step; compare with sddmm and spmm_t."""
    op, vec = make_config("FD50")
    X, G = vec["X"], vec["G"]
    V = op.values
    dV = oracle.sddmm(op, G, X)
    dX = oracle.spmm_t(op, G)

    def loss(v, x):
        return float(np.sum(oracle.spmm(op, x, values=v) * G))

    rng = np.random.default_rng(99)
    h = 1e-3
    for e in rng.choice(V.size, 200, replace=False):
        vp, vm = V.copy(), V.copy()
        vp[e] += h
        vm[e] -= h
        fd = (loss(vp, X) - loss(vm, X)) / (2 * h)
        assert abs(fd - dV[e]) <= 1e-9 * max(1.0, abs(dV[e]))
    for e in rng.choice(X.size, 100, replace=False):
        xp, xm = X.copy(), X.copy()
        xp.flat[e] += h
        xm.flat[e] -= h
        fd = (loss(V, xp) - loss(V, xm)) / (2 * h)
        assert abs(fd - dX.flat[e]) <= 1e-9 * max(1.0, abs(dX.flat[e]))


def _diag_op(diag_blocks):
    b = np.array([m.shape[0] for m in diag_blocks], dtype=np.int32)
    n = b.size
    return Operator("diag", b, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                    np.concatenate([m.ravel() for m in diag_blocks]), np.zeros(n))


def test_chebyshev_diagonal_closed_form():
    """For a diagonal operator T_k(a) = cos(k arccos a) elementwise."""
    rng = np.random.default_rng(5)
    a = rng.uniform(-0.99, 0.99, size=40)
    blocks, pos = [], 0
    for s in (1, 3, 4, 2, 5, 9, 13, 3):
        blocks.append(np.diag(a[pos:pos + s]))
        pos += s
    op = _diag_op(blocks)
    d = np.diag(np.block([[blocks[i] if i == j else np.zeros((blocks[i].shape[0], blocks[j].shape[0]))
                           for j in range(len(blocks))] for i in range(len(blocks))]))
    R = rng.standard_normal((op.N, 3))
    deg = 64
    mu = oracle.cheb_moments(op, R, deg)
    k = np.arange(deg + 1)[:, None]
    ref = np.cos(k * np.arccos(d))[:, :, None] * (R * R)[None, :, :]
    ref = ref.sum(axis=1)
    assert np.max(np.abs(mu - ref)) <= 1e-12 * np.max(np.abs(ref[0]))


def test_chebyshev_ring_trace():
    """A b=1 ring with hopping t has eigenvalues 2t cos(2 pi m / n); with R = I
    the column sum of mu_k is trace T_k(A) = sum_m T_k(lambda_m)."""
    n, t = 37, 0.45
    rows, cols = [], []
    for i in range(n):
        for j in sorted({(i - 1) % n, (i + 1) % n}):
            rows.append(i)
            cols.append(j)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    op = Operator("ring", np.ones(n, np.int32), rp, np.array(cols, np.int32),
                  np.full(len(cols), t), np.zeros(len(cols)))
    R = np.eye(n)
    deg = 64
    mu = oracle.cheb_moments(op, R, deg).sum(axis=1)
    lam = 2 * t * np.cos(2 * np.pi * np.arange(n) / n)
    ref = np.array([np.cos(k * np.arccos(lam)).sum() for k in range(deg + 1)])
    assert np.max(np.abs(mu - ref)) <= 1e-11 * n
    # cross-check the eigenvalues themselves with a dense eigensolver
    D = dense_of(op)
    assert np.allclose(np.sort(np.linalg.eigvalsh(D)), np.sort(lam), atol=1e-12)


def test_chebyshev_moment_bound_on_scaled_operator():
    op, vec = make_config("C4", scale=0.004, nrhs=4)
    mu = oracle.cheb_moments(op, vec["R"], 64)
    assert np.all(np.abs(mu) <= mu[0][None, :] * (1 + 1e-12))
    assert np.allclose(mu[0], (vec["R"] ** 2).sum(axis=0), rtol=1e-14)


def test_thread_count_does_not_change_bits():
    op, vec = make_config("C1", scale=0.3, nrhs=4)
    A = oracle.expand_op(op)
    t0 = oracle.max_threads()
    try:
        oracle.set_threads(1)
        y1 = oracle.csr_spmm(A, vec["X"])
        oracle.set_threads(max(2, t0))
        y2 = oracle.csr_spmm(A, vec["X"])
    finally:
        oracle.set_threads(t0)
    assert np.array_equal(y1, y2)
