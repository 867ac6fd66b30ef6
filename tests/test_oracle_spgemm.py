"""Pins of the oracle's thresholded block product (section 3.2, equations 2
and 3) against facts fixed independently of it: dense numpy products, SciPy's
sparse product in the scalar-block case, a brute-force evaluation of the
norm bound, the identity operator, and the guarantee that every dropped block
is below the threshold."""
import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from spgemm_util import operator_on, dense_of_blocks, blocks_dict
from test_oracle_pins import dense_of


def _structural(A, B):
    """Brute force: {(i, j)} reachable through some k, and U_ij from numpy norms."""
    Ab, Bb = blocks_dict(A), blocks_dict(B)
    U = {}
    for (i, k), a in Ab.items():
        for (k2, j), bb in Bb.items():
            if k2 == k:
                U[(i, j)] = U.get((i, j), 0.0) + np.linalg.norm(a) * np.linalg.norm(bb)
    return U


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31 - 1), n=st.integers(1, 16), density=st.floats(0.05, 0.6),
       empty=st.integers(0, 2), unsorted=st.booleans())
def test_zero_threshold_is_dense_product(seed, n, density, empty, unsorted):
    rng = np.random.default_rng(seed)
    b = rng.choice([1, 2, 3, 4, 9, 13, 17], size=n).astype(np.int32)
    A = operator_on(b, seed + 1, density, empty, unsorted)
    B = operator_on(b, seed + 2, density, empty, unsorted)
    r = oracle.spgemm(A, B, 0.0)
    ref = dense_of(A) @ dense_of(B)
    got = dense_of_blocks(b, r["rows"], r["rp"], r["col"], r["values"])
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()))
    # pattern: exactly the structurally reachable pairs, ascending per row
    U = _structural(A, B)
    pairs = {(int(i), int(r["col"][c])) for t, i in enumerate(r["rows"])
             for c in range(r["rp"][t], r["rp"][t + 1])}
    assert pairs == set(U)
    for t in range(len(r["rows"])):
        cs = r["col"][r["rp"][t]:r["rp"][t + 1]]
        assert np.all(np.diff(cs) > 0)


def test_scalar_blocks_match_scipy():
    n = 60
    b = np.ones(n, dtype=np.int32)
    A = operator_on(b, 11, 0.08)
    B = operator_on(b, 12, 0.08)
    r = oracle.spgemm(A, B, 0.0)
    As = sp.csr_matrix((A.values, A.col_idx, A.row_ptr), shape=(n, n))
    Bs = sp.csr_matrix((B.values, B.col_idx, B.row_ptr), shape=(n, n))
    Cs = (As @ Bs).toarray()
    got = dense_of_blocks(b, r["rows"], r["rp"], r["col"], r["values"])
    assert np.allclose(got, Cs, rtol=0, atol=1e-14)
    # structural pattern from SciPy's boolean product
    Ap = sp.csr_matrix((np.ones(A.nnzb), A.col_idx, A.row_ptr), shape=(n, n))
    Bp = sp.csr_matrix((np.ones(B.nnzb), B.col_idx, B.row_ptr), shape=(n, n))
    P = (Ap @ Bp).tocsr()
    P.sort_indices()
    assert np.array_equal(r["rp"], P.indptr) and np.array_equal(r["col"], P.indices)


def test_bound_of_equation_3():
    """U_ij equals the brute-force sum of norm products and bounds ||C_ij||."""
    b = np.array([4, 9, 1, 13, 9, 4, 2, 17], dtype=np.int32)
    A = operator_on(b, 21, 0.5)
    B = operator_on(b, 22, 0.5)
    r = oracle.spgemm(A, B, 0.0)
    U = _structural(A, B)
    D = dense_of(A) @ dense_of(B)
    off = np.concatenate([[0], np.cumsum(b.astype(np.int64))])
    for t, i in enumerate(r["rows"]):
        for c in range(r["sym_rp"][t], r["sym_rp"][t + 1]):
            j = int(r["sym_col"][c])
            assert r["bound"][c] == pytest.approx(U[(int(i), j)], rel=1e-14)
            blk = D[off[i]:off[i + 1], off[j]:off[j + 1]]
            assert np.linalg.norm(blk) <= r["bound"][c] * (1 + 1e-12)


@pytest.mark.parametrize("eps", [1e-3, 1e-2, 0.1, 1.0, 10.0])
def test_threshold_drops_only_small_blocks(eps):
    n = 24
    rng = np.random.default_rng(5)
    b = rng.choice([1, 4, 9, 13], size=n).astype(np.int32)
    decades = 10.0 ** rng.uniform(-3, 1, size=n)
    A = operator_on(b, 31, 0.25, scale_rows=decades)
    B = operator_on(b, 32, 0.25, scale_rows=decades[::-1].copy())
    full = oracle.spgemm(A, B, 0.0)
    r = oracle.spgemm(A, B, eps)
    U = _structural(A, B)
    # symbolic stage: kept iff U >= eps (brute-force U)
    sym = {(int(i), int(r["sym_col"][c])) for t, i in enumerate(r["rows"])
           for c in range(r["sym_rp"][t], r["sym_rp"][t + 1])}
    assert sym == {p for p, u in U.items() if u >= eps}
    assert 0 < len(sym) < len(U) or eps in (1e-3, 10.0)
    # every block of the exact product that the result lacks is below eps
    Dex = dense_of(A) @ dense_of(B)
    off = np.concatenate([[0], np.cumsum(b.astype(np.int64))])
    kept = {(int(i), int(r["col"][c])) for t, i in enumerate(r["rows"])
            for c in range(r["rp"][t], r["rp"][t + 1])}
    for (i, j) in U:
        nrm = np.linalg.norm(Dex[off[i]:off[i + 1], off[j]:off[j + 1]])
        if (i, j) not in kept:
            assert nrm < eps * (1 + 1e-12)
        else:
            assert nrm >= eps * (1 - 1e-12)
    # kept blocks carry exactly the values of the unthresholded product
    fb = {}
    pos = 0
    for t, i in enumerate(full["rows"]):
        for c in range(full["rp"][t], full["rp"][t + 1]):
            j = int(full["col"][c])
            sz = int(b[i]) * int(b[j])
            fb[(int(i), j)] = full["values"][pos:pos + sz]
            pos += sz
    pos = 0
    for t, i in enumerate(r["rows"]):
        for c in range(r["rp"][t], r["rp"][t + 1]):
            j = int(r["col"][c])
            sz = int(b[i]) * int(b[j])
            assert np.array_equal(r["values"][pos:pos + sz], fb[(int(i), j)])
            pos += sz


def test_identity_right_factor_is_exact():
    b = np.array([1, 4, 9, 13, 4, 1], dtype=np.int32)
    A = operator_on(b, 41, 0.5, unsorted=True)
    n = b.shape[0]
    from workloads.core import Operator
    vals = np.concatenate([np.eye(int(x)).ravel() for x in b])
    I = Operator("I", b, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), vals,
                 np.zeros(n))
    r = oracle.spgemm(A, I, 0.0)
    assert np.array_equal(dense_of_blocks(b, r["rows"], r["rp"], r["col"], r["values"]),
                          dense_of(A))
    r2 = oracle.spgemm(I, A, 0.0)
    assert np.array_equal(dense_of_blocks(b, r2["rows"], r2["rp"], r2["col"], r2["values"]),
                          dense_of(A))


def test_huge_threshold_gives_empty_result_and_rows_subset():
    b = np.array([4, 9, 13, 1, 9], dtype=np.int32)
    A = operator_on(b, 51, 0.6)
    B = operator_on(b, 52, 0.6)
    r = oracle.spgemm(A, B, 1e30)
    assert r["rp"][-1] == 0 and r["values"].size == 0 and r["sym_rp"][-1] == 0
    full = oracle.spgemm(A, B, 0.0)
    sub = oracle.spgemm(A, B, 0.0, rows=[3, 0, 4])
    D = dense_of_blocks(b, full["rows"], full["rp"], full["col"], full["values"])
    Ds = dense_of_blocks(b, sub["rows"], sub["rp"], sub["col"], sub["values"])
    off = np.concatenate([[0], np.cumsum(b.astype(np.int64))])
    for i in (3, 0, 4):
        assert np.array_equal(Ds[off[i]:off[i + 1]], D[off[i]:off[i + 1]])



def test_zero_blocks_survive_zero_threshold():
    """U_ij = 0 is not below a zero threshold: candidates whose every path is
    a zero block stay at eps = 0 (and their zero blocks pass the final
    filter), and are the only ones dropped at the smallest positive eps."""
    b = np.array([2, 3, 4], dtype=np.int32)
    A = operator_on(b, 61, 1.0)
    B = operator_on(b, 62, 1.0)
    base = B.block_base
    rows = B.block_rows
    for k in range(B.nnzb):
        if B.col_idx[k] == 0:                          # block column 0 of B is zero
            B.values[base[k]:base[k + 1]] = 0.0
    r = oracle.spgemm(A, B, 0.0)
    assert r["rp"][-1] == 9 and r["sym_rp"][-1] == 9
    assert np.count_nonzero(r["bound"] == 0.0) == 3
    r = oracle.spgemm(A, B, 5e-324)
    assert r["sym_rp"][-1] == 6 and 0 not in set(r["col"].tolist())
    assert rows.shape[0] == 9
