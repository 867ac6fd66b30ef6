"""Thresholded block product on the GPU (C ABI) against the oracle.

Patterns (integer work) must match exactly; a block may differ only where its
bound or its norm lies within rounding of the threshold (both sides then took
a valid decision).  Values are compared elementwise against the FP64 oracle
within a bound proportional to |A| |B| (the scale of the rounding error of a
dot product of at most a few hundred terms).
"""
import numpy as np
import pytest
import torch

import oracle
from spgemm_util import operator_on
from workloads import make_config
from workloads.configs import make_operator
from workloads.core import Operator

pytestmark = pytest.mark.gpu

from paper_2609_04397_amd import _lib
from paper_2609_04397_amd.matrix import Matrix

ELEM_TOL = 1e-13     # times (|A| |B|)_pq
TIE = 1e-12          # relative distance to eps within which either decision is valid


def absop(op):
    return Operator(op.name + "-abs", op.b, op.row_ptr, op.col_idx, np.abs(op.values), op.dist)


def gpu_product(A, B, eps, **kw):
    Am, Bm = Matrix.from_operator(A, **kw), Matrix.from_operator(B, **kw)
    C, st = Am.spgemm(Bm, eps)
    vals = C.values().cpu().numpy() if C.n_values else np.zeros(0)
    return Am, Bm, C, st, vals


def blocks_of(b, rows, rp, col, vals):
    out = {}
    pos = 0
    for t, i in enumerate(rows):
        for c in range(rp[t], rp[t + 1]):
            j = int(col[c])
            sz = int(b[i]) * int(b[j])
            out[(int(i), j)] = vals[pos:pos + sz]
            pos += sz
    return out


def compare(A, B, eps, C, vals, rows=None):
    """Pattern and values of the device result C against the oracle, on the
    block rows `rows` (all by default)."""
    b = A.b
    n = A.n
    rows = np.arange(n) if rows is None else np.asarray(rows)
    ref = oracle.spgemm(A, B, eps, rows=rows)
    # device result restricted to the rows
    vbase = np.zeros(C.col_idx.shape[0] + 1, dtype=np.int64)
    crow = np.repeat(np.arange(n), np.diff(C.row_ptr))
    np.cumsum(b[crow].astype(np.int64) * b[C.col_idx].astype(np.int64), out=vbase[1:])
    got = {}
    for i in rows:
        for c in range(C.row_ptr[i], C.row_ptr[i + 1]):
            got[(int(i), int(C.col_idx[c]))] = vals[vbase[c]:vbase[c + 1]]
        cs = C.col_idx[C.row_ptr[i]:C.row_ptr[i + 1]]
        assert np.all(np.diff(cs) > 0), "columns not ascending in row %d" % i
    exp = blocks_of(b, rows, ref["rp"], ref["col"], ref["values"])
    diff = set(got) ^ set(exp)
    if diff:
        # either decision is valid only at a near-tie of the bound or the norm
        full = oracle.spgemm(A, B, 0.0, rows=sorted({i for i, _ in diff}))
        U = {}
        N = {}
        fb = blocks_of(b, full["rows"], full["sym_rp"], full["sym_col"], full["sym_values"])
        for t, i in enumerate(full["rows"]):
            for c in range(full["sym_rp"][t], full["sym_rp"][t + 1]):
                U[(int(i), int(full["sym_col"][c]))] = full["bound"][c]
        for p in diff:
            N[p] = np.linalg.norm(fb[p])
            near = abs(U[p] - eps) <= TIE * eps or abs(N[p] - eps) <= TIE * eps
            assert near, "block %s differs: bound %.17g norm %.17g eps %.17g" % (p, U[p], N[p], eps)
    common = set(got) & set(exp)
    if not common:
        return 0
    absref = oracle.spgemm(absop(A), absop(B), 0.0, rows=rows)
    scale = blocks_of(b, rows, absref["sym_rp"], absref["sym_col"], absref["sym_values"])
    worst = 0.0
    for p in common:
        g, e, s = got[p], exp[p], scale[p]
        assert g.shape == e.shape
        err = np.abs(g - e) / np.maximum(s, 1e-300)
        worst = max(worst, float(err.max()))
    assert worst <= ELEM_TOL, "componentwise error %.3e" % worst
    return len(common)


@pytest.mark.parametrize("case", [
    dict(bset=(1, 2, 3, 4, 9, 13), n=40, density=0.15),
    dict(bset=(9, 12, 16, 17, 20), n=30, density=0.2),
    dict(bset=(1, 33, 64, 5), n=12, density=0.4),
    dict(bset=(13,), n=50, density=0.1),
])
@pytest.mark.parametrize("mode", ["zero", "symbolic", "final"])
def test_spgemm_random(case, mode):
    print("case spgemm random", case, mode, flush=True)
    rng = np.random.default_rng(case["n"])
    b = rng.choice(np.asarray(case["bset"], np.int32), size=case["n"]).astype(np.int32)
    decades = 10.0 ** rng.uniform(-2, 1, size=case["n"])
    A = operator_on(b, 1, case["density"], empty_rows=2, unsorted=True, scale_rows=decades)
    B = operator_on(b, 2, case["density"], empty_rows=1, scale_rows=decades[::-1].copy())
    full = oracle.spgemm(A, B, 0.0)
    if mode == "zero":
        eps = 0.0
    elif mode == "symbolic":
        eps = float(np.quantile(full["bound"], 0.4))
    else:  # between norm and bound of many blocks: the final filter acts
        eps = float(np.quantile(full["norms"], 0.5))
    Am, Bm, C, st, vals = gpu_product(A, B, eps)
    ncommon = compare(A, B, eps, C, vals)
    assert st["nnzb"] == C.col_idx.shape[0]
    assert st["kept_symbolic"] >= st["nnzb"]
    if mode == "zero":
        assert st["kept_symbolic"] == st["candidates"] == ncommon
    assert ncommon > 0


@pytest.mark.parametrize("name,scale", [("C1", 1.0), ("C5", 0.01), ("C2", 0.05), ("G1", 0.03),
                                        ("C3", 0.002)])
@pytest.mark.parametrize("eps", [0.0, 0.5])
def test_spgemm_workloads(name, scale, eps):
    op = make_operator(name, scale)
    print("case spgemm", name, scale, eps, op.n, flush=True)
    Am, Bm, C, st, vals = gpu_product(op, op, eps)
    compare(op, op, eps, C, vals)
    assert st["products"] > 0 and st["flops"] > 0


def test_spgemm_result_is_an_operator_and_deterministic():
    op = make_operator("C1", 0.3)
    A, B, C, st, vals = gpu_product(op, op, 0.0)
    X = torch.randn(op.N, 5, dtype=torch.float64, device="cuda")
    Y1 = C.spmm(X)
    Y2 = A.spmm(B.spmm(X))
    err = (Y1 - Y2).norm() / Y2.norm()
    assert float(err) <= 1e-12
    Y1t = C.spmm_t(X)
    Y2t = B.spmm_t(A.spmm_t(X))
    assert float((Y1t - Y2t).norm() / Y2t.norm()) <= 1e-12
    C2, _ = A.spgemm(B, 0.0)
    assert torch.equal(C2.values(), C.values())


def test_spgemm_edge_cases():
    b = np.array([4, 9, 1, 13], dtype=np.int32)
    empty = Operator("empty", b, np.zeros(5, np.int64), np.zeros(0, np.int32), np.zeros(0),
                     np.zeros(0))
    A = operator_on(b, 5, 0.6)
    for X, Y in ((empty, A), (A, empty), (empty, empty)):
        _, _, C, st, vals = gpu_product(X, Y, 0.0)
        assert C.info()["nnzb"] == 0 and st["products"] == 0
        Z = C.spmm(torch.ones(C.N, 2, dtype=torch.float64, device="cuda"))
        assert float(Z.abs().max()) == 0.0
    _, _, C, st, vals = gpu_product(A, A, 1e300)
    assert C.info()["nnzb"] == 0 and st["kept_symbolic"] == 0
    one = Operator("one", np.array([7], np.int32), np.array([0, 1], np.int64),
                   np.array([0], np.int32), np.arange(49, dtype=np.float64) / 49, np.zeros(1))
    _, _, C, st, vals = gpu_product(one, one, 0.0)
    M = one.values.reshape(7, 7)
    assert np.allclose(vals.reshape(7, 7), M @ M, rtol=1e-14, atol=0)


def test_spgemm_errors():
    b = np.array([4, 9, 1], dtype=np.int32)
    A = operator_on(b, 7, 0.7)
    Am = Matrix.from_operator(A)
    Af = Matrix.from_operator(A, prec="fp32")
    with pytest.raises(_lib.VbcsrError) as e:
        Af.spgemm(Af)
    assert e.value.code == _lib.VBCSR_EUNSUPPORTED
    for bad in (-1.0, float("nan")):
        with pytest.raises(_lib.VbcsrError) as e:
            Am.spgemm(Am, bad)
        assert e.value.code == _lib.VBCSR_EINVAL
    Bo = operator_on(np.array([4, 9, 2], dtype=np.int32), 8, 0.7)
    with pytest.raises(_lib.VbcsrError) as e:
        Am.spgemm(Matrix.from_operator(Bo))
    assert e.value.code == _lib.VBCSR_EINVAL
    with pytest.raises(_lib.VbcsrError):
        Matrix.from_operator(A, prec="bf16x3").values()


def test_get_values_roundtrip():
    op = make_operator("C5", 0.005)
    for prec in ("fp64", "fp32"):
        M = Matrix.from_operator(op, prec=prec)
        v = M.values().double().cpu().numpy()
        ref = op.values if prec == "fp64" else op.values.astype(np.float32).astype(np.float64)
        assert np.array_equal(v, ref)
        b, rp, ci = M.block_sizes, M.row_ptr, M.col_idx
        assert np.array_equal(b, op.b) and np.array_equal(rp, op.row_ptr)


@pytest.mark.parametrize("eps", [0.0, 1.0])
def test_spgemm_g1_full_size_sampled(eps):
    """The benchmarked product (G1, about 500 MiB of FP64 values, A A) on
    sampled block rows, including the first and last."""
    op = make_operator("G1")
    print("case spgemm G1 full", eps, op.n, flush=True)
    Am, Bm, C, st, vals = gpu_product(op, op, eps)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([[0, op.n - 1], rng.choice(op.n, 60, replace=False)]))
    assert compare(op, op, eps, C, vals, rows=rows) > 0
    if eps > 0:   # the threshold acts in both stages at this size
        assert st["kept_symbolic"] < st["candidates"] and st["nnzb"] < st["kept_symbolic"]
    print("G1 stats", st, flush=True)


def test_spgemm_result_planned_in_rcm_order():
    """C planned in reverse Cuthill-McKee order: same blocks and values, and
    its products agree with the atom-order plan."""
    op = make_operator("C5", 0.01)
    A = Matrix.from_operator(op)
    C1, _ = A.spgemm(A, 0.0, row_order="atom")
    C2, _ = A.spgemm(A, 0.0, row_order="rcm")
    assert np.array_equal(C1.row_ptr, C2.row_ptr) and np.array_equal(C1.col_idx, C2.col_idx)
    assert torch.equal(C1.values(), C2.values())
    X = torch.randn(op.N, 9, dtype=torch.float64, device="cuda")
    assert torch.equal(C1.spmm(X), C2.spmm(X))
    compare(op, op, 0.0, C2, C2.values().cpu().numpy())


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_spgemm_device_plan_matches_host_plan(eps):
    """C laid out on the device (row orders auto and atom) and by the host
    planner (rcm, cluster): the same operator, so its info, values, forward,
    adjoint and block-sampled products agree bit for bit (each panel sums its
    blocks in the same order whatever the processing order)."""
    print("case spgemm device plan", eps, flush=True)
    op = make_operator("C5", 0.01)
    A = Matrix.from_operator(op)
    Cs = {o: A.spgemm(A, eps, row_order=o)[0] for o in ("auto", "atom", "rcm", "cluster")}
    ref = Cs["rcm"]
    rng = np.random.default_rng(4)
    X = torch.from_numpy(rng.standard_normal((op.N, 9))).cuda()
    G = torch.from_numpy(rng.standard_normal((op.N, 9))).cuda()
    want = (ref.spmm(X), ref.spmm(X, transpose=True), ref.sddmm(G, X))
    for o, C in Cs.items():
        assert C.info() == ref.info(), o
        assert np.array_equal(C.row_ptr, ref.row_ptr) and np.array_equal(C.col_idx, ref.col_idx), o
        assert torch.equal(C.values(), ref.values()), o
        got = (C.spmm(X), C.spmm(X, transpose=True), C.sddmm(G, X))
        for g, w in zip(got, want):
            assert torch.equal(g, w), o
    compare(op, op, eps, Cs["auto"], Cs["auto"].values().cpu().numpy())


def _wide_sparse(seed, n, per, bset, b=None):
    """``per`` random columns in each of ``n`` rows (ascending): rows of the
    product have few candidates spread over many atoms."""
    rng = np.random.default_rng(seed)
    if b is None:
        b = rng.choice(np.asarray(bset, np.int32), size=n).astype(np.int32)
    cols = [np.sort(rng.choice(n, per, replace=False)) for _ in range(n)]
    row_ptr = np.arange(0, n * per + 1, per, dtype=np.int64)
    ci = np.concatenate(cols).astype(np.int32)
    rows = np.repeat(np.arange(n), per)
    values = rng.uniform(-1.0, 1.0, size=int((b[rows].astype(np.int64) * b[ci]).sum()))
    return Operator("wide", b, row_ptr, ci, values, np.zeros(ci.shape[0]), {"seed": seed})


@pytest.mark.parametrize("eps", [0.0, 0.5])
def test_spgemm_few_candidates_over_many_atoms(eps):
    """6,000 atoms with two blocks per row: each row of C has at most four
    candidates spread over the whole atom range, the case where the symbolic
    stage orders candidates by sorting rather than by a bitmap scan."""
    print("case spgemm wide sparse", eps, flush=True)
    A = _wide_sparse(11, 6000, 2, (1, 4, 9))
    B = _wide_sparse(12, 6000, 2, (1, 4, 9), b=A.b)
    Am, Bm, C, st, vals = gpu_product(A, B, eps)
    compare(A, B, eps, C, vals)
    assert st["candidates"] <= 4 * 6000
