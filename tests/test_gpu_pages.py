"""Values held in the operator's forward-page layout (vbcsr_page_size,
vbcsr_get_pages, vbcsr_use_pages, vbcsr_refresh_transposed,
vbcsr_sddmm_pages) and the page-layout autograd function.

Every product reads the same values at the same positions whichever buffer
holds them, so the page-layout results are compared bit for bit with the
graph-order ones (which the parity tests compare with the oracle); the
gradient is also checked by gradcheck and against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, check, rounded
from workloads import random_pattern

pytestmark = pytest.mark.gpu

from paper_2609_04397_amd import spmm, spmm_pages
from paper_2609_04397_amd._lib import VbcsrError
from paper_2609_04397_amd.matrix import Matrix

PATTERNS = {
    "mixed": dict(seed=1, n=40, bset=(1, 4, 9, 13), density=0.2, empty_rows=3, unsorted=True),
    "wide": dict(seed=2, n=24, bset=(2, 5, 16, 17, 20, 33), density=0.3, empty_rows=1),
    "big": dict(seed=3, n=10, bset=(64, 31, 48), density=0.5),
}


@pytest.fixture(scope="module", params=sorted(PATTERNS))
def pattern(request):
    return request.param, random_pattern(**PATTERNS[request.param])


def page_index(op, prec):
    """Page position of every graph-order value: pack 1 .. nnz (exact in
    either precision for these sizes) and read where each landed."""
    A = Matrix.from_operator(op, prec=prec, values=np.arange(1, op.nnz + 1, dtype=np.float64))
    P = A.get_pages().double().cpu().numpy()
    idx = np.full(op.nnz, -1, np.int64)
    nz = np.nonzero(P)[0]
    idx[P[nz].astype(np.int64) - 1] = nz
    assert np.all(idx >= 0) and len(nz) == op.nnz
    return torch.from_numpy(idx).cuda()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pages_drive_every_product(pattern, prec):
    name, op = pattern
    print("case pages", name, prec, flush=True)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = Matrix.from_operator(op, prec=prec)
    B = Matrix.from_operator(op, prec=prec)
    P = A.get_pages()
    assert P.numel() == A.page_size and P.dtype == dt
    # values at their positions, zeros elsewhere
    V = A.values()
    assert int((P != 0).sum()) == int((V != 0).sum())
    rng = np.random.default_rng(3)
    X = dev(rng.standard_normal((op.N, 13)), prec)
    B.use_pages(P.clone())
    assert torch.equal(B.spmm(X), A.spmm(X))
    assert torch.equal(B.values(), V)
    with pytest.raises(VbcsrError):
        B.spmm(X, transpose=True)   # transposed pages stale until refreshed
    B.refresh_transposed()
    assert torch.equal(B.spmm(X, transpose=True), A.spmm(X, transpose=True))
    # other values, supplied in the page layout only
    V2 = rng.standard_normal(op.nnz)
    A2 = Matrix.from_operator(op, prec=prec, values=V2)
    P2 = A2.get_pages()
    B.use_pages(P2)
    B.refresh_transposed()
    for T in (False, True):
        assert torch.equal(B.spmm(X, transpose=T), A2.spmm(X, transpose=T))
    # the oracle with the second set of values (rounded to the handle's type)
    op2 = type(op)(op.name, op.b, op.row_ptr, op.col_idx, rounded(V2, prec), op.dist)
    ref = oracle.spmm(op2, rounded(X.double().cpu().numpy(), prec))
    check(host(B.spmm(X)), ref, prec, None, "pages %s %s" % (name, prec))
    # back to the handle's own pages: the first values again
    B.use_pages(None)
    B.refresh_transposed()
    for T in (False, True):
        assert torch.equal(B.spmm(X, transpose=T), A.spmm(X, transpose=T))
    # set_values leaves the page buffer and rewrites both page sets
    B.use_pages(P2)
    B.set_values(torch.from_numpy(V2).to("cuda", dt))
    for T in (False, True):
        assert torch.equal(B.spmm(X, transpose=T), A2.spmm(X, transpose=T))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nrhs", [1, 7, 32, 64, 100])
def test_sddmm_pages_matches_graph_order(pattern, prec, nrhs):
    name, op = pattern
    print("case sddmm pages", name, prec, nrhs, flush=True)
    A = Matrix.from_operator(op, prec=prec)
    rng = np.random.default_rng(nrhs)
    G = dev(rng.standard_normal((op.N, nrhs)), prec)
    X = dev(rng.standard_normal((op.N, nrhs)), prec)
    out = torch.full((A.page_size,), float("nan"), dtype=G.dtype, device="cuda")
    dP = A.sddmm_pages(G, X, out)
    assert not torch.isnan(dP).any()            # gaps and slack written (zero)
    dA = A.sddmm(G, X)
    assert int((dP != 0).sum()) == int((dA != 0).sum())
    C = Matrix.from_operator(op, prec=prec)
    C.use_pages(dP)
    assert torch.equal(C.values(), dA)          # same numbers, page positions


def test_spmm_pages_gradcheck():
    op = random_pattern(seed=7, n=9, bset=(1, 3, 5), density=0.35, empty_rows=1, unsorted=True)
    A = Matrix.from_operator(op)
    idx = page_index(op, "fp64")
    rng = np.random.default_rng(0)
    v = torch.from_numpy(rng.standard_normal(op.nnz)).cuda().requires_grad_(True)
    X = torch.from_numpy(rng.standard_normal((op.N, 3))).cuda().requires_grad_(True)

    def f(v, X):
        pages = torch.zeros(A.page_size, dtype=torch.float64, device="cuda").index_put((idx,), v)
        return spmm_pages(pages, X, A)

    assert torch.autograd.gradcheck(f, (v, X), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spmm_pages_gradients_match_graph_order(pattern, prec):
    name, op = pattern
    print("case pages grad", name, prec, flush=True)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = Matrix.from_operator(op, prec=prec)
    idx = page_index(op, prec)
    rng = np.random.default_rng(5)
    vals = torch.from_numpy(rng.standard_normal(op.nnz)).to("cuda", dt)
    Xn = rng.standard_normal((op.N, 9))
    Gn = rng.standard_normal((op.N, 9))
    # graph-order autograd
    v1 = vals.clone().requires_grad_(True)
    X1 = torch.from_numpy(Xn).to("cuda", dt).requires_grad_(True)
    Y1 = spmm(v1, X1, A)
    (Y1 * torch.from_numpy(Gn).to("cuda", dt)).sum().backward()
    # page-layout autograd on another handle over the same graph
    B = Matrix.from_operator(op, prec=prec)
    pages = torch.zeros(B.page_size, dtype=dt, device="cuda")
    pages[idx] = vals
    pages.requires_grad_(True)
    X2 = torch.from_numpy(Xn).to("cuda", dt).requires_grad_(True)
    Y2 = spmm_pages(pages, X2, B)
    (Y2 * torch.from_numpy(Gn).to("cuda", dt)).sum().backward()
    assert torch.equal(Y1, Y2)
    assert torch.equal(X1.grad, X2.grad)
    assert torch.equal(pages.grad[idx], v1.grad)
    mask = torch.ones(B.page_size, dtype=torch.bool, device="cuda")
    mask[idx] = False
    assert not pages.grad[mask].any()           # no gradient in the gaps
    # and the gradient is the oracle's block-sampled product
    Gr, Xr = rounded(Gn, prec), rounded(Xn, prec)
    check(host(pages.grad[idx]), oracle.sddmm(op, Gr, Xr), prec,
          oracle.sddmm(op, np.abs(Gr), np.abs(Xr)) if prec == "fp64" else None,
          "pages grad %s %s" % (name, prec))


def test_bf16x3_has_no_page_layout():
    op = random_pattern(seed=8, n=6, bset=(2, 3), density=0.5)
    A = Matrix.from_operator(op, prec="bf16x3")
    with pytest.raises(VbcsrError):
        A.page_size


def test_block_product_needs_current_transposed_pages():
    """The block product reads A's transposed pages: refused while they are
    stale, and with page-layout values it equals the product of a handle
    built from the same values."""
    op = random_pattern(seed=9, n=20, bset=(2, 5, 9), density=0.3)
    A = Matrix.from_operator(op)
    P = A.get_pages()
    B = Matrix.from_operator(op, values=np.zeros(op.nnz))
    B.use_pages(P)
    with pytest.raises(VbcsrError):
        B.spgemm(B, 0.0)
    B.refresh_transposed()
    C1, _ = A.spgemm(A, 0.0)
    C2, _ = B.spgemm(B, 0.0)
    assert np.array_equal(C1.row_ptr, C2.row_ptr) and np.array_equal(C1.col_idx, C2.col_idx)
    assert torch.equal(C1.values(), C2.values())
