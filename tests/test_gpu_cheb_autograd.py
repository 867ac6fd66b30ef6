"""Chebyshev moments and the autograd composition on the GPU, against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, check, rounded
from metrics import rel_f
from workloads import make_config, random_pattern

pytestmark = pytest.mark.gpu

from paper_2609_04397_amd.matrix import Matrix, spmm

# moment error max_k |mu_k - mu_k^ref| / mu_0^ref (|mu_k| <= mu_0 on [-1, 1])
MOM_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 5e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("nrhs", [1, 5, 64])
def test_cheb_moments_small(prec, nrhs):
    op, vec = make_config("C4", scale=0.004, nrhs=nrhs)
    print("case cheb", prec, nrhs, op.N, flush=True)
    R = vec["R"]
    deg = 64
    ref = oracle.cheb_moments(op, rounded(R, prec), deg)
    A = Matrix.from_operator(op, prec=prec)
    mu = A.cheb_moments(dev(R, prec), deg)
    err = np.max(np.abs(mu - ref)) / np.max(np.abs(ref[0]))
    print("moment error", prec, nrhs, err)
    assert err <= MOM_TOL[prec]
    # bitwise reproducible
    assert np.array_equal(mu, A.cheb_moments(dev(R, prec), deg))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("degree", [0, 1, 2, 3, 63, 64])
def test_cheb_moments_doubled(prec, degree):
    """Moments from T_1 .. T_ceil(degree/2) and the Chebyshev product identity
    equal the plain recurrence's (symmetric operator)."""
    op, vec = make_config("C4", scale=0.004, nrhs=7)
    R = vec["R"]
    print("case doubled", prec, degree, op.N, flush=True)
    ref = oracle.cheb_moments(op, rounded(R, prec), degree)
    A = Matrix.from_operator(op, prec=prec)
    mu = A.cheb_moments(dev(R, prec), degree, doubled=True)
    err = np.max(np.abs(mu - ref)) / np.max(np.abs(ref[0]))
    print("doubled moment error", prec, degree, err)
    # the FP32/BF16x3 vectors enter twice in <T_k, T_k>: twice the bound
    assert err <= (1 if prec == "fp64" else 2) * MOM_TOL[prec]
    ws = torch.empty(A.cheb_workspace_bytes(7, degree), dtype=torch.uint8, device="cuda")
    assert np.array_equal(mu, A.cheb_moments(dev(R, prec), degree, workspace=ws, doubled=True))


def test_cheb_moments_mixed_blocks_and_workspace():
    op = random_pattern(14, 60, bset=(1, 4, 9, 13, 20), density=0.1, symmetric=True, empty_rows=2)
    from workloads.core import inf_norm_scale, scaled
    op = scaled(op, inf_norm_scale(op))
    R = np.random.default_rng(1).standard_normal((op.N, 7))
    ref = oracle.cheb_moments(op, R, 20)
    A = Matrix.from_operator(op)
    ws = torch.empty(A.cheb_workspace_bytes(7, 20), dtype=torch.uint8, device="cuda")
    for path in ("vec", "mfma"):
        A2 = Matrix.from_operator(op, path=path)
        mu = A2.cheb_moments(dev(R, "fp64"), 20, workspace=ws)
        assert np.max(np.abs(mu - ref)) / np.max(np.abs(ref[0])) <= 1e-12
    mu0 = A.cheb_moments(dev(R, "fp64"), 0)
    assert np.allclose(mu0, ref[:1], rtol=1e-14)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_cheb_step_matches_recurrence(prec):
    op, vec = make_config("C4", scale=0.004, nrhs=16)
    R = vec["R"]
    rng = np.random.default_rng(2)
    Tk = rounded(rng.uniform(-1, 1, R.shape), prec)
    Tp = rounded(rng.uniform(-1, 1, R.shape), prec)
    Rr = rounded(R, prec)
    ref_T = oracle.spmm(op, Tk, alpha=2.0, beta=-1.0, Y=Tp)
    ref_mu = (Rr * ref_T).sum(axis=0)
    A = Matrix.from_operator(op, prec=prec)
    ws = torch.empty(A.cheb_workspace_bytes(16, 0), dtype=torch.uint8, device="cuda")
    mu = torch.zeros(16, dtype=torch.float64, device="cuda")
    Tpd = dev(Tp, prec)
    A.cheb_step(dev(Tk, prec), Tpd, dev(R, prec), mu, ws)
    got = host(Tpd)
    check(got, ref_T, prec, oracle.abs_product(op, Tk) * 2 + np.abs(Tp) if prec == "fp64" else None)
    # moments of the stored (rounded) vector, accumulated in FP64
    ref_mu_stored = (Rr * got).sum(axis=0)
    assert np.max(np.abs(host(mu) - ref_mu_stored)) <= 1e-12 * np.abs(Rr * got).sum(axis=0).max()
    assert np.max(np.abs(host(mu) - ref_mu)) <= (1e-11 if prec == "fp64" else 1e-3) * np.abs(ref_mu).max()


def test_cheb_aliasing_is_rejected():
    """R aliasing the vector the step overwrites, or a workspace holding a
    vector, would silently change the moments: both are EINVAL, before any
    kernel runs (the buffers keep their contents)."""
    import ctypes
    from paper_2609_04397_amd import _lib
    op, vec = make_config("C4", scale=0.002, nrhs=4)
    A = Matrix.from_operator(op)
    lib = _lib.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    N = op.N
    Tk = torch.rand((N, 4), dtype=torch.float64, device="cuda")
    Tp = torch.rand((N, 4), dtype=torch.float64, device="cuda")
    mu = torch.zeros(4, dtype=torch.float64, device="cuda")
    need = A.cheb_workspace_bytes(4, 0)
    ws = torch.empty(need + 8 * N * 4, dtype=torch.uint8, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    before = Tp.clone()
    # R is Tprev
    assert lib.vbcsr_cheb_step(A._h, P(Tk), 4, P(Tp), 4, P(Tp), 4, 4, P(mu), P(ws), need,
                               s) == _lib.VBCSR_EINVAL
    # R lies inside the workspace
    Rin = ws[:8 * N * 4].view(torch.float64).view(N, 4)
    assert lib.vbcsr_cheb_step(A._h, P(Tk), 4, P(Tp), 4, P(Rin), 4, 4, P(mu), P(ws), need,
                               s) == _lib.VBCSR_EINVAL
    # mu_dev inside Tprev
    assert lib.vbcsr_cheb_step(A._h, P(Tk), 4, P(Tp), 4, P(Tk), 4, 4, P(Tp), P(ws), need,
                               s) == _lib.VBCSR_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(Tp, before)
    # the whole recurrence: R inside the caller's workspace
    need_m = A.cheb_workspace_bytes(4, 8)
    wsm = torch.empty(need_m, dtype=torch.uint8, device="cuda")
    Rws = wsm[:8 * N * 4].view(torch.float64).view(N, 4)
    mu_h = np.zeros((9, 4))
    for fn in (lib.vbcsr_cheb_moments, lib.vbcsr_cheb_moments_doubled):
        assert fn(A._h, P(Rws), 4, 4, 8, mu_h.ctypes.data, P(wsm), need_m, s) == _lib.VBCSR_EINVAL
    # a valid call still works after the rejected ones
    R = torch.from_numpy(vec["R"]).to("cuda")
    got = A.cheb_moments(R, 8, workspace=wsm)
    ref = oracle.cheb_moments(op, vec["R"], 8)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref[0]))


def test_autograd_gradcheck_fp64():
    op, vec = make_config("FD50", nrhs=3)
    A = Matrix.from_operator(op)
    V = torch.from_numpy(op.values.copy()).cuda().requires_grad_(True)
    X = torch.from_numpy(vec["X"][:, :3].copy()).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v, x: spmm(v, x, A), (V, X), eps=1e-3, atol=1e-9,
                                    rtol=1e-7, fast_mode=True)


def test_autograd_matches_oracle_and_finite_differences():
    op, vec = make_config("FD50")
    X, G = vec["X"], vec["G"]
    A = Matrix.from_operator(op)
    V = torch.from_numpy(op.values.copy()).cuda().requires_grad_(True)
    Xd = torch.from_numpy(X.copy()).cuda().requires_grad_(True)
    Gd = torch.from_numpy(G).cuda()
    L = (spmm(V, Xd, A) * Gd).sum()
    L.backward()
    dV, dX = host(V.grad), host(Xd.grad)
    dV_ref = oracle.sddmm(op, G, X)
    dX_ref = oracle.spmm_t(op, G)
    assert rel_f(dV, dV_ref) <= 1e-12 and rel_f(dX, dX_ref) <= 1e-12

    # central differences are exact for this bilinear loss (up to rounding)
    def loss(v, x):
        with torch.no_grad():
            return float((spmm(torch.from_numpy(v).cuda(), torch.from_numpy(x).cuda(), A) * Gd).sum())

    rng = np.random.default_rng(7)
    h = 1e-3
    for e in rng.choice(op.nnz, 300, replace=False):
        vp, vm = op.values.copy(), op.values.copy()
        vp[e] += h
        vm[e] -= h
        fd = (loss(vp, X) - loss(vm, X)) / (2 * h)
        assert abs(fd - dV[e]) <= 1e-9 * max(1.0, abs(dV[e]))
    for e in rng.choice(X.size, 150, replace=False):
        xp, xm = X.copy(), X.copy()
        xp.flat[e] += h
        xm.flat[e] -= h
        fd = (loss(op.values, xp) - loss(op.values, xm)) / (2 * h)
        assert abs(fd - dX.flat[e]) <= 1e-9 * max(1.0, abs(dX.flat[e]))


def test_autograd_fp32_form():
    op, vec = make_config("C5", scale=0.01)
    X, G = vec["X"], vec["G"]
    A = Matrix.from_operator(op, prec="fp32")
    V = torch.from_numpy(op.values.astype(np.float32)).cuda().requires_grad_(True)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda().requires_grad_(True)
    Y = spmm(V, Xd, A)
    (Y * torch.from_numpy(G.astype(np.float32)).cuda()).sum().backward()
    Vr = op.values.astype(np.float32).astype(np.float64)
    Xr = X.astype(np.float32).astype(np.float64)
    Gr = G.astype(np.float32).astype(np.float64)
    assert rel_f(host(Y), oracle.spmm(op, X, values=op.values)) <= 1e-5
    assert rel_f(host(Xd.grad), oracle.spmm_t(op, Gr, values=Vr)) <= 1e-5
    assert rel_f(host(V.grad), oracle.sddmm(op, Gr, Xr)) <= 1e-5


def test_autograd_values_change_between_calls():
    op, vec = make_config("FD50", nrhs=4)
    A = Matrix.from_operator(op)
    X = torch.from_numpy(vec["X"][:, :4].copy()).cuda()
    V1 = torch.from_numpy(op.values.copy()).cuda().requires_grad_(True)
    V2 = torch.from_numpy(op.values[::-1].copy()).cuda().requires_grad_(True)
    Xg = X.clone().requires_grad_(True)
    Y1 = spmm(V1, Xg, A)
    Y2 = spmm(V2, X, A)       # repacks A with V2
    Y1.sum().backward()       # must use V1 again for A^T
    ref = oracle.spmm_t(op, np.ones((op.N, 4)), values=op.values)
    assert rel_f(host(Xg.grad), ref) <= 1e-12
    assert rel_f(host(Y2), oracle.spmm(op, vec["X"][:, :4], values=op.values[::-1].copy())) <= 1e-12

