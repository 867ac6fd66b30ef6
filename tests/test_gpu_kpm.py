"""KPM density of states on the GPU (Clenshaw per point) against the oracle
(direct cos(k arccos x) sums), and the whole pipeline from an operator's
Chebyshev moments to its gap."""
import numpy as np
import pytest
import torch

from oracle import kpm as okpm
from test_oracle_kpm import moments_of_spectrum
from workloads.core import Operator

pytestmark = pytest.mark.gpu

from paper_2609_04397_amd import kpm
from paper_2609_04397_amd.matrix import Matrix


def d(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def check_dos(mu, x, damping, got):
    ref = okpm.dos(mu, x, damping=damping)
    g = okpm.jackson(len(mu)) if damping == "jackson" else np.ones(len(mu))
    scale = (np.abs(g * mu).sum() * 2) / (np.pi * np.sqrt(1 - x * x))
    # Clenshaw/series rounding, plus the conditioning of sqrt(1 - x^2) near
    # |x| = 1 (the two sides may round x*x differently or fuse it)
    tol = 64 * len(mu) * 2.0 ** -53 * scale + 4 * 2.0 ** -53 * np.abs(ref) / (1 - x * x) + 1e-300
    err = np.abs(got - ref)
    assert np.all(err <= tol), "max err/tol %.3g" % (err / tol).max()


@pytest.mark.parametrize("M", [1, 2, 3, 17, 256, 1000])
@pytest.mark.parametrize("damping", ["jackson", "none"])
def test_dos_matches_oracle(M, damping):
    print("case kpm dos", M, damping, flush=True)
    rng = np.random.default_rng(M)
    mu = moments_of_spectrum(rng.uniform(-0.95, 0.95, 50), M)
    x = np.concatenate([np.linspace(-0.999999, 0.999999, 1001), rng.uniform(-1, 1, 77) * 0.99])
    got = kpm.dos(d(mu), d(x), damping).cpu().numpy()
    check_dos(mu, x, damping, got)
    # the same with a caller workspace
    work = torch.empty(M, dtype=torch.float64, device="cuda")
    got2 = kpm.dos(d(mu), d(x), damping, work=work).cpu().numpy()
    assert np.array_equal(got, got2)


def test_dos_paper_scale_moment_count_sampled():
    """147,456 moments (the paper's count) on 300,000 points; the oracle
    checks 64 sampled points."""
    M = 147456
    rng = np.random.default_rng(5)
    mu = moments_of_spectrum(rng.uniform(-0.9, 0.9, 64), M)
    x = np.linspace(-0.99, 0.99, 300000)
    got = kpm.dos(d(mu), d(x)).cpu().numpy()
    idx = np.unique(np.concatenate([[0, x.size - 1], rng.choice(x.size, 62, replace=False)]))
    check_dos(mu, x[idx], "jackson", got[idx])
    assert np.isfinite(got).all()


def test_dos_empty_points_and_edges():
    mu = d(moments_of_spectrum([0.3], 8))
    assert kpm.dos(mu, d(np.zeros(0))).numel() == 0
    r = kpm.dos(mu, d(np.array([1.0, -1.0, 0.5]))).cpu().numpy()
    assert not np.isfinite(r[0]) and not np.isfinite(r[1]) and np.isfinite(r[2])


def test_pipeline_gap_of_block_operator():
    """A block-diagonal operator whose blocks have eigenvalues in two bands
    separated by a known gap: GPU moments -> GPU density -> gap, against the
    oracle's density and gap from the same moments, and the true gap."""
    rng = np.random.default_rng(9)
    b = np.array([9, 13, 4, 9, 13, 1, 4] * 12, dtype=np.int32)
    vals, lam_all = [], []
    for bi in b:
        lam = np.where(rng.random(bi) < 0.5, rng.uniform(-0.8, -0.3, bi), rng.uniform(0.2, 0.7, bi))
        Q, _ = np.linalg.qr(rng.standard_normal((bi, bi)))
        vals.append((Q @ np.diag(lam) @ Q.T).ravel())
        lam_all.append(lam)
    n = b.size
    op = Operator("bands", b, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                  np.concatenate(vals), np.zeros(n))
    lam_all = np.concatenate(lam_all)
    N, R, M = op.N, 16, 256
    A = Matrix.from_operator(op)
    Rv = torch.from_numpy(rng.standard_normal((N, R))).cuda()
    mu_cols = A.cheb_moments(Rv, M - 1)                 # (M, R)
    mu = mu_cols.sum(axis=1) / (N * R)
    x = np.linspace(-0.99, 0.99, 4001)
    rho = kpm.dos(d(mu), d(x)).cpu().numpy()
    check_dos(mu, x, "jackson", rho)
    thr = kpm.threshold(M, N, 0.1)
    g = kpm.gap(x, rho, thr)
    ref_rho = okpm.dos(mu, x)
    go = okpm.gap(x, ref_rho, thr)
    assert g is not None and go is not None
    for a, b_ in zip(g, go):   # a different edge is valid only at a near-tie
        if a != b_:
            for v in (a, b_):
                i = int(np.argmin(np.abs(x - v)))
                assert abs(ref_rho[i] - thr) <= 1e-9 * thr
    top_lo, bot_hi = lam_all[lam_all < 0].max(), lam_all[lam_all > 0].min()
    sigma = np.pi / M
    assert abs(g[0] - top_lo) < 6 * sigma and abs(g[1] - bot_hi) < 6 * sigma


def test_pipeline_with_doubled_moments():
    """Moment doubling (half the products) feeds the same density: the
    doubled and the plain moments give densities within rounding."""
    rng = np.random.default_rng(12)
    b = np.array([9, 13, 4] * 20, dtype=np.int32)
    vals, n = [], b.size
    for bi in b:
        lam = rng.uniform(-0.9, 0.9, bi)
        Q, _ = np.linalg.qr(rng.standard_normal((bi, bi)))
        vals.append((Q @ np.diag(lam) @ Q.T).ravel())
    op = Operator("diag-blocks", b, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                  np.concatenate(vals), np.zeros(n))
    A = Matrix.from_operator(op)
    R = torch.from_numpy(rng.standard_normal((op.N, 8))).cuda()
    M = 128
    mu_p = A.cheb_moments(R, M - 1).sum(axis=1) / (op.N * 8)
    mu_d = A.cheb_moments(R, M - 1, doubled=True).sum(axis=1) / (op.N * 8)
    assert np.max(np.abs(mu_p - mu_d)) <= 1e-12
    x = np.linspace(-0.99, 0.99, 2001)
    rp = kpm.dos(d(mu_p), d(x)).cpu().numpy()
    rd = kpm.dos(d(mu_d), d(x)).cpu().numpy()
    assert np.max(np.abs(rp - rd)) <= 1e-10 * np.max(np.abs(rp))
    check_dos(mu_d, x, "jackson", rd)
