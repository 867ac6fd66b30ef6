"""Pins of the oracle's KPM reconstruction (damping kernel, density of
states, gap) against facts fixed independently of it: hand-derived Jackson
factors, Gauss-Chebyshev quadrature (exact for the polynomial part), NumPy's
Chebyshev series evaluation, positivity of the Jackson kernel, the known
width of a damped delta, and a spectrum with a known gap."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npc

from oracle import kpm


def moments_of_spectrum(lam, M):
    """mu_k = mean_i T_k(lam_i) by the three-term recurrence (test side)."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.empty(M)
    t0, t1 = np.ones_like(lam), lam.copy()
    mu[0] = t0.mean()
    if M > 1:
        mu[1] = t1.mean()
    for k in range(2, M):
        t0, t1 = t1, 2 * lam * t1 - t0
        mu[k] = t1.mean()
    return mu


def test_jackson_hand_values():
    assert np.allclose(kpm.jackson(1), [1.0], rtol=0, atol=1e-15)
    assert np.allclose(kpm.jackson(2), [1.0, 0.5], rtol=0, atol=1e-15)
    assert np.allclose(kpm.jackson(3), [1.0, np.sqrt(0.5), 0.25], rtol=0, atol=1e-15)
    g = kpm.jackson(1000)
    assert g[0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diff(g) < 0) and g[-1] > 0


def test_undamped_series_matches_numpy_chebval():
    rng = np.random.default_rng(0)
    mu = rng.standard_normal(40) / np.arange(1, 41)
    x = np.linspace(-0.99, 0.99, 301)
    a = 2 * mu
    a[0] = mu[0]
    ref = npc.chebval(x, a) / (np.pi * np.sqrt(1 - x * x))
    assert np.allclose(kpm.dos(mu, x, damping="none"), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("M", [16, 200, 1024])
def test_quadrature_integral_is_mu0(M):
    """Gauss-Chebyshev with P > M nodes integrates rho exactly: g_0 mu_0."""
    rng = np.random.default_rng(M)
    mu = moments_of_spectrum(rng.uniform(-0.9, 0.9, 300), M)
    P = 2 * M + 7
    xj = np.cos(np.pi * (np.arange(P) + 0.5) / P)
    integral = (np.pi / P) * (kpm.dos(mu, xj) * np.sqrt(1 - xj * xj)).sum()
    assert integral == pytest.approx(mu[0], rel=1e-12)


def test_jackson_density_is_positive_and_peaks_at_eigenvalues():
    lam = np.array([-0.9, -0.6, -0.2, 0.1, 0.45, 0.8])
    M = 400
    mu = moments_of_spectrum(lam, M)
    x = np.linspace(-0.999, 0.999, 8001)
    rho = kpm.dos(mu, x)
    assert rho.min() >= -1e-10 * rho.max()
    rho_none = kpm.dos(mu, x, damping="none")
    assert rho_none.min() < -1e-3 * rho_none.max()      # Gibbs oscillations without damping
    for l in lam:
        w = np.abs(x - l) < 0.02
        assert abs(x[w][np.argmax(rho[w])] - l) <= 2 * (x[1] - x[0]) + 1e-3


@pytest.mark.parametrize("x0", [0.0, 0.5, -0.7])
def test_damped_delta_width(x0):
    """A single state broadens to a peak of standard deviation close to
    (pi / M) sqrt(1 - x0^2) (the Jackson resolution)."""
    M = 512
    mu = moments_of_spectrum([x0], M)
    x = np.linspace(-0.9999, 0.9999, 40001)
    rho = kpm.dos(mu, x)
    w = rho / np.trapezoid(rho, x)
    mean = np.trapezoid(w * x, x)
    sd = np.sqrt(np.trapezoid(w * (x - mean) ** 2, x))
    assert mean == pytest.approx(x0, abs=2e-3)
    assert sd == pytest.approx(np.pi / M * np.sqrt(1 - x0 * x0), rel=0.15)


def test_gap_of_known_spectrum():
    lam = np.concatenate([np.linspace(-0.8, -0.3, 1000), np.linspace(0.2, 0.7, 1000)])
    M = 1024
    mu = moments_of_spectrum(lam, M)
    x = np.linspace(-0.99, 0.99, 20001)
    rho = kpm.dos(mu, x)
    thr = 0.1 * kpm.single_state_peak(M, lam.size)
    lo, hi = kpm.gap(x, rho, thr)
    sigma = np.pi / M
    assert abs(lo - (-0.3)) < 4 * sigma and abs(hi - 0.2) < 4 * sigma
    assert kpm.gap(x, np.ones_like(x), 0.5) is None


@pytest.mark.parametrize("M", [256, 2048])
def test_single_state_peak_height(M):
    """One state of weight 1/N at x = 0: the damped density peaks at
    1 / (N sigma sqrt(2 pi)) with sigma = pi / M (Gaussian limit)."""
    N = 1000
    mu = moments_of_spectrum([0.0], M) / N
    peak = kpm.dos(mu, np.array([0.0]))[0]
    assert peak == pytest.approx(kpm.single_state_peak(M, N), rel=0.05)
