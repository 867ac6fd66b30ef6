"""Kernel polynomial method after the moments -- TEST INFRASTRUCTURE.

Plain numpy, FP64, written from the definitions (section 5 uses the KPM with
a damping kernel, reconstructs the density of states and reads a gap off the
low-DOS interval with a threshold tied to the kernel's resolution):

* :func:`jackson`  Jackson damping factors
  ``g_k = [(M-k+1) cos(pi k/(M+1)) + sin(pi k/(M+1)) cot(pi/(M+1))] / (M+1)``
  for ``M`` moments, ``k = 0..M-1``;
* :func:`dos`      ``rho(x) = [g_0 mu_0 + 2 sum_{k>=1} g_k mu_k T_k(x)] / (pi sqrt(1-x^2))``
  with ``T_k(x) = cos(k arccos x)`` evaluated directly (no recurrence);
* :func:`single_state_peak` peak of one state of weight 1/N broadened by a
  Gaussian of the kernel width ``sigma = pi / M``: ``1 / (N sigma sqrt(2 pi))``;
* :func:`gap`      the widest run of points with ``rho < threshold`` that has
  points at or above the threshold on both sides; returns those two bounding
  points' abscissae.
"""
from __future__ import annotations

import numpy as np


def jackson(M: int) -> np.ndarray:
    """Jackson damping factors for M moments (k = 0 .. M-1)."""
    k = np.arange(M, dtype=np.float64)
    q = np.pi / (M + 1)
    return ((M - k + 1) * np.cos(q * k) + np.sin(q * k) / np.tan(q)) / (M + 1)


def dos(mu, x, damping: str = "jackson", chunk: int = 256) -> np.ndarray:
    """Density of states at the points x (|x| < 1) from moments mu[0..M-1]."""
    mu = np.asarray(mu, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    M = mu.shape[0]
    g = jackson(M) if damping == "jackson" else np.ones(M)
    c = g * mu
    theta = np.arccos(x)
    acc = np.full(x.shape, c[0])
    for k0 in range(1, M, chunk):
        ks = np.arange(k0, min(M, k0 + chunk), dtype=np.float64)
        acc += 2.0 * (c[k0:k0 + ks.shape[0]][:, None] * np.cos(ks[:, None] * theta[None, :])).sum(0)
    return acc / (np.pi * np.sqrt(1.0 - x * x))


def single_state_peak(M: int, N: int) -> float:
    sigma = np.pi / M
    return 1.0 / (N * sigma * np.sqrt(2.0 * np.pi))


def gap(x, rho, threshold: float):
    """(x_lo, x_hi) bounding the widest below-threshold run, or None."""
    above = np.asarray(rho) >= threshold
    idx = np.nonzero(above)[0]
    best = None
    for a, b in zip(idx[:-1], idx[1:]):
        if b - a > 1 and (best is None or x[b] - x[a] > best[1] - best[0]):
            best = (float(x[a]), float(x[b]))
    return best
