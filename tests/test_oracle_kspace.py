"""Pins of the oracle's reciprocal-space sampling (equation 4, both phase
conventions) and its complex products: a dense assembly written in the
test, the closed-form bands of a dimerised chain, Hermiticity, periodicity
in k, the unitary relation between the two conventions, and the adjoint
identity."""
import numpy as np
import pytest

from oracle.kspace import KOperator
from workloads.periodic import ImageOperator, random_images


def dense_k(Z, k, convention="R"):
    off = np.concatenate([[0], np.cumsum(Z.b.astype(np.int64))])
    D = np.zeros((Z.N, Z.N), dtype=np.complex128)
    base = np.concatenate([[0], np.cumsum(Z.block_sizes)])
    rows = Z.block_rows
    for t in range(Z.nnzb):
        i, j = int(rows[t]), int(Z.col_idx[t])
        d = Z.shifts[Z.image[t]].astype(float)
        if convention == "R+tau":
            d = d + Z.tau[j] - Z.tau[i]
        ph = np.exp(-2j * np.pi * float(np.dot(k, d)))
        blk = Z.values[base[t]:base[t + 1]].reshape(Z.b[i], Z.b[j])
        D[off[i]:off[i + 1], off[j]:off[j + 1]] += ph * blk
    return D


@pytest.mark.parametrize("conv", ["R", "R+tau"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_products_match_dense_assembly(conv, seed):
    Z = random_images(seed, 14, hermitian=seed != 2, empty_rows=1)
    rng = np.random.default_rng(seed)
    k = rng.uniform(-1, 1, 3)
    X = rng.standard_normal((Z.N, 3)) + 1j * rng.standard_normal((Z.N, 3))
    D = dense_k(Z, k, conv)
    K = KOperator(Z, k, conv)
    assert np.allclose(K.spmm(X), D @ X, rtol=0, atol=1e-12)
    assert np.allclose(K.spmm_h(X), D.conj().T @ X, rtol=0, atol=1e-12)


def test_dimerised_chain_bands():
    """Two orbitals per cell, intra-cell hopping v, inter-cell hopping w to
    the next cell: O(k) = [[0, v + w e^{2 pi i k}], [c.c., 0]], eigenvalues
    +-|v + w e^{-2 pi i k}|."""
    v, w = 0.7, -0.4
    b = np.array([2], np.int32)
    H0 = np.array([[0.0, v], [v, 0.0]])
    H1 = np.array([[0.0, 0.0], [w, 0.0]])     # couples to the cell at +1
    Z = ImageOperator("chain", b, np.array([0, 3], np.int64), np.zeros(3, np.int32),
                      np.array([0, 1, 2], np.int32),
                      np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0]], np.int32),
                      np.concatenate([H0.ravel(), H1.ravel(), H1.T.ravel()]),
                      np.zeros((1, 3)))
    for kx in np.linspace(-0.5, 0.5, 11):
        K = KOperator(Z, [kx, 0.3, -0.2])
        M = K.spmm(np.eye(2))
        ev = np.sort(np.linalg.eigvalsh(M))
        e = abs(v + w * np.exp(-2j * np.pi * kx))
        assert np.allclose(ev, [-e, e], atol=1e-14)


def test_hermitian_and_periodic():
    Z = random_images(7, 12, hermitian=True)
    rng = np.random.default_rng(0)
    k = rng.uniform(-1, 1, 3)
    M = KOperator(Z, k).spmm(np.eye(Z.N))
    assert np.allclose(M, M.conj().T, atol=1e-14)
    G = np.array([1, -2, 3])
    assert np.allclose(KOperator(Z, k + G).spmm(np.eye(Z.N)), M, atol=1e-12)
    # R+tau: O(k + G) = D O(k) D^*, D = diag(exp(2 pi i G . tau_i)) per orbital
    Mt = KOperator(Z, k, "R+tau").spmm(np.eye(Z.N))
    MtG = KOperator(Z, k + G, "R+tau").spmm(np.eye(Z.N))
    dvec = np.repeat(np.exp(2j * np.pi * (Z.tau @ G)), Z.b)
    assert np.allclose(MtG, dvec[:, None] * Mt * dvec.conj()[None, :], atol=1e-12)
    # conventions: O_tau(k) = U O_R(k) U^*, U = diag(exp(2 pi i k . tau_i))
    u = np.repeat(np.exp(2j * np.pi * (Z.tau @ k)), Z.b)
    assert np.allclose(Mt, u[:, None] * M * u.conj()[None, :], atol=1e-12)
    assert np.allclose(np.linalg.eigvalsh(Mt), np.linalg.eigvalsh(M), atol=1e-12)


def test_gamma_point_is_sum_of_images_and_adjoint_identity():
    Z = random_images(11, 16, hermitian=False)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((Z.N, 2))
    K0 = KOperator(Z, [0, 0, 0])
    assert np.abs(K0.spmm(X).imag).max() == 0.0
    assert np.allclose(K0.spmm(X).real, dense_k(Z, [0, 0, 0]).real @ X, atol=1e-12)
    k = rng.uniform(-1, 1, 3)
    K = KOperator(Z, k)
    x = rng.standard_normal((Z.N, 1)) + 1j * rng.standard_normal((Z.N, 1))
    y = rng.standard_normal((Z.N, 1)) + 1j * rng.standard_normal((Z.N, 1))
    lhs = np.vdot(y, K.spmm(x))
    rhs = np.vdot(K.spmm_h(y), x)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
