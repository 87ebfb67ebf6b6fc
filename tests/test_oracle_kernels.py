"""Pins of the oracle's whitening, spatial taps and range kernels
(eqs. (kernel), (COB), (approx), (expansion), Propositions 1 and 2)."""

import math

import numpy as np
import pytest

from oracle import mcsf as O
from synth import random_spd


# --- spatial kernel -----------------------------------------------------------

@pytest.mark.parametrize("sigma_s,window", [(2.0, 13), (5.0, 31), (10.0, 61), (4.0, 25)])
def test_window_sizes(sigma_s, window):
    # square window [-3 sigma_s, 3 sigma_s]^2 of the workloads: 13/31/61/25 taps
    assert len(O.spatial_taps(sigma_s)) == window


def test_taps_values():
    w = O.spatial_taps(2.0)
    R = 6
    assert w[R] == 1.0
    assert math.isclose(w[R + 2], math.exp(-0.5), rel_tol=1e-15)   # u = sigma
    assert math.isclose(w[0], math.exp(-4.5), rel_tol=1e-15)       # u = 3 sigma
    assert np.array_equal(w, w[::-1])
    assert O.window_radius(0) == 0 and np.array_equal(O.spatial_taps(0), [1.0])
    assert O.window_radius(0.5) == 2 and O.window_radius(1.0) == 3


# --- whitening (eq. (COB)) ----------------------------------------------------

def test_whiten_closed_form_block_matrix():
    # C = diag(100) (+) [[25, 12.5], [12.5, 25]]: eigenpairs by hand
    C = np.array([[100.0, 0, 0], [0, 25, 12.5], [0, 12.5, 25]])
    s2 = 1 / math.sqrt(2)
    expect = np.array([[0, s2, -s2] / np.float64(math.sqrt(12.5)),
                       [0, s2, s2] / np.float64(math.sqrt(37.5)),
                       [0.1, 0, 0]])
    assert np.allclose(O.whiten(C), expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,seed", [(2, 1), (3, 2), (6, 3), (8, 4)])
def test_whiten_inverse_covariance(d, seed):
    C = random_spd(d, -3, -1, seed)
    W = O.whiten(C)
    Ci = np.linalg.inv(C)
    assert np.max(np.abs(W.T @ W - Ci)) <= 1e-12 * np.max(np.abs(Ci))
    # rows are alpha_k q_k^T with ascending eigenvalues -> descending norms
    norms = np.linalg.norm(W, axis=1)
    assert np.all(np.diff(norms) <= 0)
    # each row is an eigenvector of C with eigenvalue 1/alpha_k^2
    for k in range(d):
        q = W[k] / norms[k]
        assert np.allclose(C @ q, q / norms[k] ** 2, rtol=1e-10, atol=0)
        first = np.argmax(np.abs(q) > 1e-6 * np.max(np.abs(q)))
        assert q[first] > 0


def test_whiten_diagonal():
    C = np.diag([0.01, 4.0, 0.25])
    assert np.array_equal(O.whiten(C), np.diag([10.0, 0.5, 2.0]))
    # isotropic C: Q = I (the paper's setting for all its experiments)
    assert np.array_equal(O.whiten(np.eye(3) * 0.0064), np.eye(3) / 0.08)


def test_whiten_modes_closed_form_2x2():
    # C = [[4, 2], [2, 5]] = L L^T with L = [[2, 0], [1, 2]]
    C = np.array([[4.0, 2.0], [2.0, 5.0]])
    W = O.whiten(C, O.WHITEN_CHOL)
    assert np.allclose(W, [[0.5, 0.0], [-0.25, 0.5]], rtol=0, atol=1e-15)
    # C^{1/2} = (C + sqrt(det C) I) / sqrt(tr C + 2 sqrt(det C)) = [[8, 2], [2, 9]] / sqrt(17)
    W = O.whiten(C, O.WHITEN_SYM)
    expect = math.sqrt(17.0) / 68.0 * np.array([[9.0, -2.0], [-2.0, 8.0]])
    assert np.allclose(W, expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,seed", [(2, 5), (3, 6), (6, 7), (8, 8)])
def test_whiten_modes_invariants(d, seed):
    C = random_spd(d, -3, -1, seed)
    Ci = np.linalg.inv(C)
    Wc = O.whiten(C, O.WHITEN_CHOL)
    Ws = O.whiten(C, O.WHITEN_SYM)
    for W in (Wc, Ws):
        assert np.max(np.abs(W.T @ W - Ci)) <= 1e-11 * np.max(np.abs(Ci))
    # Cholesky: lower triangular with a positive diagonal, and W^{-1} W^{-T} = C
    assert np.array_equal(Wc, np.tril(Wc)) and np.all(np.diag(Wc) > 0)
    Li = np.linalg.inv(Wc)
    assert np.max(np.abs(Li @ Li.T - C)) <= 1e-11 * np.max(np.abs(C))
    # symmetric root: symmetric, positive definite, squares to C^{-1}
    assert np.max(np.abs(Ws - Ws.T)) <= 1e-12 * np.max(np.abs(Ws))
    assert np.min(np.linalg.eigvalsh(Ws)) > 0
    assert np.max(np.abs(Ws @ Ws - Ci)) <= 1e-11 * np.max(np.abs(Ci))


def test_whiten_modes_agree_on_diagonal_covariance():
    C = np.diag([0.01, 4.0, 0.25])
    for mode in (O.WHITEN_EIG, O.WHITEN_CHOL, O.WHITEN_SYM):
        assert np.array_equal(O.whiten(C, mode), np.diag([10.0, 0.5, 2.0]))


def test_whiten_rejects_bad_covariance():
    with pytest.raises(ValueError):
        O.whiten(np.array([[1.0, 0.5], [0.4, 1.0]]))
    with pytest.raises(ValueError):
        O.whiten(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(ValueError):
        O.whiten(np.zeros((2, 2)))


# --- range kernels -------------------------------------------------------------

def test_gauss_kernel_diagonal_closed_form():
    C = np.diag([0.04, 1.0, 9.0])
    D = np.array([[0.2, -1.0, 3.0], [0.0, 0.0, 0.0]])
    expect = np.exp(-0.5 * (0.2 ** 2 / 0.04 + 1.0 + 1.0))
    assert math.isclose(O.psi_gauss(D, C)[0], expect, rel_tol=1e-14)
    assert O.psi_gauss(D, C)[1] == 1.0


def test_raised_cosine_limit_proposition1():
    # cos(z/sqrt(N))^N -> exp(-z^2/2), with error ~ -exp(-z^2/2) z^4 / (12 N)
    z = np.linspace(-3, 3, 13)
    g = np.exp(-z * z / 2)
    for N in (1000, 10000, 100000):
        rc = np.cos(z / math.sqrt(N)) ** N
        err = rc - g
        pred = -g * z ** 4 / (12 * N)
        big = np.abs(z) > 0.5
        assert np.allclose(err[big] / pred[big], 1.0, atol=30.0 / N ** 0.5 + 2e-3)
    assert np.max(np.abs(np.cos(z / math.sqrt(1e6)) ** 1e6 - g)) < 1e-5


@pytest.mark.parametrize("d,N", [(1, 1), (1, 7), (2, 5), (3, 4), (2, 10)])
def test_expansion_identity_proposition2(d, N):
    # eq. (expansion): prod_k cos(z_k/sqrt N)^N equals the binomially weighted
    # sum over all Y of cos(<Y, z>/sqrt N) -- checked against the closed form.
    rng = np.random.default_rng(d * 100 + N)
    C = random_spd(d, -1, 0, d + N) if d > 1 else np.array([[0.3]])
    W = O.whiten(C)
    w, wt = O.full_expansion_terms(W, N)
    assert math.isclose(wt.sum(), 1.0, rel_tol=1e-14)
    D = rng.normal(size=(50, d))
    closed = O.psi_raised_cosine(D, W, N)
    enum = O.psi_sampled(D, w, wt)
    assert np.max(np.abs(closed - enum)) < 1e-13


def test_sampled_kernel_unbiased_with_known_variance():
    # E[cos<w,D>] = psi_N(D);  Var = (1 + psi_N(2D))/2 - psi_N(D)^2
    C = np.diag([0.01, 0.02, 0.015])
    W = O.whiten(C)
    N = 12
    D = np.array([[0.05, -0.1, 0.08], [0.2, 0.1, -0.05], [0.01, 0.0, 0.0]])
    _, w = O.sample_terms(C, N, 40000, 77)
    vals = np.cos(D @ w.T)                          # (3, K)
    psi = O.psi_raised_cosine(D, W, N)
    var = (1 + O.psi_raised_cosine(2 * D, W, N)) / 2 - psi ** 2
    se = np.sqrt(var / vals.shape[1])
    assert np.all(np.abs(vals.mean(axis=1) - psi) < 5 * se + 1e-15)
    assert np.all(np.abs(vals.var(axis=1) - var) < 0.05 * var + 1e-6)
    assert np.allclose(O.psi_sampled(np.zeros((1, 3)), w), 1.0)
