"""Pins of the oracle's generator and Monte Carlo draws (Proposition 2)."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x32_10
from oracle import mcsf as O


def test_philox_known_answer_vectors(kat_vectors):
    for ctr, key, expected in kat_vectors:
        out = philox4x32_10([ctr], key)[0]
        assert [int(x) for x in out] == expected


def test_philox_vectorised_matches_rowwise():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(17, 4), dtype=np.uint64).astype(np.uint32)
    key = (0x12345678, 0x9ABCDEF0)
    batch = philox4x32_10(ctr, key)
    for i in range(17):
        assert np.array_equal(batch[i], philox4x32_10([ctr[i]], key)[0])


def test_binomial_bit_count_matches_python_popcount():
    # X for N = 70 counts bits of words 0, 1 (all 32) and the low 6 bits of word 2,
    # counted here with Python's own integer popcount.
    seed = 0xDEADBEEF12345678
    X = O.draw_binomial(seed, 3, 2, 70)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for t in range(3):
        for m in range(2):
            words = philox4x32_10([[t, m, 0, 0]], key)[0]
            expect = (bin(int(words[0])).count("1") + bin(int(words[1])).count("1")
                      + bin(int(words[2]) & 0x3F).count("1"))
            assert X[t, m] == expect


@pytest.mark.parametrize("N", [1, 10, 33, 64, 309])
def test_binomial_law_chi_square(N):
    # Proposition 2: X ~ B(N, 1/2).  Pearson chi-square against the pmf.
    K, d = 4000, 5
    X = O.draw_binomial(12345 + N, K, d, N).ravel()
    assert X.min() >= 0 and X.max() <= N
    pmf = stats.binom.pmf(np.arange(N + 1), N, 0.5)
    # pool the tails so every expected count is >= 5
    exp = pmf * X.size
    obs = np.bincount(X, minlength=N + 1).astype(float)
    keep = exp >= 5
    e = np.append(exp[keep], exp[~keep].sum())
    o = np.append(obs[keep], obs[~keep].sum())
    if e[-1] == 0:
        e, o = e[:-1], o[:-1]
    chi2 = np.sum((o - e) ** 2 / e)
    p = stats.chi2.sf(chi2, len(e) - 1)
    assert p > 1e-4, (chi2, p)


def test_y_moments_and_symmetry():
    N, K, d = 33, 20000, 3
    Y = N - 2 * O.draw_binomial(7, K, d, N)
    assert np.all((Y + N) % 2 == 0) and np.abs(Y).max() <= N
    se = math.sqrt(N / Y.size)
    assert abs(Y.mean()) < 5 * se
    assert abs(Y.var() - N) < 5 * N * math.sqrt(2.0 / Y.size)
    # independence across channels and across consecutive terms
    c01 = np.corrcoef(Y[:, 0], Y[:, 1])[0, 1]
    ct = np.corrcoef(Y[:-1, 0], Y[1:, 0])[0, 1]
    assert abs(c01) < 5 / math.sqrt(K) and abs(ct) < 5 / math.sqrt(K)


def test_draws_deterministic_and_seed_dependent():
    a = O.draw_binomial(99, 50, 3, 40)
    b = O.draw_binomial(99, 50, 3, 40)
    c = O.draw_binomial(100, 50, 3, 40)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    # a prefix of the table does not depend on K (counter-based draws)
    assert np.array_equal(O.draw_binomial(99, 10, 3, 40), a[:10])


def test_sample_terms_frequency_vectors():
    # w_t = W^T Y_t / sqrt(N): <w_t, x> = sum_k Y_k alpha_k (q_k . x) / sqrt(N)
    C = np.array([[100.0, 0, 0], [0, 25, 12.5], [0, 12.5, 25]])
    N = 50
    Y, w = O.sample_terms(C, N, 16, 3)
    lam = np.array([12.5, 37.5, 100.0])
    q = np.array([[0, 1, -1], [0, 1, 1], [1, 0, 0]]) / np.array([[math.sqrt(2)], [math.sqrt(2)], [1]])
    x = np.array([0.3, -1.2, 2.5])
    expect = (Y * (q @ x)[None, :] / np.sqrt(lam)[None, :]).sum(axis=1) / math.sqrt(N)
    assert np.allclose(w @ x, expect, rtol=0, atol=1e-13)
