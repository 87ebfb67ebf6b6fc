"""Pins of the oracle filters: direct exact (O1), direct with the sampled kernel
(O2), separable MCSF of Algorithm 1 (O3) and the full unsampled expansion (O4)."""

import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import mcsf as O
from synth import random_spd, voronoi_image


def _img(H, W, d, seed, lo=0.0, hi=1.0, noise=0.02, cells=5):
    return voronoi_image(H, W, d, cells, lo, hi, noise, seed).astype(np.float64)


def _terms(d, K, seed, scale=8.0):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=(K, d))


# --- O1 against a plain-Python brute force ---------------------------------------

def _brute_bf(f, sigma_s, C):
    H, W, d = f.shape
    R = O.window_radius(sigma_s)
    Ci = np.linalg.inv(C)
    out = np.zeros_like(f)
    for y in range(H):
        for x in range(W):
            num = [0.0] * d
            Z = 0.0
            for jy in range(-R, R + 1):
                for jx in range(-R, R + 1):
                    yy, xx = y - jy, x - jx
                    if not (0 <= yy < H and 0 <= xx < W):
                        continue
                    sp = math.exp(-(jy * jy + jx * jx) / (2 * sigma_s * sigma_s))
                    D = [f[yy, xx, m] - f[y, x, m] for m in range(d)]
                    q = sum(D[a] * Ci[a, b] * D[b] for a in range(d) for b in range(d))
                    wgt = sp * math.exp(-0.5 * q)
                    Z += wgt
                    for m in range(d):
                        num[m] += wgt * f[yy, xx, m]
            out[y, x] = [v / Z for v in num]
    return out


@pytest.mark.parametrize("d", [1, 3])
def test_direct_exact_matches_brute_force(d):
    f = _img(6, 7, d, 11)
    C = np.eye(d) * 0.05 if d == 1 else random_spd(d, -2, -1, 5)
    out, _ = O.direct_exact(f, 1.0, C)
    assert np.max(np.abs(out - _brute_bf(f, 1.0, C))) < 1e-14


# --- O3 (separable, Algorithm 1) equals O2 (direct, sampled kernel) --------------

@pytest.mark.parametrize("d", [1, 3, 6])
@pytest.mark.parametrize("sigma_s", [0.0, 0.5, 1.0, 2.0])
def test_separable_equals_direct_sampled(d, sigma_s):
    # shapes smaller than the window exercise the domain restriction on borders
    f = _img(9, 5, d, 3 + d)
    w = _terms(d, 7, 17 + d)
    o3, num, Z = O.mcsf_separable(f, sigma_s, w)
    o2, Z2 = O.direct_sampled(f, sigma_s, w)
    assert np.max(np.abs(o3 - o2)) < 1e-12
    assert np.max(np.abs(Z / w.shape[0] - Z2)) < 1e-12


def test_separable_weighted_equals_direct_weighted():
    f = _img(8, 8, 3, 4)
    w = _terms(3, 9, 5)
    wt = np.random.default_rng(1).uniform(0.1, 2.0, size=9)
    o3, _, _ = O.mcsf_separable(f, 1.5, w, weights=wt)
    o2, _ = O.direct_sampled(f, 1.5, w, weights=wt)
    assert np.max(np.abs(o3 - o2)) < 1e-12


# --- O4: the full expansion through Algorithm 1 equals the closed form ------------

@pytest.mark.parametrize("d,N", [(1, 6), (2, 4), (3, 3)])
def test_full_expansion_equals_raised_cosine_filter(d, N):
    f = _img(7, 6, d, 20 + d)
    C = np.eye(d) * 0.09 if d != 2 else random_spd(2, -1.5, -0.5, 8)
    W = O.whiten(C)
    w, wt = O.full_expansion_terms(W, N)
    o3, _, _ = O.mcsf_separable(f, 1.0, w, weights=wt)
    o4, _ = O.direct_raised_cosine(f, 1.0, W, N)
    assert np.max(np.abs(o3 - o4)) < 1e-12


# --- invariants ---------------------------------------------------------------

def test_constant_image_unchanged():
    f = np.ones((6, 9, 3)) * np.array([0.2, -0.7, 1.3])
    C = np.eye(3) * 0.01
    w = _terms(3, 5, 2)
    assert np.max(np.abs(O.direct_exact(f, 2.0, C)[0] - f)) < 1e-15
    assert np.max(np.abs(O.direct_sampled(f, 2.0, w)[0] - f)) < 1e-15
    assert np.max(np.abs(O.mcsf_separable(f, 2.0, w)[0] - f)) < 1e-14


def test_sigma_zero_is_identity():
    f = _img(5, 6, 3, 9)
    w = _terms(3, 4, 9)
    assert np.max(np.abs(O.mcsf_separable(f, 0.0, w)[0] - f)) < 1e-15
    assert np.max(np.abs(O.direct_exact(f, 0.0, np.eye(3) * 0.01)[0] - f)) < 1e-15


def test_huge_covariance_gives_gaussian_blur():
    # C -> infinity: phi -> 1 and the filter is the normalised truncated Gaussian
    # blur; computed here with scipy's correlate (zero padding, so the
    # normaliser is the blurred indicator of the image).
    f = _img(10, 12, 3, 31)
    sigma = 1.5
    R = O.window_radius(sigma)
    u = np.arange(-R, R + 1)
    k2 = np.exp(-(u[:, None] ** 2 + u[None, :] ** 2) / (2 * sigma ** 2))
    ones = ndimage.correlate(np.ones(f.shape[:2]), k2, mode="constant")
    blur = np.stack([ndimage.correlate(f[..., m], k2, mode="constant") / ones
                     for m in range(3)], axis=-1)
    out, _ = O.direct_exact(f, sigma, np.eye(3) * 1e12)
    assert np.max(np.abs(out - blur)) < 1e-11
    # the MCSF with near-zero frequencies also reduces to the blur
    w = _terms(3, 6, 3, scale=1e-7)
    o3, _, _ = O.mcsf_separable(f, sigma, w)
    assert np.max(np.abs(o3 - blur)) < 1e-10


def test_shift_and_transpose_invariance():
    f = _img(7, 9, 3, 41)
    w = _terms(3, 6, 4)
    c = np.array([0.5, -2.0, 3.0])
    o, _, _ = O.mcsf_separable(f, 1.0, w)
    o_shift, _, _ = O.mcsf_separable(f + c, 1.0, w)
    assert np.max(np.abs(o_shift - (o + c))) < 1e-12
    o_t, _, _ = O.mcsf_separable(np.transpose(f, (1, 0, 2)), 1.0, w)
    assert np.max(np.abs(o_t - np.transpose(o, (1, 0, 2)))) < 1e-13


def test_whitening_scale_equivariance():
    # B_{s^2 C}[s f] = s B_C[f] for the same seed and order
    f = _img(8, 8, 3, 51)
    C = random_spd(3, -2, -1, 9)
    s = 3.0
    o1, N, _, _ = O.mcsf(f, 1.0, C, 16, 123, N=20)
    o2, _, _, _ = O.mcsf(s * f, 1.0, s * s * C, 16, 123, N=20)
    assert np.max(np.abs(o2 - s * o1)) < 1e-12


def test_order_rule():
    # isotropic sigma_r = 0.1 on a [0,1] image with noise: T = span/0.1
    f = np.zeros((4, 4, 3))
    f[0, 0] = [1.0, 0.5, 0.25]
    W = O.whiten(np.eye(3) * 0.01)
    N = O.choose_order(f, W)
    assert N == math.ceil(((10.0 + 4.0) / math.pi) ** 2)
    assert O.choose_order(np.zeros((2, 2, 1)), np.eye(1)) == 10
    # at that order the kernel has no alias inside the data range
    z = np.linspace(-10.0, 10.0, 2001)
    rc = np.abs(np.cos(z / math.sqrt(N))) ** N
    assert np.all(rc[np.abs(z) > 6] < 1e-3)


# --- Monte Carlo convergence towards the exact filter (statistical) -----------------

def test_sampled_filter_converges_to_exact():
    f = _img(12, 12, 3, 61, noise=0.02, cells=4)
    C = np.eye(3) * 0.15 ** 2
    exact, _ = O.direct_exact(f, 1.0, C)
    W = O.whiten(C)
    N = O.choose_order(f, W)
    rc, _ = O.direct_raised_cosine(f, 1.0, W, N)
    errs = []
    Ks = [8, 32, 128, 512]
    for K in Ks:
        e = []
        for seed in range(6):
            _, w = O.sample_terms(C, N, K, 1000 * K + seed)
            o, _ = O.direct_sampled(f, 1.0, w)
            e.append(O.mse(o, rc))
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(Ks), np.log(errs), 1)[0]
    assert -1.4 < slope < -0.6, slope
    # the order-N kernel itself is close to the Gaussian
    assert O.mse(rc, exact) < 1e-6


def test_mse_hand_values():
    # eq. (MSE): the mean over pixels and channels of the squared difference.
    # a - b = [[1, -2], [3, -4]] (a 2 x 1 x 2 image): (1 + 4 + 9 + 16) / 4 = 7.5
    a = np.array([[[1.0, 0.0]], [[5.0, 2.0]]])
    b = np.array([[[0.0, 2.0]], [[2.0, 6.0]]])
    assert O.mse(a, b) == 7.5
    assert O.mse(a, a) == 0.0
    # in dB on a 255 scale: 10 log10(7.5 * 255^2) = 10 log10(487687.5)
    assert abs(O.mse_db(a, b, scale=255.0) - 56.8814162) < 1e-6
    # 10 log10(100) = 20 dB exactly: a constant offset of 10
    assert abs(O.mse_db(np.full((3, 4, 3), 10.0), np.zeros((3, 4, 3))) - 20.0) < 1e-12
