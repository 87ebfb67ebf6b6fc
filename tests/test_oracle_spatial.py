"""Pins of the oracle's box-family spatial filters (Section 3, remark after
Algorithm 1: the Gaussian omega may be replaced by a box, a hat or any other
spatial filter).  Taps are checked against closed forms and brute-force
counts, the radius rule against hand values, and the filter itself against
scipy's uniform filter on a zero-padded image (an independent library)."""

import itertools
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import mcsf as O
from synth import voronoi_image


def sigma_for(r, n):
    """sigma_s whose variance rule gives exactly radius r for n boxes."""
    return math.sqrt(n * ((2 * r + 1) ** 2 - 1) / 12.0)


def count_sums(r, n, u):
    """Number of (a_1..a_n) in [-r, r]^n with sum u (stars and bars with
    inclusion-exclusion over the n upper bounds)."""
    w = 2 * r + 1
    s = u + n * r                        # shift each a_i to [0, w - 1]
    tot = 0
    for k in range(n + 1):
        m = s - k * w
        if m >= 0:
            tot += (-1) ** k * math.comb(n, k) * math.comb(m + n - 1, n - 1)
    return tot


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("r", [0, 1, 2, 5, 10])
def test_box_taps_closed_form(n, r):
    sig = sigma_for(r, n)
    taps = O.spatial_taps(sig, n)
    R = O.window_radius(sig, n)
    assert R == n * r and len(taps) == 2 * R + 1
    u = np.arange(-R, R + 1)
    expect = np.array([count_sums(r, n, int(v)) for v in u], dtype=np.float64)
    assert np.array_equal(taps, expect)
    if n == 1:
        assert np.array_equal(taps, np.ones(2 * r + 1))
    if n == 2:                                   # hat: 2r + 1 - |u|
        assert np.array_equal(taps, (2 * r + 1 - np.abs(u)).astype(np.float64))
    # normalisation and second moment of the n-fold box
    assert taps.sum() == (2 * r + 1) ** n
    var = float((u * u * taps).sum() / taps.sum())
    assert math.isclose(var, n * ((2 * r + 1) ** 2 - 1) / 12.0, rel_tol=1e-12, abs_tol=1e-12)
    assert math.isclose(var, sig * sig, rel_tol=1e-12, abs_tol=1e-12)


@pytest.mark.parametrize("r", [1, 2])
def test_three_box_taps_brute_force(r):
    taps = O.spatial_taps(sigma_for(r, 3), 3)
    counts = np.zeros(6 * r + 1)
    for a, b, c in itertools.product(range(-r, r + 1), repeat=3):
        counts[a + b + c + 3 * r] += 1
    assert np.array_equal(taps, counts)


def test_box_radius_rule_hand_values():
    # r = round((sqrt(12 sigma^2 / n + 1) - 1) / 2)
    assert O.box_radius(10.0, 3) == 10        # x = 9.51
    assert O.box_radius(10.0, 2) == 12        # x = 11.76
    assert O.box_radius(10.0, 1) == 17        # x = 16.83
    assert O.box_radius(2.0, 3) == 2          # x = 1.56
    assert O.box_radius(1.0, 1) == 1          # x = 1.0 exactly
    assert O.box_radius(0.0, 3) == 0
    assert O.window_radius(10.0, 3) == 30 and O.window_radius(0.0, 2) == 0
    # identity at r = 0
    assert np.array_equal(O.spatial_taps(0.0, 3), [1.0])


@pytest.mark.parametrize("n", [1, 2, 3])
def test_box_filter_at_zero_phase_is_normalised_smoothing(n):
    # one term with w = 0: cos = 1, sin = 0, so out = (omega * f) / (omega * 1)
    # over the image domain.  Reference: scipy's box mean filter applied n times
    # per axis to the image zero-padded by R (so intermediates are exact), then
    # cropped; the division cancels the 1/(2r+1)^n scale.
    f = voronoi_image(23, 31, 3, 4, 0.0, 1.0, 0.05, 17).astype(np.float64)
    sig = 1.7
    r = O.box_radius(sig, n)
    R = n * r
    out, num, Z = O.mcsf_separable(f, sig, np.zeros((1, 3)), spatial=n)

    def smooth(a):
        p = np.pad(a, ((R, R), (R, R)))
        for _ in range(n):
            for ax in (0, 1):
                p = ndimage.uniform_filter1d(p, 2 * r + 1, axis=ax, mode="constant", cval=0.0)
        return p[R:R + a.shape[0], R:R + a.shape[1]]

    ones = smooth(np.ones(f.shape[:2]))
    for m in range(3):
        ref = smooth(f[..., m]) / ones
        assert np.max(np.abs(out[..., m] - ref)) < 1e-12
    assert np.allclose(Z, ones * (2 * r + 1) ** (2 * n), rtol=1e-12)


@pytest.mark.parametrize("n", [1, 3])
def test_box_separable_equals_direct_sampled(n):
    # O3 (separable, modulated) against O2 (direct, sampled kernel) with the
    # same box-family omega: cos(a - b) = cos a cos b + sin a sin b
    f = voronoi_image(14, 17, 2, 3, 0.0, 1.0, 0.02, 5)
    rng = np.random.default_rng(3)
    w = rng.normal(scale=4.0, size=(5, 2))
    out3, _, Z3 = O.mcsf_separable(f, 1.3, w, spatial=n)
    out2, Z2 = O.direct_sampled(f, 1.3, w, spatial=n)
    assert np.max(np.abs(out3 - out2)) < 1e-10
    assert np.max(np.abs(Z3 - Z2 * 5)) < 1e-9 * np.abs(Z3).max()
