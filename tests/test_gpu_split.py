"""The FP32 mode with a split vertical pass (BF_FP32_SPLIT) against the FP64
oracle.

This mode keeps the modulated channels and the horizontal pass in FP32 and
stores each horizontal-pass row as an FP16 pair hi + lo (about 22 significant
bits), so that the vertical pass (the sums of eqs. (numerator) and (denom)
over the window rows) runs as exact FP16 products accumulated in FP32.  It is
held to the FP32 bounds of the other parity tests:

* every instance (R = 18, 21, 24, 30) over a whole image of several strips with
  ragged edges against O3: num and Z within 1e-5 of their scale, the output
  within 1e-4 of each channel's range where z >= 0.1;
* the 4096^2 benchmark workload (sigma_s = 10, K = 256) at 4096 sampled
  pixels, every pixel within R of the corners and pixel pairs across the
  strip seams, against O2 (the direct filter with the same terms);
* strip heights change no output bit (the pair's k-blocks are fixed relative
  to the pair), and the result stays within 1e-5 of the range of plain FP32;
* the FP16 range rule of BF_FP16 applies to the FP16 halves;
* edge shapes (shorter than the window, one ragged strip, odd sizes) at
  every split radius against O3 over the whole image;
* a plan (graph, FP64-phase instance) and bf_vec_static give bf_vec_ex's
  bits, and merged +-Y draws stay within FP32 rounding of the full sum;
* phases beyond 2^8 turns (uncentred data near 100) take the instance with
  the FP64 phase reduction; there the halves' rounding (2^-22 of |f|) grows
  relative to the range by max|f| / range, and the bound is scaled so.
"""

import numpy as np
import pytest

import paper_1605_02164_amd as P
from paper_1605_02164_amd import bfvec as B
from oracle import mcsf as O
from synth import workload, voronoi_image
from tests.helpers import (sample_pixels, rel_err_per_channel, corner_blocks, strip_seams,
                           merge_pixels, parallel_pixels)
from tests.test_gpu_parity import assert_close, oracle_terms, cuda, host, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _span(f):
    f2 = np.asarray(f, np.float64).reshape(-1, f.shape[-1])
    s = f2.max(0) - f2.min(0)
    s[s == 0] = 1.0
    return s


@pytest.mark.parametrize("R", [18, 21, 24, 30])
def test_split_instance_against_oracle(R):
    say(f"case split R={R}")
    H, W, d = 2 * R + 45, 3 * 32 + 7, 3
    f = voronoi_image(H, W, d, 5, 0.0, 1.0, 0.02, seed=300 + R)
    C = np.eye(d) * 0.15 ** 2
    sigma = R / 3.0
    assert O.window_radius(sigma) == R
    K, seed = 4, 1000 + R
    fg = cuda(f)
    num = torch.empty_like(fg)
    zo = torch.empty(fg.shape[:2], device="cuda", dtype=torch.float32)
    got, o = P.bf_vec_ex(fg, sigma, C, K, seed, precision="fp32_split", tile_h=24,
                         num_out=num, z_out=zo, return_opts=True)
    got, num, zo = host(got), host(num), host(zo)
    assert o.tile_w_used == 32 and o.tile_h_used == 32 and o.mfma_used == 1
    f64 = f.astype(np.float64)
    W_ = O.whiten(C)
    N = O.choose_order(f64, W_)
    assert o.N_used == N
    _, w = O.sample_terms(C, N, K, seed, W=W_)
    ref, rnum, rZ = O.mcsf_separable(f64, sigma, w)
    scale = K * O.spatial_taps(sigma).sum() ** 2
    z = rZ / scale
    ez = np.max(np.abs(zo - rZ)) / scale
    en = np.max(np.abs(num - rnum)) / (scale * np.abs(f64).max())
    say(f"  N={N} Z err {ez:.3e}, num err {en:.3e} (of their scale); min z {z.min():.3f}")
    assert ez <= 1e-5 and en <= 1e-5
    good = z >= 0.1
    err = rel_err_per_channel(got[good], ref[good], f)
    say(f"  output rel_err={err} (z >= 0.1), {int((~good).sum())} pixels below")
    assert np.all(err <= 1e-4), err
    mid = ~good & (z >= 0.01)
    if mid.any():
        e = np.abs(got[mid] - ref[mid]) / _span(f)
        assert np.all(e * z[mid][:, None] <= 1e-5)


def test_split_full_size_sampled():
    say("case split voronoi4096_d3_s10_K256 full size, sampled pixels")
    f, C, p = workload("voronoi4096_d3_s10_K256")
    H, W, d = f.shape
    sigma, K, seed = p["sigma_s"], p["K"], p["term_seed"]
    R = O.window_radius(sigma)
    fg = cuda(f)
    P.bf_autotune(fg, sigma, precision="fp32_split")
    out, o = P.bf_vec_ex(fg, sigma, C, K, seed, precision="fp32_split", return_opts=True)
    got = host(out)
    say(f"  N={o.N_used} strips {o.tile_h_used} x {o.tile_w_used}")
    pix = merge_pixels(sample_pixels(H, W, 4096, 12, R=R, seams_y=strip_seams(H, o.tile_h_used),
                                     seams_x=strip_seams(W, o.tile_w_used)),
                       corner_blocks(H, W, R))
    f64 = f.astype(np.float64)
    Nref, w = oracle_terms(f64, C, K, seed)
    assert o.N_used == Nref
    ref, Z = parallel_pixels(lambda c: O.direct_sampled(f64, sigma, w, pixels=c), pix)
    z = Z / O.spatial_taps(sigma).sum() ** 2
    say(f"  pixels={len(pix)}")
    assert_close(got[pix[:, 0], pix[:, 1]], ref, f, z)


def test_split_heights_bitwise_and_close_to_fp32():
    say("case split strip heights, against FP32")
    f, C, p = workload("lab1024_d3_s5_K128")
    f = np.ascontiguousarray(f[:512, :384])
    sigma, K, seed = 10.0, 32, 5
    fg = cuda(f)
    outs = []
    for th in (32, 96, 0):
        out, o = P.bf_vec_ex(fg, sigma, C, K, seed, precision="fp32_split", tile_h=th,
                             return_opts=True)
        outs.append(host(out))
        say(f"  tile_h {th} -> {o.tile_h_used}")
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ref, _ = P.bf_vec_ex(fg, sigma, C, K, seed, precision="fp32")
    d = np.abs(outs[0] - host(ref)).reshape(-1, 3).max(0) / _span(f)
    say(f"  max |split - fp32| / range = {d}")
    assert np.all(d <= 1e-5), d


def test_split_fp16_range_guard():
    say("case split range guard")
    f = voronoi_image(40, 48, 3, 4, 0.0, 4000.0, 1.0, seed=9)
    C = 400.0 ** 2 * np.eye(3)
    with pytest.raises(P.BfError) as e:
        P.bf_vec_ex(cuda(f), 10.0, C, 4, 1, precision="fp32_split")
    assert e.value.code == B.BF_EUNSUPPORTED and "FP16" in str(e.value)


def test_split_large_phases_reduced_in_fp64():
    # uncentred data near 100 with sigma_r = 0.02: phases reach thousands of
    # turns and the instance with the FP64 phase reduction runs; the split
    # halves hold |f| x sum(omega_1) ~ 2.5e3 (within the FP16 range rule)
    say("case split large phases: 160x160x3 in [100, 101], sigma_r = 0.02, no centring")
    # (an image several windows across, so that most pixels see a well
    # conditioned normaliser)
    f = voronoi_image(160, 160, 3, 3, 100.0, 101.0, 0.02, 123)
    C = 0.02 ** 2 * np.eye(3)
    K, seed, sigma = 32, 17, 10.0
    got, N_used = P.bf_vec_ex(cuda(f), sigma, C, K, seed, center=False, precision="fp32_split")
    got = host(got)
    f64 = f.astype(np.float64)
    Nref, w = oracle_terms(f64, C, K, seed)
    assert N_used == Nref
    turns = np.abs(np.tensordot(f64, w.T, axes=(2, 0))).max() / (2 * np.pi)
    say(f"  N={N_used} max |phase| = {turns:.0f} turns")
    assert turns > 256
    ref, _, Z = O.mcsf_separable(f64, sigma, w)
    z = Z / (K * O.spatial_taps(sigma).sum() ** 2)
    # uncentred data: the stored values carry the offset (|f| ~ 100 against a
    # range of 1), so relative to the range the rounding of the stored halves
    # (about 2^-22 of |f|, against FP32's 2^-24) grows by max|f| / range; the
    # bound is FP32's 1e-4 at |f|/range = 1 scaled that way (16 ulps of the
    # split values), taken where the ratio is well conditioned
    ok = z >= 0.1
    tol = 16.0 * np.abs(f64).max() / _span(f).min() * 2.0 ** -22
    err = rel_err_per_channel(got[ok], ref[ok], f)
    ref32 = host(P.bf_vec_ex(cuda(f), sigma, C, K, seed, center=False, precision="fp32")[0])
    err32 = rel_err_per_channel(ref32[ok], ref[ok], f)
    say(f"  rel_err={err} (FP32 {err32}; bound {tol:.2e}; z >= 0.1), "
        f"{int((~ok).sum())} pixels below")
    assert ok.sum() > 0.5 * ok.size and np.all(err <= tol), err


def test_split_plan_bitwise_equal_to_vec_ex():
    # a plan runs the FP64-phase instance in a captured graph; lanes below
    # 2^8 turns run the same operations as bf_vec_ex's instance
    say("case split plan")
    f, C, p = workload("lab1024_d3_s5_K128")
    f = np.ascontiguousarray(f[:256, :200])
    sigma, K, seed = 8.0, 16, 21
    fg = cuda(f)
    ref, o = P.bf_vec_ex(fg, sigma, C, K, seed, precision="fp32_split", return_opts=True)
    ref = host(ref)
    with P.Plan(*f.shape, sigma, C, K, seed, N=o.N_used, precision="fp32_split") as plan:
        assert plan.tile_w_used == 32 and plan.mfma_used == 1
        for _ in range(3):
            assert np.array_equal(host(plan(fg)), ref)


def test_split_static_dedup_and_weighted_terms():
    # the split instances behind the other entry points: bf_vec_static (static
    # scratch) gives bf_vec_ex's bits; merged +-Y draws (exact in arithmetic)
    # stay within FP32 rounding of the K drawn terms
    say("case split static / dedup")
    f = voronoi_image(256, 320, 3, 12, 0.0, 1.0, 0.02, seed=77)
    C = 0.1 ** 2 * np.eye(3)
    fg = cuda(f)
    ref, o = P.bf_vec_ex(fg, 10.0, C, 48, 5, precision="fp32_split", return_opts=True)
    got, os_ = P.bf_vec_static(fg, 10.0, C, 48, 5, precision="fp32_split", return_opts=True)
    assert (os_.tile_h_used, os_.tile_w_used) == (o.tile_h_used, o.tile_w_used)
    assert np.array_equal(host(got), host(ref))
    dd, od = P.bf_vec_ex(fg, 10.0, C, 48, 5, precision="fp32_split", dedup=True, return_opts=True)
    say(f"  K_used {od.K_used} of 48")
    assert od.K_used < 48
    e = np.abs(host(dd) - host(ref)).reshape(-1, 3).max(0) / _span(f)
    say(f"  max |dedup - full| / range = {e}")
    assert np.all(e <= 1e-5), e


@pytest.mark.parametrize("H,W,sigma", [(17, 33, 10.0), (40, 200, 6.0), (300, 35, 8.0),
                                       (129, 97, 7.0)])
def test_split_edge_shapes(H, W, sigma):
    # images shorter than the window, one ragged strip across, odd sizes
    say(f"case split edge shape {H}x{W} sigma_s={sigma}")
    f = voronoi_image(H, W, 3, 4, 0.0, 1.0, 0.02, seed=H * 7 + W)
    C = 0.12 ** 2 * np.eye(3)
    K, seed = 8, 3
    got, N = P.bf_vec_ex(cuda(f), sigma, C, K, seed, precision="fp32_split")
    got = host(got)
    f64 = f.astype(np.float64)
    Nref, w = oracle_terms(f64, C, K, seed)
    assert N == Nref
    ref, _, Z = O.mcsf_separable(f64, sigma, w)
    assert_close(got, ref, f, Z / (K * O.spatial_taps(sigma).sum() ** 2))
