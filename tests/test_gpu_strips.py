"""GPU tests of the strip width of the fused kernel (through the C ABI).

For d = 3 at the radii with compile-time kernels the fused kernel has
instances with 32-column strips (eight waves per workgroup) beside the
16-column ones; opts.tile_w forces a width (0 = automatic: 32 where such an
instance exists, occupancy allows and the image fills the GPU) and
opts.tile_w_used reports it.

At these radii the passes run as banded matrix products on the matrix cores:
both passes with 16-bit storage at either width, and for FP32 the horizontal
pass of 32-column strips from R = 12 up.  Each output pixel then sees the
same operations in the same order at either width, except FP32 at R >= 12,
where the 32-column strips' matrix-core sums run in another order than the
16-column FMA passes: there both widths are held to the oracle bound (FP32
1e-4); everywhere else the two must agree bit for bit (16-bit results are
also held to the storage bound against the oracle, as in test_gpu_parity).
At equal width, plans and the serving scheduler's batched launches must
equal bf_vec_ex bit for bit.
"""

import sys

import numpy as np
import pytest

import paper_1605_02164_amd as P
from paper_1605_02164_amd import bfvec as B
from oracle import mcsf as O
from synth import workload, voronoi_image
from tests.helpers import rel_err_per_channel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp32": 1e-4, "fp16": 3e-3, "bf16": 3e-2}
ZMIN = 1e-2


def widths_differ(precision, R):
    """Whether 32- and 16-column strips sum in different orders (the library's
    rule for FP32 matrix-core passes)."""
    return precision == "fp32" and R >= 12


def oracle(f, sigma, C, K, seed, N):
    """O3 and the normaliser's conditioning z = Z / (K sum omega)."""
    _, w = O.sample_terms(C, N, K, seed, W=O.whiten(C))
    ref, _, Z = O.mcsf_separable(np.asarray(f, np.float64), sigma, w)
    return ref, Z / (K * O.spatial_taps(sigma).sum() ** 2)


def check_oracle(got, ref, f, z, precision):
    """FP32: 1e-4 of the range where z >= 1e-2.  16-bit storage: the storage
    bound on error x min(1, z / 0.1), as in test_gpu_parity."""
    ok = z >= ZMIN
    err = rel_err_per_channel(np.asarray(got, np.float64)[ok], ref[ok], f)
    if precision == "fp32":
        say(f"  rel_err={err}")
        assert np.all(err <= TOL["fp32"]), err
        return
    f2 = np.asarray(f, np.float64).reshape(-1, f.shape[-1])
    span = np.maximum(f2.max(0) - f2.min(0), 1e-30)
    d = np.abs(np.asarray(got, np.float64)[ok] - ref[ok]).reshape(-1, f.shape[-1]) / span
    scaled = (d * np.minimum(1.0, z[ok] / 0.1)[:, None]).max()
    say(f"  max err {d.max():.3e} scaled {scaled:.3e}")
    assert scaled <= TOL[precision]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run(fg, sigma, C, K, seed, N, precision, tile_w, **kw):
    out, o = P.bf_vec_ex(fg, sigma, C, K, seed, N=N, precision=precision, tile_w=tile_w,
                         return_opts=True, **kw)
    return host(out), o


# H, W, sigma_s (R = 3 sigma_s), K, precision: ragged widths (W not a multiple
# of 32), every specialised radius, one strip across
CASES = [
    (72, 100, 2.0, 12, "fp32"),
    (64, 97, 3.0, 12, "fp16"),
    (50, 130, 4.0, 8, "bf16"),
    (90, 33, 10.0, 6, "fp32"),
    (41, 64, 8.0, 6, "fp16"),
    (120, 250, 5.0, 10, "bf16"),
    (33, 161, 7.0, 6, "fp32"),
    (100, 70, 6.0, 6, "fp16"),
    (56, 90, 6.0, 6, "fp32"),
    (40, 120, 10.0, 4, "bf16"),
]


@pytest.mark.parametrize("H,W,sigma,K,precision", CASES)
def test_wide_strips_against_narrow(H, W, sigma, K, precision):
    R = O.window_radius(sigma)
    say(f"case strips {H}x{W}x3 sigma_s={sigma} (R={R}) K={K} {precision}: "
        "32 vs 16 columns, bf_vec_ex and plans")
    C = np.diag([0.12, 0.1, 0.15]) ** 2
    f = voronoi_image(H, W, 3, 10, 0.0, 1.0, 0.02, 100 + H + W)
    fg = cuda(f)
    narrow, o16 = run(fg, sigma, C, K, 5, 14, precision, 16)
    wide, o32 = run(fg, sigma, C, K, 5, 14, precision, 32)
    auto, oa = run(fg, sigma, C, K, 5, 14, precision, 0)
    say(f"  automatic width {oa.tile_w_used}")
    assert (o16.tile_w_used, o32.tile_w_used) == (16, 32)
    assert oa.tile_w_used in (16, 32)
    assert np.array_equal(auto, wide if oa.tile_w_used == 32 else narrow)
    if not widths_differ(precision, R):
        assert np.array_equal(wide, narrow)
    if widths_differ(precision, R) or precision != "fp32":
        ref, z = oracle(f, sigma, C, K, 5, 14)
        check_oracle(narrow, ref, f, z, precision)
        check_oracle(wide, ref, f, z, precision)
    for tw, same in ((16, narrow), (32, wide)):
        with B.Plan(H, W, 3, sigma, C, K, 5, 14, precision=precision, tile_w=tw) as plan:
            assert plan.tile_w_used == tw
            assert np.array_equal(host(plan(fg)), same)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_wide_strips_against_oracle(precision):
    say(f"case strips 80x112x3 sigma_s=3 K=16 N=14 {precision}: 32-column strips vs oracle")
    f, C, _ = workload("voronoi128_d3_s2_K64", H=80, W=112)
    K, N, seed, sigma = 16, 14, 9, 3.0
    got, o = run(cuda(f), sigma, C, K, seed, N, precision, 32)
    assert o.tile_w_used == 32
    ref, z = oracle(f, sigma, C, K, seed, N)
    check_oracle(got, ref, f, z, precision)


def test_wide_strips_with_fp64_phase_path():
    say("case strips 256x320x3 sigma_s=3, uncentred data near 3000 (FP64 phase path): "
        "32 vs 16 columns")
    C = np.eye(3) * 0.1 ** 2
    fg = cuda(voronoi_image(256, 320, 3, 6, 0.0, 1.0, 0.02, 4) + 3000.0)
    narrow, _ = run(fg, 3.0, C, 6, 1, 12, "fp32", 16, center=False)
    wide, o = run(fg, 3.0, C, 6, 1, 12, "fp32", 0, center=False)
    assert o.tile_w_used == 32
    assert np.array_equal(wide, narrow)


def test_automatic_width():
    say("case strips: automatic width -> 32 columns on a 256x320 image at R = 9, 16 for "
        "d = 4, W < 32, a radius without a compile-time kernel, the running-sum variant, "
        "an image too small to fill the GPU")
    C3 = np.eye(3) * 0.1 ** 2

    def width(f, sigma, C, **kw):
        return run(cuda(f), sigma, C, 2, 1, 12, "fp32", 0, **kw)[1].tile_w_used

    f3 = voronoi_image(256, 320, 3, 6, 0.0, 1.0, 0.02, 4)
    assert width(f3, 3.0, C3) == 32
    assert width(f3, 2.5, C3) == 16                                    # R = 8
    assert width(f3, 3.0, C3, spatial="box+runsum") == 16              # FP64 running sums
    assert width(f3, 3.0, C3, spatial="box3+runsum") == 16             # (sliding sums: asked for)
    f4 = voronoi_image(256, 320, 4, 6, 0.0, 1.0, 0.02, 5)
    assert width(f4, 3.0, np.eye(4) * 0.1 ** 2) == 16                  # d = 4
    f3 = voronoi_image(4096, 20, 3, 6, 0.0, 1.0, 0.02, 3)
    assert width(f3, 3.0, C3) == 16                                    # W < 32
    small = voronoi_image(128, 128, 3, 6, 0.0, 1.0, 0.02, 6)
    assert width(small, 3.0, C3) == 16                                 # 8 x 16 strips
    assert run(cuda(small), 3.0, C3, 2, 1, 12, "fp32", 32)[1].tile_w_used == 32


@pytest.mark.parametrize("precision,sigma", [("fp32", 3.0), ("fp32", 5.0), ("fp16", 3.0),
                                             ("bf16", 5.0)])
def test_server_batches_with_wide_strips(precision, sigma):
    say(f"case strips: serving scheduler (32 columns, one term per round) vs bf_vec_ex, "
        f"three d = 3 requests, {precision}, sigma_s={sigma} (R={O.window_radius(sigma)})")
    C = np.eye(3) * 0.12 ** 2
    imgs = [cuda(voronoi_image(256 + 8 * i, 300 + 20 * i, 3, 8, 0.0, 1.0, 0.02, 70 + i))
            for i in range(3)]
    assert run(imgs[0], sigma, C, 8, 4, 14, precision, 0)[1].tile_w_used == 32
    refs = [run(g, sigma, C, 8, 4, 14, precision, 0)[0] for g in imgs]
    with P.Server(quantum_us=1e-9) as srv:
        subs = [srv.submit(g, sigma, C, 8, 4, N=14, precision=precision) for g in imgs]
        for (t, out), ref in zip(subs, refs):
            st = srv.wait(t, 60.0)
            assert st["state"] == "done", st
            assert np.array_equal(host(out), ref)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_wide_strips_full_size_against_narrow(precision):
    say(f"case strips voronoi4096_d3_s10_K256 full size, K=8 {precision}: "
        "32 columns (benchmark launch) vs 16")
    f, C, p = workload("voronoi4096_d3_s10_K256")
    fg = cuda(f)
    wide, o = run(fg, p["sigma_s"], C, 8, p["term_seed"], 37, precision, 0)
    say(f"  tile_w_used={o.tile_w_used} tile_h_used={o.tile_h_used}")
    assert o.tile_w_used == 32
    zt = torch.empty(fg.shape[:2], dtype=torch.float32, device="cuda")
    narrow, _ = run(fg, p["sigma_s"], C, 8, p["term_seed"], 37, precision, 16, z_out=zt)
    if not widths_differ(precision, O.window_radius(p["sigma_s"])):
        assert np.array_equal(wide, narrow)
    else:
        # two evaluations of the same sum: their difference, scaled by
        # the normaliser's conditioning as in the oracle bound, stays inside
        # the bound each meets against the oracle
        z = (host(zt).astype(np.float64) / (8 * O.spatial_taps(p["sigma_s"]).sum() ** 2)).ravel()
        span = f.reshape(-1, 3).max(0) - f.reshape(-1, 3).min(0)
        dev = np.abs(wide.astype(np.float64) - narrow).reshape(-1, 3) / span
        scaled = (dev * np.minimum(1.0, np.abs(z) / 0.1)[:, None])[np.abs(z) >= ZMIN].max()
        say(f"  max |32 - 16 columns| / range = {dev.max():.3e}, scaled {scaled:.3e}")
        assert scaled <= TOL[precision]
