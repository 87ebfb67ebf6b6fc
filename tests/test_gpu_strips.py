"""GPU tests of the strip width of the fused kernel (through the C ABI).

For d = 3 at the radii with compile-time kernels, launches without the FP64
phase path run 32-column strips (eight waves per workgroup); every other
launch, and every plan (plans always take the instance with the FP64 phase
path), runs 16-column strips.  Each output pixel is computed by the same
operations in the same order in both, so bf_vec_ex (wide strips) and a plan
with the same arguments (narrow strips) must agree bit for bit.  The width
each ran with is reported in tile_w_used.  One case per precision is also
checked against the FP64 oracle.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def wide_and_narrow(fg, sigma, C, K, seed, N, precision, **kw):
    H, W, d = fg.shape
    wide, o = P.bf_vec_ex(fg, sigma, C, K, seed, N=N, precision=precision, return_opts=True,
                          **kw)
    wide = host(wide)
    with B.Plan(H, W, d, sigma, C, K, seed, N, precision=precision, **kw) as plan:
        narrow = host(plan(fg))
        assert plan.tile_w_used == 16
    return wide, narrow, o


# H, W, sigma_s (R = 3 sigma_s), K, precision, expected width (None: set by
# the instance's occupancy, either is valid): ragged widths (W not a multiple
# of 32), every specialised radius, one strip across
CASES = [
    (72, 100, 2.0, 12, "fp32", 32),
    (64, 97, 3.0, 12, "fp16", 32),
    (50, 130, 4.0, 8, "bf16", 32),
    (90, 33, 10.0, 6, "fp32", 32),
    (41, 64, 8.0, 6, "fp16", 32),
    (120, 250, 5.0, 10, "bf16", 32),
    (33, 161, 7.0, 6, "fp32", 32),
    (100, 70, 6.0, 6, "fp16", 32),
    (56, 90, 6.0, 6, "fp32", None),
    (40, 120, 10.0, 4, "bf16", 32),
]


@pytest.mark.parametrize("H,W,sigma,K,precision,width", CASES)
def test_wide_strips_bitwise_equal_to_narrow(H, W, sigma, K, precision, width):
    R = O.window_radius(sigma)
    say(f"case strips {H}x{W}x3 sigma_s={sigma} (R={R}) K={K} {precision}: "
        "bf_vec_ex (32 columns) vs plan (16 columns)")
    C = np.diag([0.12, 0.1, 0.15]) ** 2
    fg = cuda(voronoi_image(H, W, 3, 10, 0.0, 1.0, 0.02, 100 + H + W))
    wide, narrow, o = wide_and_narrow(fg, sigma, C, K, 5, 14, precision)
    say(f"  tile_w_used={o.tile_w_used}")
    assert o.tile_w_used == width if width else o.tile_w_used in (16, 32)
    assert np.array_equal(wide, narrow)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_wide_strips_against_oracle(precision):
    say(f"case strips 80x112x3 sigma_s=3 K=16 N=14 {precision}: 32-column strips vs oracle")
    f, C, _ = workload("voronoi128_d3_s2_K64", H=80, W=112)
    K, N, seed, sigma = 16, 14, 9, 3.0
    got, o = P.bf_vec_ex(cuda(f), sigma, C, K, seed, N=N, precision=precision,
                         return_opts=True)
    assert o.tile_w_used == 32
    W = O.whiten(C)
    _, w = O.sample_terms(C, N, K, seed, W=W)
    ref, _, Z = O.mcsf_separable(np.asarray(f, np.float64), sigma, w)
    z = Z / (K * O.spatial_taps(sigma).sum() ** 2)
    ok = z >= 1e-2
    err = rel_err_per_channel(host(got).astype(np.float64)[ok], ref[ok], f)
    say(f"  rel_err={err} ill-conditioned={int((~ok).sum())}")
    assert np.all(err <= TOL[precision]), err


def test_narrow_strips_where_no_wide_instance():
    say("case strips: d = 4, W < 32, a radius without a compile-time kernel, large "
        "phases, the running-sum variant -> 16 columns")
    C3 = np.eye(3) * 0.1 ** 2
    f3 = voronoi_image(40, 20, 3, 6, 0.0, 1.0, 0.02, 3)
    _, o = P.bf_vec_ex(cuda(f3), 3.0, C3, 4, 1, N=12, return_opts=True)
    assert o.tile_w_used == 16                       # W < 32
    f3 = voronoi_image(40, 64, 3, 6, 0.0, 1.0, 0.02, 4)
    _, o = P.bf_vec_ex(cuda(f3), 2.5, C3, 4, 1, N=12, return_opts=True)
    assert o.tile_w_used == 16                       # R = 8
    _, o = P.bf_vec_ex(cuda(f3), 3.0, C3, 4, 1, N=12, spatial="box3+runsum", return_opts=True)
    assert o.tile_w_used == 16                       # running-sum variant
    _, o = P.bf_vec_ex(cuda(f3 + 3000.0), 3.0, C3, 4, 1, N=12, center=False, return_opts=True)
    assert o.tile_w_used == 16                       # FP64 phase path
    f4 = voronoi_image(40, 64, 4, 6, 0.0, 1.0, 0.02, 5)
    _, o = P.bf_vec_ex(cuda(f4), 3.0, np.eye(4) * 0.1 ** 2, 4, 1, N=12, return_opts=True)
    assert o.tile_w_used == 16                       # d = 4


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_wide_strips_full_size_bitwise_equal_to_narrow(precision):
    say(f"case strips voronoi4096_d3_s10_K256 full size, K=8 {precision}: "
        "bf_vec_ex (32 columns, benchmark launch) vs plan (16 columns)")
    f, C, p = workload("voronoi4096_d3_s10_K256")
    fg = cuda(f)
    wide, narrow, o = wide_and_narrow(fg, p["sigma_s"], C, 8, p["term_seed"], 37, precision)
    say(f"  tile_w_used={o.tile_w_used} tile_h_used={o.tile_h_used}")
    assert o.tile_w_used == 32
    assert np.array_equal(wide, narrow)
