"""GPU parity of the box-family spatial filters (box, hat, three boxes) against
the FP64 oracle, through the C ABI.

By default both passes are FIR passes over the box taps; with "+runsum"
(BF_SPATIAL_RUNSUM, FP32) the vertical pass is FP64 running sums over the
horizontal-pass rows.  Both paths are checked.
Tolerances as for the Gaussian: 1e-4 of each channel's range for FP32 where
the normaliser is well conditioned (z >= 1e-2, see test_gpu_parity), 3e-3 for
FP16 storage.  The full-size case runs the benchmark's launch configuration
(4096^2, 1024-row strips), where the running sums span the longest strips.
"""

import sys

import numpy as np
import pytest

import paper_1605_02164_amd as P
from paper_1605_02164_amd import bfvec as B
from oracle import mcsf as O
from synth import workload, voronoi_image, random_spd
from tests.helpers import sample_pixels, rel_err_per_channel

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
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_full(f, sigma, C, K, seed, N, n):
    W = O.whiten(C)
    _, w = O.sample_terms(C, N, K, seed, W=W)
    ref, _, Z = O.mcsf_separable(np.asarray(f, np.float64), sigma, w, spatial=n)
    return ref, Z / (K * O.spatial_taps(sigma, n).sum() ** 2)


def check(got, ref, f, z, tol):
    ok = z >= 1e-2
    err = rel_err_per_channel(got[ok], ref[ok], f)
    say(f"  rel_err={err} ill-conditioned={int((~ok).sum())}")
    assert np.all(err <= tol), err


SPATIAL = [("box", 1), ("hat", 2), ("box3", 3)]


@pytest.mark.parametrize("name,n", SPATIAL)
@pytest.mark.parametrize("precision,flag", [("fp32", ""), ("fp32", "+runsum"), ("fp16", "")])
def test_box_family_full_image(name, n, precision, flag):
    say(f"case spatial={name}{flag} {precision} 96x80x3 sigma_s=2.5 K=24 N=16")
    f, C, p = workload("voronoi128_d3_s2_K64", H=96, W=80)
    K, N, seed, sigma = 24, 16, 7, 2.5
    got = host(P.bf_vec_ex(cuda(f), sigma, C, K, seed, N=N, precision=precision,
                           spatial=name + flag)[0])
    ref, z = oracle_full(f, sigma, C, K, seed, N, n)
    check(got, ref, f, z, TOL[precision])


EDGE = [
    # H, W, d, sigma_s, K, spatial
    (1, 1, 3, 2.0, 4, 3),
    (37, 1, 2, 2.0, 3, 2),
    (33, 17, 4, 0.0, 3, 3),       # r = 0: the identity
    (40, 23, 5, 1.5, 3, 1),
    (70, 50, 8, 2.5, 2, 3),
    (130, 41, 3, 10.0, 2, 3),     # R = 30: window taller than the strip's width
    (64, 48, 3, 13.0, 2, 3),      # R = 39, the largest three-box window
    (50, 60, 3, 23.4, 2, 1),      # R = 40 box
    (48, 40, 6, 8.0, 2, 2),       # d = 6 hat, R = 2 * 9
]


@pytest.mark.parametrize("H,W,d,sigma,K,n", EDGE)
def test_box_family_edge_shapes(H, W, d, sigma, K, n):
    say(f"case spatial edge H={H} W={W} d={d} sigma_s={sigma} K={K} n={n} "
        f"R={O.window_radius(sigma, n)}, FIR and running-sum vertical passes")
    f = voronoi_image(H, W, d, 3, 0.0, 1.0, 0.02, 11 + H + W + d)
    C = np.eye(d) * 0.15 ** 2 if d % 2 else random_spd(d, -2.0, -1.0, d)
    ref, z = oracle_full(f, sigma, C, K, 5, 12, n)
    for sp in (n, n | B.BF_SPATIAL_RUNSUM):
        got = host(P.bf_vec_ex(cuda(f), sigma, C, K, 5, N=12, spatial=sp)[0])
        check(got, ref, f, z, TOL["fp32"])


@pytest.mark.parametrize("spatial", ["box3", "box3+runsum"])
def test_box3_full_size_sampled(spatial):
    say(f"case spatial={spatial} voronoi4096_d3_s10_K256 full size (benchmark launch), "
        "sampled pixels")
    f, C, p = workload("voronoi4096_d3_s10_K256")
    K, seed, sigma = p["K"], p["term_seed"], p["sigma_s"]
    fg = cuda(f)
    got, o = P.bf_vec_ex(fg, sigma, C, K, seed, spatial=spatial, return_opts=True)
    got = host(got)
    say(f"  N={o.N_used} tile_h={o.tile_h_used}")
    f64 = f.astype(np.float64)
    W = O.whiten(C)
    _, w = O.sample_terms(C, o.N_used, K, seed, W=W)
    pix = sample_pixels(p["H"], p["W"], 48, 9, R=O.window_radius(sigma, 3))
    ref, Z = O.direct_sampled(f64, sigma, w, pixels=pix, spatial=3)
    z = Z / O.spatial_taps(sigma, 3).sum() ** 2
    check(got[pix[:, 0], pix[:, 1]], ref, f, z, TOL["fp32"])


@pytest.mark.parametrize("precision,name", [("fp32", "box3+runsum"), ("fp32", "box"),
                                            ("fp16", "hat")])
def test_box_family_plan_and_server_match_standalone(precision, name):
    say(f"case spatial={name} {precision}: plan and server bitwise equal to bf_vec_ex")
    H, W, d, sigma, K, N = 72, 90, 3, 3.0, 16, 14
    C = np.eye(3) * 0.12 ** 2
    f = cuda(voronoi_image(H, W, d, 8, 0.0, 1.0, 0.02, 31))
    ref = host(P.bf_vec_ex(f, sigma, C, K, 4, N=N, precision=precision, spatial=name)[0])
    with B.Plan(H, W, d, sigma, C, K, 4, N, precision=precision, spatial=name) as plan:
        got = host(plan(f))
    assert np.array_equal(got, ref)
    with P.Server(quantum_us=1e-9) as srv:        # one term per round: resumed term ranges
        t, out = srv.submit(f, sigma, C, K, 4, N=N, precision=precision, spatial=name)
        st = srv.wait(t, 60.0)
        assert st["state"] == "done", st
        assert np.array_equal(host(out), ref)


@pytest.mark.parametrize("R", [6, 9, 12, 15, 18, 21, 24, 30])
def test_box3_sliding_sums_every_radius(R):
    # Three boxes with BF_SPATIAL_RUNSUM at d = 3 and a compile-time radius:
    # with 32-column strips asked for, the vertical pass is cascaded sliding
    # box sums (and the horizontal pass a matrix-core product over the box
    # taps); the automatic width and forced 16-column strips run the FP64
    # running-sum instance.  All against the oracle's three-box filter over a
    # whole image of several strips both ways (ragged), at the automatic strip
    # height and at 24 rows.
    r = R // 3
    sigma = float(np.sqrt(r * (r + 1)))      # box_radius(sigma, 3) = r exactly
    assert O.window_radius(sigma, 3) == R
    H, W = 2 * R + 45, 3 * 32 + 7
    say(f"case sliding three-box sums R={R} (r={r}) {H}x{W}x3")
    f = voronoi_image(H, W, 3, 5, 0.0, 1.0, 0.02, 200 + R)
    C = np.eye(3) * 0.15 ** 2
    K, N, seed = 5, 14, 3 + R
    ref, z = oracle_full(f, sigma, C, K, seed, N, 3)
    fg = cuda(f)
    for tile_w, tile_h in ((32, 0), (32, 24), (16, 24), (0, 0)):
        got, o = P.bf_vec_ex(fg, sigma, C, K, seed, N=N, spatial="box3+runsum", tile_w=tile_w,
                             tile_h=tile_h, return_opts=True)
        say(f"  tile_w={o.tile_w_used} tile_h={o.tile_h_used} matrix cores={o.mfma_used}")
        assert o.tile_w_used == (32 if tile_w == 32 else 16)
        assert o.mfma_used == (1 if tile_w == 32 else 0)
        check(host(got), ref, f, z, TOL["fp32"])
