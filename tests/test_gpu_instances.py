"""Every compiled instance of the fused kernel against the FP64 oracle.

The fused kernel exists as separately compiled instances: one per window
radius with a fully unrolled specialisation (6, 9, 12, 15, 18, 21, 24, 30; the
workload and serving radii) and d in {3, 6}, each for FP32 channels and
FP16/BF16 storage, for 16- and (d = 3) 32-column strips, with the separable
passes on the vector ALUs or as banded products on the matrix cores, and with
or without the FP64 phase path; plus the runtime-radius instances.  Each
instance has its own unrolled window blocks, matrix-core k-block counts and
ring wrap constants, so each is compared here with the oracle's separable
filter (O3, Algorithm 1 in FP64) over a whole image of several strips in both
directions with ragged edges:

* bf_vec_ex at the instance's strip width, with and without the matrix-core
  passes (bf_opts.valu_only), against O3: FP32 within 1e-4 of each channel's
  range (1e-5/z where the normaliser z is small, as in test_gpu_parity), FP16
  and BF16 within the storage-rounding bound of test_gpu_parity;
* a plan with the same options runs the instance with the FP64 phase path
  (a plan's graph is captured before the image range is known) and must
  equal the bf_vec_ex result bit for bit (lanes below 2^8 turns run the same
  operations in both instances).
"""

import numpy as np
import pytest

import paper_1605_02164_amd as P
from oracle import mcsf as O
from synth import voronoi_image, random_spd
from tests.test_gpu_parity import assert_close, lp_errors, LP_BOUND, cuda, host, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPECIALISED = (6, 9, 12, 15, 18, 21, 24, 30)


def _mf_expected(prec, R, TW, valu):
    """The launcher's matrix-core rule: 16-bit storage at either width, FP32
    horizontal pass of 32-column strips from R = 12, compile-time radii only."""
    if valu or R not in SPECIALISED:
        return 0
    if prec in ("fp16", "bf16"):
        return 1
    return 1 if (TW == 32 and R >= 12) else 0


def _cases():
    out = []
    for R in SPECIALISED:
        for d in (3, 6):
            for prec in ("fp32", "fp16", "bf16"):
                for TW in ((16, 32) if d == 3 else (16,)):
                    valus = (0, 1) if _mf_expected(prec, R, TW, 0) else (0,)
                    for valu in valus:
                        out.append((d, R, prec, TW, valu))
    for R in (4, 10, 27, 40):          # runtime-radius instances
        for d in (3, 6):
            for prec in ("fp32", "fp16", "bf16"):
                out.append((d, R, prec, 16, 0))
    return out


CASES = _cases()


def _image(d, R, TW):
    # several strips across (ragged last strip) and down (tile_h = 24), and
    # an image narrower / shorter than the window at the larger radii
    H = 2 * R + 45
    W = 3 * TW + 7
    f = voronoi_image(H, W, d, 5, 0.0, 1.0, 0.02, seed=100 * d + R + TW)
    C = np.eye(d) * 0.15 ** 2 if d == 3 else random_spd(d, -2.0, -1.0, R)
    return f, C


@pytest.mark.parametrize("d,R,prec,TW,valu", CASES,
                         ids=[f"d{c[0]}-R{c[1]}-{c[2]}-w{c[3]}-{'valu' if c[4] else 'auto'}"
                              for c in CASES])
def test_instance_against_oracle(d, R, prec, TW, valu):
    say(f"case instance d={d} R={R} {prec} tile_w={TW} valu_only={valu}")
    f, C = _image(d, R, TW)
    sigma = R / 3.0
    assert O.window_radius(sigma) == R
    K, seed, TH = 3, 1000 + R, 24
    fg = cuda(f)
    got, o = P.bf_vec_ex(fg, sigma, C, K, seed, precision=prec, tile_h=TH, tile_w=TW,
                         valu_only=bool(valu), return_opts=True)
    got = host(got)
    assert o.tile_w_used == TW and o.tile_h_used == TH
    assert o.mfma_used == _mf_expected(prec, R, TW, valu)
    f64 = f.astype(np.float64)
    W_ = O.whiten(C)
    N = O.choose_order(f64, W_)
    assert o.N_used == N
    _, w = O.sample_terms(C, N, K, seed, W=W_)
    ref, _, Z = O.mcsf_separable(f64, sigma, w)
    z = Z / (K * O.spatial_taps(sigma).sum() ** 2)
    if prec == "fp32":
        assert_close(got, ref, f, z)
    else:
        mx, mean, sc = lp_errors(got, ref, f, z)
        say(f"  {prec}: max err {mx:.3e} mean err {mean:.3e} conditioning-scaled {sc:.3e}")
        assert sc <= LP_BOUND[prec]
    # the FP64-phase-path instance (plans) gives the same bits
    with P.Plan(*f.shape, sigma, C, K, seed, N=N, precision=prec, tile_h=TH, tile_w=TW,
                valu_only=bool(valu)) as plan:
        assert plan.tile_w_used == TW and plan.mfma_used == o.mfma_used
        pout = host(plan(fg))
    assert np.array_equal(pout, got)
