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
  passes (bf_opts.valu_only), against O3.  The accumulated numerator and
  normaliser (eqs. (numerator), (denom); the num_out / z_out outputs) are
  linear in the filtered channels, so their error does not depend on the
  conditioning of the ratio: every pixel within 1e-5 (FP32) or 4u (16-bit
  storage, u the unit roundoff, two roundings of each stored value) of their
  scale K sum(omega) (times max |f| for the numerator).  The output num/Z:
  FP32 within 1e-4 of each channel's range where z = Z / (K sum omega) >=
  0.1 and within 1e-5/z for 0.01 <= z < 0.1 (test_gpu_parity's bound for
  ill-conditioned pixels, continued up to where it meets 1e-4: with a few
  terms z comes close to zero at some pixels, and the ratio amplifies the
  FP32 rounding of num, Z and the term table by 1/z; below z = 0.01 the
  num and Z checks stand alone), FP16 and BF16 within the storage-rounding
  bound 4u/z of test_gpu_parity (z >= 0.01);
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
from tests.helpers import rel_err_per_channel
from tests.test_gpu_parity import lp_errors, LP_UNIT, cuda, host, say

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


def _span(f):
    f2 = np.asarray(f, np.float64).reshape(-1, f.shape[-1])
    s = f2.max(0) - f2.min(0)
    s[s == 0] = 1.0
    return s


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
    K, seed, TH = 4, 1000 + R, 24
    fg = cuda(f)
    num = torch.empty_like(fg)
    zo = torch.empty(fg.shape[:2], device="cuda", dtype=torch.float32)
    got, o = P.bf_vec_ex(fg, sigma, C, K, seed, precision=prec, tile_h=TH, tile_w=TW,
                         valu_only=bool(valu), num_out=num, z_out=zo, return_opts=True)
    got, num, zo = host(got), host(num), host(zo)
    # the pipelined FP32 matrix-core instances (R >= 21) take pairs of 8-row
    # steps: strip heights are rounded up to 16 rows there
    pipe = prec == "fp32" and _mf_expected(prec, R, TW, valu) and R >= 21
    assert o.tile_w_used == TW and o.tile_h_used == (32 if pipe else TH)
    assert o.mfma_used == _mf_expected(prec, R, TW, valu)
    f64 = f.astype(np.float64)
    W_ = O.whiten(C)
    N = O.choose_order(f64, W_)
    assert o.N_used == N
    _, w = O.sample_terms(C, N, K, seed, W=W_)
    ref, rnum, rZ = O.mcsf_separable(f64, sigma, w)
    scale = K * O.spatial_taps(sigma).sum() ** 2
    z = rZ / scale
    eps = 1e-5 if prec == "fp32" else 4.0 * LP_UNIT[prec]
    ez = np.max(np.abs(zo - rZ)) / scale
    en = np.max(np.abs(num - rnum)) / (scale * np.abs(f64).max())
    say(f"  N={N} Z err {ez:.3e}, num err {en:.3e} (of their scale; bound {eps:.1e});"
        f" min z {z.min():.3f}")
    assert ez <= eps and en <= eps
    if prec == "fp32":
        good = z >= 0.1
        err = rel_err_per_channel(got[good], ref[good], f)
        say(f"  output rel_err={err} (z >= 0.1), {int((~good).sum())} pixels below")
        assert np.all(err <= 1e-4), err
        mid = ~good & (z >= 0.01)
        if mid.any():
            e = np.abs(got[mid] - ref[mid]) / _span(f)
            assert np.all(e * z[mid][:, None] <= 1e-5)
    else:
        mx, mean, rb = lp_errors(got, ref, f, z, prec)
        say(f"  {prec}: max err {mx:.3e} mean err {mean:.3e}, {rb:.3f} of the bound")
        assert rb <= 1.0
    # the FP64-phase-path instance (plans) gives the same bits
    with P.Plan(*f.shape, sigma, C, K, seed, N=N, precision=prec, tile_h=TH, tile_w=TW,
                valu_only=bool(valu)) as plan:
        assert plan.tile_w_used == TW and plan.mfma_used == o.mfma_used
        pout = host(plan(fg))
    assert np.array_equal(pout, got)
