"""Accuracy against the number of terms (the paper's error-plot study, Section 4).

The MCSF estimator's variance falls as 1/K with the number K of Monte Carlo
terms (Proposition 2; each term is an independent draw), so its mean squared
error against the exact filter (eq. (MSE)) has log-log slope -1 in K while the
order-N bias (Proposition 1, about z^4 / 12N) stays negligible.  Both filters
run on the GPU: the MCSF through bf_vec_ex (FP32) and the direct filter of
eqs. (BF)/(normal) through bf_direct (itself held to the FP64 oracle in
test_gpu_parity).  N = 400 keeps the bias below the K = 256 variance.  The
per-realisation MSE has a heavy tail at small K (the normaliser comes close to
zero at a few pixels in some draws), so the location over realisations is the
median; a CPU run of the oracle with the same settings gives slopes -0.93 to
-1.12 over four blocks of 24 seeds.
"""

import numpy as np
import pytest

import paper_1605_02164_amd as P
from synth import voronoi_image

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_mse_against_direct_falls_as_one_over_K():
    print("case MSE vs K: 48x56x3 Voronoi [0,255], sigma_s=1.5, sigma_r=30, N=400, 24 seeds",
          flush=True)
    f = torch.from_numpy(voronoi_image(48, 56, 3, 6, 0.0, 255.0, 5.0, seed=7002)).cuda()
    C = 30.0 ** 2 * np.eye(3)
    ref = P.bf_direct(f, 1.5, C).double()
    Ks = [16, 32, 64, 128, 256]
    med = []
    out = torch.empty_like(f)
    for K in Ks:
        v = []
        for r in range(24):
            P.bf_vec_ex(f, 1.5, C, K, 500000 + r, out=out, N=400)
            v.append(float(torch.mean((out.double() - ref) ** 2)))
        med.append(float(np.median(v)))
    slope = float(np.polyfit(np.log(Ks), np.log(med), 1)[0])
    print("  median MSE:", ["%.3g" % m for m in med], "slope %.3f" % slope, flush=True)
    assert -1.2 <= slope <= -0.8, slope
    assert all(a > b for a, b in zip(med, med[1:]))
