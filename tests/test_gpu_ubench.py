"""GPU test of the device probes (bf_ubench): each returns a rate of the
right magnitude for an MI355X (broad bounds around the published peaks:
157.3 TFLOP/s FP32 matrix and vector, 2.5 PFLOP/s FP16 matrix, 8 TB/s HBM),
and the matrix probe shows the dependent-chain effect: with one wave per
SIMD, one chain per wave runs well below two chains; with two waves per
SIMD one chain each already comes close to the rate.  The overlap probes
return a fraction of at most about 1 (1: matrix and vector work on one SIMD
run side by side; 0: their times add)."""

import pytest

import paper_1605_02164_amd as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_probe_rates():
    print("case ubench probes", flush=True)
    r = {"mfma_f32_1": P.bf_ubench("mfma_f32", 1), "mfma_f32_2": P.bf_ubench("mfma_f32", 2),
         "solo_1": P.bf_ubench("mfma_f32_solo", 1), "solo_2": P.bf_ubench("mfma_f32_solo", 2),
         "mfma_f16_2": P.bf_ubench("mfma_f16", 2), "valu_f32_4": P.bf_ubench("valu_f32", 4),
         "trans_f32": P.bf_ubench("trans_f32"), "lds_read": P.bf_ubench("lds_read"),
         "hbm_copy": P.bf_ubench("hbm_copy", 512),
         "overlap_f32": P.bf_ubench("overlap_f32"), "overlap_f16": P.bf_ubench("overlap_f16")}
    print("  ", {k: round(v, 2) for k, v in r.items()}, flush=True)
    assert 60 <= r["mfma_f32_2"] <= 170
    assert r["solo_1"] < 0.8 * r["solo_2"]
    assert r["mfma_f32_1"] > 0.8 * r["mfma_f32_2"]
    assert 400 <= r["mfma_f16_2"] <= 2600
    assert 20 <= r["valu_f32_4"] <= 170
    assert 1 <= r["trans_f32"] <= 100
    assert 10 <= r["lds_read"] <= 1000
    assert 1 <= r["hbm_copy"] <= 8.5
    assert -2.0 <= r["overlap_f32"] <= 1.1
    assert -2.0 <= r["overlap_f16"] <= 1.1
