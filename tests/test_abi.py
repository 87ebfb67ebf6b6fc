"""CPU tests of the C ABI: the library loads, exports every declared symbol,
and its host-side logic (whitening, draws, order rule, validation) agrees with
the oracle.  No device work is started here."""

import ctypes
import math

import numpy as np
import pytest

import paper_1605_02164_amd as P
from paper_1605_02164_amd import bfvec as B
from oracle import mcsf as O
from synth import random_spd
from tests.helpers import header_functions


def test_library_exports_every_declared_symbol():
    L = P.lib()
    declared = header_functions()
    assert set(declared) == set(P.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name
    assert P.version() >= 10000


def test_opts_struct_layout(tmp_path):
    # the ctypes mirror of bf_opts must match the C layout of include/bfvec.h
    import subprocess
    from tests.helpers import ROOT
    fields = [name for name, _ in B.bf_opts._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "bfvec.h"\n'
                   "int main(void){printf(\"%zu\", sizeof(bf_opts));" +
                   "".join(f'printf(" %zu", offsetof(bf_opts, {n}));' for n in fields) +
                   "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", f"{ROOT}/include", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(B.bf_opts)
    assert got[1:] == [getattr(B.bf_opts, n).offset for n in fields]
    o = B.bf_opts()
    B.lib().bf_opts_init(ctypes.byref(o))
    assert (o.N, o.precision, o.center, o.tile_h) == (0, 0, 1, 0)


@pytest.mark.parametrize("d,seed", [(1, 1), (3, 2), (6, 3), (8, 4)])
def test_whitening_matches_oracle(d, seed):
    C = random_spd(d, -3, -1, seed)
    W = P.bf_whiten(C)
    assert np.max(np.abs(W - O.whiten(C))) <= 1e-13 * np.max(np.abs(W))
    Ci = np.linalg.inv(C)
    assert np.max(np.abs(W.T @ W - Ci)) <= 1e-12 * np.max(np.abs(Ci))


def test_whitening_block_and_diagonal():
    C = np.array([[100.0, 0, 0], [0, 25, 12.5], [0, 12.5, 25]])
    assert np.max(np.abs(P.bf_whiten(C) - O.whiten(C))) < 1e-16
    Cd = np.diag([0.0064, 0.0064, 0.0064])
    assert np.array_equal(P.bf_whiten(Cd), O.whiten(Cd))


@pytest.mark.parametrize("d,N,K,seed", [(3, 33, 256, 2003), (3, 309, 128, 2002),
                                        (6, 40, 64, 2004), (1, 1, 50, 0),
                                        (2, 65, 17, 2**63 + 12345)])
def test_draws_match_oracle(d, N, K, seed):
    C = random_spd(d, -3, -1, d + 10) if d > 1 else np.array([[0.04]])
    Y, w = P.bf_sample_terms(C, N, K, seed)
    Yo, wo = O.sample_terms(C, N, K, seed)
    assert np.array_equal(Y, Yo)
    assert np.max(np.abs(w - wo)) <= 1e-13 * max(1.0, np.max(np.abs(wo)))


@pytest.mark.parametrize("mode,omode", [("eig", O.WHITEN_EIG), ("chol", O.WHITEN_CHOL),
                                        ("sym", O.WHITEN_SYM)])
def test_order_rule_matches_oracle(mode, omode):
    rng = np.random.default_rng(5)
    for d in (1, 3, 6):
        C = random_spd(d, -3, -1, d) if d > 1 else np.array([[0.01]])
        W = O.whiten(C, omode)
        f = rng.uniform(-0.3, 1.2, size=(5, 7, d)).astype(np.float32)
        lo, hi = f.reshape(-1, d).min(0), f.reshape(-1, d).max(0)
        assert P.bf_choose_N(C, lo, hi, whiten=mode) == O.choose_order(f, W)


def test_order_rule_limit_and_arguments():
    C = np.eye(1) * 1e-6
    with pytest.raises(P.BfError) as e:
        P.bf_choose_N(C, [0.0], [1.0])
    assert e.value.code == B.BF_EUNSUPPORTED
    with pytest.raises(P.BfError) as e:          # lo above hi
        P.bf_choose_N(np.eye(2), [0.0, 1.0], [1.0, 0.5])
    assert e.value.code == B.BF_EINVAL
    with pytest.raises(P.BfError) as e:          # not SPD
        P.bf_choose_N(np.array([[1.0, 2.0], [2.0, 1.0]]), [0.0, 0.0], [1.0, 1.0])
    assert e.value.code == B.BF_ENOTSPD
    with pytest.raises(P.BfError) as e:          # unknown whitening mode
        P.bf_choose_N(np.eye(2), [0.0, 0.0], [1.0, 1.0], whiten=5)
    assert e.value.code == B.BF_EINVAL


@pytest.mark.parametrize("mode,omode", [("chol", O.WHITEN_CHOL), ("sym", O.WHITEN_SYM)])
@pytest.mark.parametrize("d,N,K,seed", [(3, 309, 128, 2002), (6, 40, 64, 2004)])
def test_draws_match_oracle_every_whitening(mode, omode, d, N, K, seed):
    # the C ABI reproduces the draws bf_vec_ex runs with opts.whiten: the same
    # Y (whitening does not enter the bits) and w = W^T Y / sqrt(N) with the
    # mode's W
    C = (np.array([[100.0, 0, 0], [0, 25, 12.5], [0, 12.5, 25]]) if d == 3
         else random_spd(d, -3, -1, d + 10))
    Y, w = P.bf_sample_terms(C, N, K, seed, whiten=mode)
    Yo, wo = O.sample_terms(C, N, K, seed, W=O.whiten(C, omode))
    assert np.array_equal(Y, Yo)
    assert np.max(np.abs(w - wo)) <= 1e-13 * max(1.0, np.max(np.abs(wo)))
    _, we = P.bf_sample_terms(C, N, K, seed)       # non-diagonal C: the modes differ
    assert np.max(np.abs(we - w)) > 1e-6


def _call_vec(f=0x1000, H=8, W=8, d=3, sigma=1.0, C=None, K=4, out=0x100000):
    C = np.eye(d) * 0.01 if C is None else C
    Ch = np.ascontiguousarray(C, dtype=np.float64)
    rc = B.lib().bf_vec(f, H, W, d, sigma, Ch.ctypes.data_as(ctypes.c_void_p) if C is not False else None,
                        K, 1, out)
    return rc, B.lib().bf_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(H=0), B.BF_EINVAL), (dict(W=-1), B.BF_EINVAL), (dict(d=0), B.BF_EINVAL),
    (dict(d=9, C=np.eye(9)), B.BF_EINVAL), (dict(K=0), B.BF_EINVAL),
    (dict(sigma=-1.0), B.BF_EINVAL), (dict(sigma=float("nan")), B.BF_EINVAL),
    (dict(sigma=40.0), B.BF_EINVAL), (dict(f=0), B.BF_EINVAL), (dict(out=0), B.BF_EINVAL),
    (dict(out=0x1000 + 16), B.BF_EINVAL),                # out overlaps f
    (dict(C=np.array([[1.0, 0.5, 0], [0.4, 1, 0], [0, 0, 1]])), B.BF_ENOTSPD),
    (dict(C=np.array([[1.0, 2, 0], [2, 1, 0], [0, 0, 1]])), B.BF_ENOTSPD),
    (dict(C=np.diag([1.0, 0.0, 1.0])), B.BF_ENOTSPD),
    (dict(sigma=14.0), B.BF_EUNSUPPORTED),               # R = 42 > 40
    # (H+16)(W+16)(d+1) above 2^30 floats: 32-bit byte offsets would overflow
    (dict(H=20000, W=20000, out=0x1000 + 20000 * 20000 * 12 + 4096), B.BF_EUNSUPPORTED),
])
def test_argument_errors_before_device_work(kw, code):
    rc, msg = _call_vec(**kw)
    assert rc == code, msg
    assert msg


def test_invalid_options_rejected():
    o = B.make_opts()
    o.precision = 7
    Ch = np.eye(3) * 0.01
    rc = B.lib().bf_vec_ex(0x1000, 8, 8, 3, 1.0, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                           0x100000, ctypes.byref(o))
    assert rc == B.BF_EINVAL
    o = B.make_opts()
    o.N = -2
    rc = B.lib().bf_vec_ex(0x1000, 8, 8, 3, 1.0, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                           0x100000, ctypes.byref(o))
    assert rc == B.BF_EINVAL


@pytest.mark.parametrize("kw", [
    dict(sigma=2.0),                      # R = 6: no split instance
    dict(sigma=5.0),                      # R = 15
    dict(d=6, C=np.eye(6) * 0.01),        # d = 6
    dict(W=24),                           # narrower than a 32-column strip
    dict(tile_w=16),
    dict(valu_only=True),
])
def test_split_precision_refused_before_device_work(kw):
    # BF_FP32_SPLIT runs only the pipelined d = 3 instances at R = 18, 21, 24, 30
    d = kw.pop("d", 3)
    C = kw.pop("C", np.eye(3) * 0.01)
    sigma = kw.pop("sigma", 10.0)
    W = kw.pop("W", 64)
    o = B.make_opts(precision="fp32_split", **kw)
    Ch = np.ascontiguousarray(C, dtype=np.float64)
    rc = B.lib().bf_vec_ex(0x1000, 64, W, d, sigma, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                           0x4000000, ctypes.byref(o))
    assert rc == B.BF_EUNSUPPORTED, B.lib().bf_last_error().decode()
    assert "SPLIT" in B.lib().bf_last_error().decode()


def test_term_table_validation():
    w = np.array([[1.0, float("inf"), 0.0]])
    rc = B.lib().bf_vec_terms(0x1000, 4, 4, 3, 1.0, w.ctypes.data_as(ctypes.c_void_p), None, 1,
                              0x100000, None)
    assert rc == B.BF_EINVAL
    w = np.ones((2, 3))
    wt = np.array([1.0, -1.0])
    rc = B.lib().bf_vec_terms(0x1000, 4, 4, 3, 1.0, w.ctypes.data_as(ctypes.c_void_p),
                              wt.ctypes.data_as(ctypes.c_void_p), 2, 0x100000, None)
    assert rc == B.BF_EINVAL


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    # a missing library is an error, never a silent CPU path
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        B.lib()


def test_autotune_validation_before_device_work():
    import ctypes
    L = P.lib()
    th = ctypes.c_int(0)
    fake = ctypes.c_void_p(0x1000)
    assert L.bf_autotune(fake, 16, 16, 9, 2.0, 0, None, ctypes.byref(th), None) == B.BF_EINVAL
    assert L.bf_autotune(fake, 16, 16, 3, 2.0, 7, None, ctypes.byref(th), None) == B.BF_EINVAL
    assert L.bf_autotune(fake, 16, 16, 3, 14.0, 0, None, ctypes.byref(th), None) == B.BF_EUNSUPPORTED
    assert L.bf_autotune(None, 16, 16, 3, 2.0, 0, None, ctypes.byref(th), None) == B.BF_EINVAL


def test_plan_validation_before_device_work():
    L = P.lib()
    C = np.eye(3) * 0.01
    Cp = C.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p(0x1234)

    def create(H=16, W=16, d=3, sigma=2.0, Cp=Cp, K=4, **kw):
        o = B.make_opts(**{"N": 12, **kw})
        return L.bf_plan_create(H, W, d, sigma, Cp, K, 1, ctypes.byref(o), ctypes.byref(h))

    assert create(N=0) == B.BF_EINVAL                     # the order must be explicit
    assert h.value is None                                # *plan is cleared on failure
    assert create(H=0) == B.BF_EINVAL
    assert create(d=9) == B.BF_EINVAL
    assert create(K=0) == B.BF_EINVAL
    assert create(sigma=float("nan")) == B.BF_EINVAL
    assert create(Cp=None) == B.BF_EINVAL
    assert create(precision=7) == B.BF_EINVAL
    assert create(precision="fp32_split", sigma=2.0, H=64, W=64) == B.BF_EUNSUPPORTED   # R = 6
    assert create(precision="fp32_split", sigma=10.0, H=64, W=64,
                  valu_only=True) == B.BF_EUNSUPPORTED
    assert create(time_kernel=True) == B.BF_EINVAL
    bad = np.array([[1.0, 2, 0], [2, 1, 0], [0, 0, 1]])
    assert create(Cp=bad.ctypes.data_as(ctypes.c_void_p)) == B.BF_ENOTSPD
    assert create(sigma=14.0) == B.BF_EUNSUPPORTED
    assert L.bf_plan_create(16, 16, 3, 2.0, Cp, 4, 1, None, None) == B.BF_EINVAL
    assert L.bf_plan_execute(None, 0x1000, 0x100000, None) == B.BF_EINVAL
    assert L.bf_plan_destroy(None) == B.BF_OK


def test_spatial_option_validation_before_device_work():
    L = P.lib()
    Ch = np.eye(3) * 0.01

    def vec(spatial, precision="fp32"):
        o = B.make_opts(precision=precision)
        o.spatial = spatial
        return L.bf_vec_ex(0x1000, 8, 8, 3, 1.0, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                           0x100000, ctypes.byref(o))

    assert vec(4) == B.BF_EINVAL                                   # not a filter
    assert vec(B.BF_SPATIAL_RUNSUM) == B.BF_EINVAL                 # running sums need boxes
    assert vec(B.BF_SPATIAL_BOX3 | B.BF_SPATIAL_RUNSUM, "fp16") == B.BF_EUNSUPPORTED
    assert vec(B.BF_SPATIAL_HAT | 32) == B.BF_EINVAL
    assert B._spatial("box3+runsum") == 3 | B.BF_SPATIAL_RUNSUM
    with pytest.raises(ValueError):
        B._spatial("box3+fast")


def test_strip_width_validation_before_device_work():
    L = P.lib()

    def vec(tile_w, d=3, W=64, sigma=3.0, precision="fp32", spatial="gauss"):
        o = B.make_opts(precision=precision, spatial=spatial, tile_w=tile_w)
        Ch = np.eye(d) * 0.01
        return L.bf_vec_ex(0x1000, 40, W, d, sigma, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                           0x10000000, ctypes.byref(o))

    assert vec(7) == B.BF_EINVAL                                   # not 0, 16 or 32
    assert vec(-16) == B.BF_EINVAL
    assert vec(32, d=4) == B.BF_EUNSUPPORTED                       # d = 3 only
    assert vec(32, W=31) == B.BF_EUNSUPPORTED                      # narrower than a strip
    assert vec(32, sigma=2.5) == B.BF_EUNSUPPORTED                 # R = 8: runtime radius
    assert vec(32, spatial="box+runsum") == B.BF_EUNSUPPORTED      # running-sum box: 16 columns
    assert vec(32, spatial="hat+runsum") == B.BF_EUNSUPPORTED      # (three boxes have both)
    assert b"32-column" in L.bf_last_error()


@pytest.mark.parametrize("mode", ["chol", "sym"])
@pytest.mark.parametrize("d,seed", [(2, 11), (3, 12), (6, 13), (8, 14)])
def test_whitening_modes_match_oracle(mode, d, seed):
    C = random_spd(d, -3, -1, seed)
    W = P.bf_whiten(C, mode)
    ref = O.whiten(C, {"chol": O.WHITEN_CHOL, "sym": O.WHITEN_SYM}[mode])
    assert np.max(np.abs(W - ref)) <= 1e-12 * np.max(np.abs(ref))
    if mode == "chol":
        assert np.array_equal(W, np.tril(W))


def test_whitening_mode_validation():
    L = P.lib()
    C = np.eye(3) * 0.01
    W = np.empty((3, 3))
    assert L.bf_whiten_mode(3, C.ctypes.data_as(ctypes.c_void_p), 3,
                            W.ctypes.data_as(ctypes.c_void_p)) == B.BF_EINVAL
    bad = np.array([[1.0, 2, 0], [2, 1, 0], [0, 0, 1]])
    for mode in (0, 1, 2):
        assert L.bf_whiten_mode(3, bad.ctypes.data_as(ctypes.c_void_p), mode,
                                W.ctypes.data_as(ctypes.c_void_p)) == B.BF_ENOTSPD
    o = B.make_opts()
    o.whiten = 5
    rc = L.bf_vec_ex(0x1000, 8, 8, 3, 1.0, C.ctypes.data_as(ctypes.c_void_p), 4, 1, 0x100000,
                     ctypes.byref(o))
    assert rc == B.BF_EINVAL


def test_strip_height_bounded_by_accumulator_offsets():
    # A requested strip height is clamped to one strip (the image height), so
    # a huge value cannot inflate the padded accumulators; a height that
    # splits the image into two tall strips whose padding pushes
    # (d+1) x padded rows x padded columns past 2^30 floats is refused before
    # any device work (32-bit byte offsets in the kernels).
    H = W = 16000
    d = 3
    out = 0x1000 + H * W * d * 4 + 4096
    Ch = np.ascontiguousarray(np.eye(d) * 0.01)
    for tile_h in (8400, 12000):
        o = B.make_opts(tile_h=tile_h)
        rc = B.lib().bf_vec_ex(0x1000, H, W, d, 1.0, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                               out, ctypes.byref(o))
        assert rc == B.BF_EUNSUPPORTED, B.lib().bf_last_error().decode()
        assert "accumulators too large" in B.lib().bf_last_error().decode()
        o = B.make_opts(tile_h=tile_h, N=20)
        h = ctypes.c_void_p()
        rc = B.lib().bf_plan_create(H, W, d, 1.0, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                                    ctypes.byref(o), ctypes.byref(h))
        assert rc == B.BF_EUNSUPPORTED and not h.value


def test_valu_only_option_validated():
    o = B.make_opts()
    o.valu_only = 2
    Ch = np.eye(3) * 0.01
    rc = B.lib().bf_vec_ex(0x1000, 8, 8, 3, 1.0, Ch.ctypes.data_as(ctypes.c_void_p), 4, 1,
                           0x100000, ctypes.byref(o))
    assert rc == B.BF_EINVAL and "valu_only" in B.lib().bf_last_error().decode()


@pytest.mark.parametrize("probe,param", [(9, 1), (-1, 1), (0, 3), (1, 0), (2, 16), (5, 0),
                                         (5, 20000), (6, 3), (7, 1), (8, 2), (10, 0)])
def test_ubench_arguments_refused_before_device_work(probe, param):
    r = ctypes.c_double(1.0)
    assert B.lib().bf_ubench(probe, param, ctypes.byref(r)) == B.BF_EINVAL
    assert r.value == 0.0 and "bf_ubench" in B.lib().bf_last_error().decode()
    assert B.lib().bf_ubench(0, 1, None) == B.BF_EINVAL
