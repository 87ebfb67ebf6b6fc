"""The allocation-free entry point bf_vec_static against bf_vec_ex.

bf_vec_static runs the same kernels as bf_vec_ex with every device buffer
(min/max partials, term table, accumulators) in the library's static scratch
array, so its output must equal bf_vec_ex's bit for bit; the small case is
also held to the FP64 oracle's 1e-4 bound.  Two calls in a row (the second
smaller, with another d, window and precision) show that the scratch keeps
no state that matters between calls; a call beyond the scratch is refused
before any kernel runs, and the next call still works.
"""

import ctypes

import numpy as np
import pytest

import paper_1605_02164_amd as P
from paper_1605_02164_amd import bfvec as B
from oracle import mcsf as O
from synth import voronoi_image, random_spd
from tests.helpers import rel_err_per_channel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_static_scratch_equals_bf_vec_ex_twice_then_smaller():
    print("case bf_vec_static: 512x640x3 fp32 sigma_s=5 K=32, then 90x77x6 fp16 sigma_s=2 K=12",
          flush=True)
    cases = [
        (voronoi_image(512, 640, 3, 40, 0.0, 1.0, 0.02, seed=31), 5.0, 0.1 ** 2 * np.eye(3), 32,
         dict(precision="fp32")),
        (voronoi_image(90, 77, 6, 6, 0.0, 1.0, 0.02, seed=32), 2.0, random_spd(6, -2.0, -1.0, 3),
         12, dict(precision="fp16", dedup=True)),
    ]
    for f, sigma, C, K, kw in cases:
        fg = _cuda(f)
        ref, o_ref = P.bf_vec_ex(fg, sigma, C, K, 7, return_opts=True, **kw)
        got, o = P.bf_vec_static(fg, sigma, C, K, 7, return_opts=True, **kw)
        ref, got = _host(ref), _host(got)
        assert (o.N_used, o.K_used, o.tile_h_used, o.tile_w_used) == \
            (o_ref.N_used, o_ref.K_used, o_ref.tile_h_used, o_ref.tile_w_used)
        assert np.array_equal(got, ref), np.abs(got - ref).max()
    # the smaller FP32 case against the oracle as well
    f, sigma, C, K = voronoi_image(40, 52, 3, 5, 0.0, 1.0, 0.02, seed=33), 2.0, 0.1 ** 2 * np.eye(3), 16
    got, N = P.bf_vec_static(_cuda(f), sigma, C, K, 9)
    ref, Nref, _, _ = O.mcsf(f.astype(np.float64), sigma, C, K, 9)
    assert N == Nref
    assert np.all(rel_err_per_channel(_host(got), ref, f) <= 1e-4)


def test_static_scratch_limit_refused_before_any_kernel():
    print("case bf_vec_static: 2048^2 x 3 exceeds the scratch", flush=True)
    fg = torch.rand(2048, 2048, 3, device="cuda")
    out = torch.full_like(fg, -7.0)
    with pytest.raises(P.BfError) as e:
        P.bf_vec_static(fg, 3.0, 0.1 ** 2 * np.eye(3), 8, 1, out=out)
    assert e.value.code == B.BF_EUNSUPPORTED and "static scratch" in str(e.value)
    assert bool((out == -7.0).all())          # nothing written
    assert B.BF_STATIC_SCRATCH_BYTES == 64 << 20
    # time_kernel needs events: refused
    o = B.make_opts(time_kernel=True)
    Ch = np.ascontiguousarray(0.01 * np.eye(3))
    small = fg[:64, :64].contiguous()
    rc = B.lib().bf_vec_static(small.data_ptr(), 64, 64, 3, 1.0, Ch.ctypes.data_as(ctypes.c_void_p),
                               4, 1, out.data_ptr(), ctypes.byref(o))
    assert rc == B.BF_EINVAL
    # a call after the refusals still works
    got, _ = P.bf_vec_static(small, 1.0, 0.1 ** 2 * np.eye(3), 4, 1)
    ref, _ = P.bf_vec_ex(small, 1.0, 0.1 ** 2 * np.eye(3), 4, 1)
    assert torch.equal(got, ref)
