"""GPU tests of fixed-shape plans (bf_plan_* through the C ABI).

A plan's execution is one HIP graph launch of the same kernels bf_vec_ex
runs, with the centre read on the device from the min/max result instead of
passed from the host.  Its output must therefore be bitwise equal to
bf_vec_ex with the same arguments, on every replay of a graph: replays are
interleaved with eager device work and with executions on other buffers, and
each is checked.  One small case is also checked against the FP64 oracle.
"""

import sys

import numpy as np
import pytest

import paper_1605_02164_amd as P
from paper_1605_02164_amd import bfvec as B
from oracle import mcsf as O
from synth import workload, voronoi_image, random_spd
from tests.helpers import rel_err_per_channel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("precision,center,dedup", [
    ("fp32", True, False), ("fp32", False, False), ("fp16", True, False),
    ("bf16", True, True), ("fp32", True, True),
])
def test_plan_replays_match_bf_vec_ex(precision, center, dedup):
    say(f"case plan 96x136x3 sigma_s=3 K=24 N=16 {precision} center={center} dedup={dedup}")
    H, W, d, sigma, K, N, seed = 96, 136, 3, 3.0, 24, 16, 11
    C = np.diag([0.12, 0.1, 0.15]) ** 2
    imgs = [cuda(voronoi_image(H, W, d, 12, -0.3 + 0.2 * i, 1.0 + 0.5 * i, 0.02, 40 + i))
            for i in range(3)]
    refs = [host(P.bf_vec_ex(g, sigma, C, K, seed, N=N, precision=precision, center=center,
                             dedup=dedup)[0]) for g in imgs]
    outs = [torch.full_like(imgs[0], float("nan")) for _ in range(3)]
    with B.Plan(H, W, d, sigma, C, K, seed, N, precision=precision, center=center,
                dedup=dedup) as plan:
        assert plan.N_used == N
        assert (plan.K_used <= K) if dedup else (plan.K_used == K)
        # image i -> out i, three rounds; eager work between the replays
        for rnd in range(3):
            for i in (0, 1, 2):
                outs[i].fill_(float("nan"))
                plan(imgs[i], outs[i])
                junk = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
                assert np.array_equal(host(outs[i]), refs[i]), (rnd, i)
                del junk
        # one image into two other outputs (new graphs), then the first pair again
        plan(imgs[0], outs[1])
        plan(imgs[0], outs[2])
        plan(imgs[2], outs[0])
        assert np.array_equal(host(outs[1]), refs[0])
        assert np.array_equal(host(outs[2]), refs[0])
        assert np.array_equal(host(outs[0]), refs[2])


def test_plan_graph_cache_eviction():
    say("case plan with more (f, out) pairs than cached graphs")
    H, W, d, sigma, K, N = 40, 56, 3, 2.0, 8, 12
    C = np.eye(3) * 0.15 ** 2
    imgs = [cuda(voronoi_image(H, W, d, 6, 0.0, 1.0, 0.02, 60 + i)) for i in range(6)]
    refs = [host(P.bf_vec_ex(g, sigma, C, K, 3, N=N)[0]) for g in imgs]
    outs = [torch.empty_like(imgs[0]) for _ in range(6)]
    with B.Plan(H, W, d, sigma, C, K, 3, N) as plan:
        for rnd in range(2):
            for i in range(6):
                plan(imgs[i], outs[i])
            for i in range(6):
                assert np.array_equal(host(outs[i]), refs[i]), (rnd, i)


def test_plan_on_a_side_stream_and_shape_check():
    say("case plan on a side stream; wrong shape rejected")
    H, W, d, sigma, K, N = 33, 45, 2, 1.5, 6, 14
    C = random_spd(2, -2.0, -1.0, 5)
    f = cuda(voronoi_image(H, W, d, 5, 0.0, 1.0, 0.02, 8))
    ref = host(P.bf_vec_ex(f, sigma, C, K, 9, N=N)[0])
    s = torch.cuda.Stream()
    out = torch.empty_like(f)
    with B.Plan(H, W, d, sigma, C, K, 9, N) as plan:
        with torch.cuda.stream(s):
            plan(f, out, stream=s)
        s.synchronize()
        assert np.array_equal(host(out), ref)
        with pytest.raises(ValueError):
            plan(cuda(np.zeros((H + 1, W, d))))


def test_plan_matches_oracle():
    say("case plan voronoi128 recipe 64x80 against the FP64 oracle")
    f, C, p = workload("voronoi128_d3_s2_K64", H=64, W=80)
    K, N, seed = 16, 10, 21
    with B.Plan(64, 80, 3, p["sigma_s"], C, K, seed, N) as plan:
        got = host(plan(cuda(f))).astype(np.float64)
    Wm = O.whiten(C)
    _, w = O.sample_terms(C, N, K, seed, W=Wm)
    ref, _, Z = O.mcsf_separable(np.asarray(f, np.float64), p["sigma_s"], w)
    z = Z / (K * O.spatial_taps(p["sigma_s"]).sum() ** 2)
    ok = z >= 1e-2
    err = rel_err_per_channel(got[ok], ref[ok], f)
    say(f"  rel_err={err} ill-conditioned={int((~ok).sum())}")
    assert np.all(err <= 1e-4), err
