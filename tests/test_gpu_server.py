"""GPU tests of the continuous-batching server: every request's result equals
the same filter run alone through bf_vec_ex, bit for bit, when it is chunked
into many rounds and batched with requests of other sizes, dimensions,
windows and precisions; plus status, arrival and error behaviour."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1605_02164_amd as P  # noqa: E402
from paper_1605_02164_amd import bfvec as B  # noqa: E402
from synth import voronoi_image, feature_image, random_spd  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pools():
    f3 = voronoi_image(256, 300, 3, 24, 0.0, 1.0, 0.02, seed=71)
    f6 = feature_image(160, 176, 12, seed=72, smooth_sigma=8.0)
    return torch.from_numpy(f3).to(DEV), torch.from_numpy(f6).to(DEV)


# (pool, y0, x0, H, W, sigma_s, K, N, precision, center, cov)
MIX = [
    (3, 0, 0, 256, 300, 5.0, 32, 0, "fp16", True, "iso"),
    (3, 13, 7, 100, 61, 2.0, 17, 0, "fp32", True, "iso"),
    (3, 40, 200, 1, 37, 1.0, 5, 0, "fp16", True, "iso"),
    (3, 5, 9, 37, 1, 2.0, 9, 12, "bf16", False, "iso"),
    (6, 0, 0, 160, 176, 3.4, 24, 0, "fp16", True, "spd"),
    (6, 9, 21, 70, 50, 2.0, 11, 0, "fp32", False, "spd"),
    (3, 100, 33, 150, 211, 8.0, 20, 0, "fp16", True, "iso"),
    (3, 77, 41, 64, 48, 13.0, 3, 0, "fp32", True, "iso"),
    (6, 31, 3, 33, 17, 0.0, 4, 0, "bf16", True, "spd"),
    (3, 1, 1, 200, 250, 10.0, 12, 0, "fp16", True, "iso"),
]


def _cov(kind, d):
    return 0.05 ** 2 * np.eye(d) if kind == "iso" else random_spd(d, -2.5, -1.0, seed=5)


def _crop(pools, spec):
    pool, y0, x0, H, W = spec[:5]
    f = pools[0] if pool == 3 else pools[1]
    return f[y0:y0 + H, x0:x0 + W, :]


def _alone(fc, spec):
    _, _, _, _, _, s, K, N, prec, center, cov = spec
    d = fc.shape[2]
    out, n = P.bf_vec_ex(fc.contiguous(), s, _cov(cov, d), K, seed=1000 + K, N=N,
                         precision=prec, center=center)
    torch.cuda.synchronize()
    return out, n


def test_mix_matches_standalone_bitwise(pools):
    alone = []
    for spec in MIX:
        alone.append(_alone(_crop(pools, spec), spec))
    # a small quantum splits every request into many chunks and rounds
    with P.Server(arena_bytes=1 << 30, streams=3, depth=2, quantum_us=20.0) as srv:
        tickets = []
        for spec in MIX:
            fc = _crop(pools, spec)
            _, _, _, _, _, s, K, N, prec, center, cov = spec
            print("submit", spec, flush=True)
            t, out = srv.submit(fc, s, _cov(cov, fc.shape[2]), K, seed=1000 + K, N=N,
                                precision=prec, center=center)
            tickets.append((t, out))
        srv.drain(timeout=60.0)
        stats = srv.stats()
        for spec, (t, out), (ref, n_ref) in zip(MIX, tickets, alone):
            st = srv.poll(t)
            assert st["state"] == "done", (spec, st)
            assert st["N_used"] == n_ref, spec
            assert torch.equal(out, ref), (spec, float((out - ref).abs().max()))
        assert max(srv.poll(t)["chunks"] for t, _ in tickets) > 3
        assert stats["completed"] == len(MIX) and stats["failed"] == 0
        assert stats["rounds"] >= 4 and stats["launches"] >= stats["rounds"]


def test_batched_launches_share_requests(pools):
    # many small requests of one instance arriving together: with N given,
    # centring off and BF16 storage no reduction is needed (FP16 storage needs
    # the image range for its range check), so all 40 are ready at admission
    # and the first round packs them into 16 + 16 + 8 (whole K in one chunk)
    f = pools[0]
    C = 0.05 ** 2 * np.eye(3)
    specs = [(3 + 7 * i % 50, 2 + 11 * i % 60, 9 + i % 13, 20 + i % 17) for i in range(40)]
    with P.Server(arena_bytes=1 << 28, max_active=64, quantum_us=1e6) as srv:
        start = srv.clock() + 0.2   # all arrive together, after submission
        tickets = []
        for (y0, x0, H, W) in specs:
            t, out = srv.submit(f[y0:y0 + H, x0:x0 + W], 2.0, C, 6, seed=9, N=16, center=False,
                                arrival=start, precision="bf16")
            tickets.append((t, out))
        srv.drain(timeout=60.0)
        stats = srv.stats()
        assert stats["completed"] == 40
        assert stats["rounds"] == 1 and stats["launches"] == 3, stats
        for (y0, x0, H, W), (t, out) in list(zip(specs, tickets))[::7]:
            ref, _ = P.bf_vec_ex(f[y0:y0 + H, x0:x0 + W].contiguous(), 2.0, C, 6, seed=9, N=16,
                                 center=False, precision="bf16")
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            st = srv.poll(t)
            assert st["admitted"] >= start and st["done"] >= st["admitted"]
            srv.forget(t)
            with pytest.raises(B.BfError):
                srv.poll(t)


def test_arrival_in_future_and_cancel_on_close(pools):
    f = pools[0][:64, :64]
    C = 0.05 ** 2 * np.eye(3)
    srv = P.Server(arena_bytes=1 << 28)
    t0 = srv.clock()
    t1, _ = srv.submit(f, 2.0, C, 4, seed=3, arrival=t0 + 0.3)
    t2, _ = srv.submit(f, 2.0, C, 4, seed=3, arrival=t0 + 3600.0)
    st = srv.wait(t1, timeout=30.0)
    assert st["state"] == "done"
    assert st["admitted"] >= t0 + 0.3 - 1e-6
    assert srv.poll(t2)["state"] == "queued"
    with pytest.raises(B.BfError) as e:
        srv.wait(t2, timeout=0.05)
    assert e.value.code == B.BF_ETIMEDOUT
    srv.close()   # cancels the request that has not arrived


def test_submit_errors(pools):
    f = pools[0][:32, :32]
    C = 0.05 ** 2 * np.eye(3)
    with P.Server(arena_bytes=1 << 20) as srv:
        with pytest.raises(B.BfError) as e:
            srv.submit(f, 14.0, C, 4, seed=1)           # R = 42 > 40
        assert e.value.code == B.BF_EUNSUPPORTED
        with pytest.raises(B.BfError) as e:
            srv.submit(f, 2.0, -C, 4, seed=1)           # not SPD
        assert e.value.code == B.BF_ENOTSPD
        with pytest.raises(B.BfError) as e:
            srv.submit(f, 2.0, C, 0, seed=1)            # K = 0
        assert e.value.code == B.BF_EINVAL
        with pytest.raises(B.BfError) as e:
            srv.submit(pools[0], 2.0, C, 4, seed=1)   # 1.2 MB of accumulators > 1 MiB arena
        assert e.value.code == B.BF_ENOMEM
        with pytest.raises(ValueError):
            srv.submit(f, 2.0, C, 4, seed=1, out=torch.empty(31, 32, 3, device=DEV))
        overlap = pools[0].reshape(-1)[:32 * 32 * 3].view(32, 32, 3)
        with pytest.raises(B.BfError) as e:
            srv.submit(f, 2.0, C, 4, seed=1, out=overlap)   # out overlaps f
        assert e.value.code == B.BF_EINVAL
        t, _ = srv.submit(f, 2.0, C, 4, seed=1)
        assert srv.wait(t, timeout=30.0)["state"] == "done"
        assert srv.stats()["failed"] == 0


def test_nan_request_fails_alone(pools):
    f = pools[0][:40, :40].clone()
    f[5, 7, 1] = float("nan")
    good = pools[0][40:80, :40]
    C = 0.05 ** 2 * np.eye(3)
    with P.Server(arena_bytes=1 << 28) as srv:
        tb, _ = srv.submit(f, 2.0, C, 4, seed=1)
        tg, out = srv.submit(good, 2.0, C, 4, seed=1)
        sb = srv.wait(tb, timeout=30.0)
        sg = srv.wait(tg, timeout=30.0)
        assert sb["state"] == "failed" and sb["error"] == B.BF_EINVAL and "NaN" in sb["message"]
        assert sg["state"] == "done"
        ref, _ = P.bf_vec_ex(good.contiguous(), 2.0, C, 4, seed=1, precision="fp16")
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_merged_terms_match_standalone(pools):
    # requests with equal +-Y draws merged give the same bits as bf_vec_ex
    # with the same option
    C = 0.1 ** 2 * np.eye(3)
    crops = [pools[0][:96, :128], pools[0][50:163, 31:90]]
    with P.Server(arena_bytes=1 << 28, quantum_us=30.0) as srv:
        ts = []
        for i, fc in enumerate(crops):
            for prec in ("fp32", "fp16"):
                t, out = srv.submit(fc, 2.0, C, 64, seed=40 + i, precision=prec, dedup=True)
                ts.append((fc, prec, i, t, out))
        srv.drain(timeout=60.0)
        for fc, prec, i, t, out in ts:
            assert srv.poll(t)["state"] == "done"
            ref, o = P.bf_vec_ex(fc.contiguous(), 2.0, C, 64, seed=40 + i, precision=prec,
                                 dedup=True, return_opts=True)
            torch.cuda.synchronize()
            assert o.K_used < 64
            assert torch.equal(out, ref), (prec, i)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_every_dimension_served_equals_standalone(prec):
    # the batched kernel instances for d = 1..8 (runtime window radius except
    # d = 3, 6 at fixed radii), one launch holding several requests per d
    specs = [(d, 29 + 3 * d, 41 - 2 * d, 1.0 + 0.5 * (d % 3)) for d in range(1, 9)]
    imgs = [torch.from_numpy(voronoi_image(H, W, d, 7, 0.0, 1.0, 0.02, seed=300 + d)).to(DEV)
            for d, H, W, _ in specs]
    with P.Server(arena_bytes=1 << 28, quantum_us=5.0) as srv:
        ts = []
        for (d, H, W, s), f in zip(specs, imgs):
            C = random_spd(d, -2.5, -1.5, seed=d)
            for k in (3, 7):
                t, out = srv.submit(f, s, C, k, seed=d * 10 + k, precision=prec)
                ts.append((f, s, C, k, d, t, out))
        srv.drain(timeout=60.0)
        for f, s, C, k, d, t, out in ts:
            assert srv.poll(t)["state"] == "done"
            ref, _ = P.bf_vec_ex(f, s, C, k, seed=d * 10 + k, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (prec, d, k)


def test_random_mix_matches_standalone():
    # 60 seeded random requests: every d, odd sizes, windows up to R = 39,
    # K up to 40, all precisions, merged draws, centring on/off, given N, and
    # (from a second stream of draws) every spatial filter, the running-sum
    # pass and every whitening mode, so one server mixes all kernel variants
    rng = np.random.default_rng(2024)
    rng2 = np.random.default_rng(4048)
    reqs = []
    for i in range(60):
        d = int(rng.integers(1, 9))
        H, W = int(rng.integers(1, 160)), int(rng.integers(1, 160))
        sigma = float(rng.choice([0.0, 0.7, 1.5, 2.0, 3.3, 5.0, 8.0, 13.0]))
        K = int(rng.integers(1, 41))
        prec = str(rng.choice(["fp32", "fp16", "bf16"]))
        N = int(rng.choice([0, 0, 12, 40]))
        center = bool(rng.integers(0, 2))
        dedup = bool(rng.integers(0, 2))
        spatial = str(rng2.choice(["gauss", "gauss", "box", "hat", "box3", "box3+runsum"]))
        if prec != "fp32":
            spatial = spatial.replace("+runsum", "")
        whiten = str(rng2.choice(["eig", "chol", "sym"]))
        f = torch.from_numpy(voronoi_image(H, W, d, 5, 0.0, 1.0, 0.02, seed=900 + i)).to(DEV)
        C = random_spd(d, -2.0, -1.0, seed=i)
        reqs.append((f, sigma, C, K, 77 + i, N, prec, center, dedup, spatial, whiten))
    with P.Server(arena_bytes=1 << 28, quantum_us=float(rng.choice([3.0, 50.0, 1e4]))) as srv:
        ts = []
        for f, sigma, C, K, seed, N, prec, center, dedup, spatial, whiten in reqs:
            try:
                t, out = srv.submit(f, sigma, C, K, seed, N=N, precision=prec, center=center,
                                    dedup=dedup, spatial=spatial, whiten=whiten)
            except B.BfError as e:
                # only a window too large for the LDS budget is refused, and
                # the standalone call refuses it too
                assert e.code == B.BF_EUNSUPPORTED, e
                with pytest.raises(B.BfError):
                    P.bf_vec_ex(f, sigma, C, K, seed, N=N, precision=prec, spatial=spatial)
                t, out = None, None
            ts.append((t, out))
        srv.drain(timeout=120.0)
        n_run = 0
        for (f, sigma, C, K, seed, N, prec, center, dedup, spatial, whiten), (t, out) in \
                zip(reqs, ts):
            if t is None:
                continue
            st = srv.poll(t)
            assert st["state"] == "done", st
            ref, _ = P.bf_vec_ex(f, sigma, C, K, seed, N=N, precision=prec, center=center,
                                 dedup=dedup, spatial=spatial, whiten=whiten)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (tuple(f.shape), sigma, K, prec, N, center, dedup,
                                           spatial, whiten)
            n_run += 1
        assert n_run >= 50


def test_concurrent_submitters():
    # four host threads submit at once; every request completes and equals
    # the standalone call
    import threading
    C = 0.08 ** 2 * np.eye(3)
    imgs = [torch.from_numpy(voronoi_image(64 + 8 * i, 80, 3, 9, 0.0, 1.0, 0.02, seed=40 + i))
            .to(DEV) for i in range(4)]
    with P.Server(arena_bytes=1 << 28, quantum_us=20.0) as srv:
        results, errors = {}, []

        def worker(i):
            try:
                for k in range(8):
                    t, out = srv.submit(imgs[i], 2.0, C, 4 + k, seed=100 * i + k)
                    results[(i, k)] = (t, out)
            except Exception as e:   # surfaced below
                errors.append(e)

        th = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors
        srv.drain(timeout=60.0)
        assert srv.stats()["completed"] == 32
        for (i, k), (t, out) in results.items():
            ref, _ = P.bf_vec_ex(imgs[i], 2.0, C, 4 + k, seed=100 * i + k, precision="fp16")
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (i, k)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_resumed_term_ranges_small_radius(prec):
    # one term per round: every launch after the first resumes at t0 > 0; with
    # 2R <= 8 the vertical pass writes in the launch's first two steps, whose
    # accumulators must be loaded at launch start (regression)
    f = torch.from_numpy(voronoi_image(57, 71, 3, 8, 0.0, 1.0, 0.02, seed=5)).to(DEV)
    C = 0.1 ** 2 * np.eye(3)
    with P.Server(arena_bytes=1 << 28, quantum_us=1e-9) as srv:   # below any term's cost
        ts = []
        for sigma in (0.0, 0.4, 0.7, 1.0, 1.3, 2.0):
            t, out = srv.submit(f, sigma, C, 24, seed=3, precision=prec)
            ts.append((sigma, t, out))
        srv.drain(timeout=60.0)
        for sigma, t, out in ts:
            assert srv.poll(t)["chunks"] == 24
            ref, _ = P.bf_vec_ex(f, sigma, C, 24, seed=3, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), sigma


def test_injected_launch_fault_fails_only_its_requests(monkeypatch):
    # The hook refuses the server's second batched launch from the host
    # (nothing runs on the device for it).  Requests go one at a time, each in
    # one launch: only the second fails, with BF_EDEVICE; the server keeps
    # serving, and the others equal their standalone results.
    monkeypatch.setenv("BF_FAULT_INJECT", "launch:2")
    C = 0.1 ** 2 * np.eye(3)
    imgs = [torch.from_numpy(voronoi_image(48 + 8 * i, 56, 3, 7, 0.0, 1.0, 0.02, seed=70 + i))
            .to(DEV) for i in range(5)]
    sts, outs = [], []
    with P.Server(arena_bytes=1 << 26, quantum_us=1e9) as srv:
        for i, f in enumerate(imgs):
            t, out = srv.submit(f, 2.0, C, 8, seed=5 + i, N=16, precision="fp32")
            sts.append(srv.wait(t, 60.0))
            outs.append(out)
        stats = srv.stats()
    assert sts[1]["state"] == "failed" and sts[1]["error"] == B.BF_EDEVICE, sts[1]
    assert "injected" in sts[1]["message"]
    for i in (0, 2, 3, 4):
        assert sts[i]["state"] == "done", sts[i]
        ref, _ = P.bf_vec_ex(imgs[i], 2.0, C, 8, 5 + i, N=16, precision="fp32")
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), i
    assert stats["failed"] == 1 and stats["completed"] == 4


@pytest.mark.parametrize("policy,graph_rounds,autotune,host_io", [
    ("shortest", False, False, False),
    ("share", True, False, False),
    ("share", False, True, False),
    ("shortest", True, True, True),
])
def test_server_modes_match_standalone_bitwise(pools, policy, graph_rounds, autotune, host_io):
    # shortest-remaining-work-first rounds, graph-captured rounds, strip
    # heights measured per size class at submit, and host-resident images and
    # results (uploaded and downloaded by the server): none changes a result
    # bit (chunking and batching only split Algorithm 1's term loop; the strip
    # height changes no bit)
    print(f"case server policy={policy} graph_rounds={graph_rounds} autotune={autotune} "
          f"host_io={host_io}", flush=True)
    alone = [_alone(_crop(pools, spec), spec) for spec in MIX]
    hosts = (pools[0].cpu().pin_memory(), pools[1].cpu().pin_memory()) if host_io else None
    with P.Server(arena_bytes=1 << 30, streams=3, depth=2, quantum_us=20.0, policy=policy,
                  graph_rounds=graph_rounds, autotune=autotune) as srv:
        tickets = []
        for spec in MIX:
            fc = _crop(hosts if host_io else pools, spec)
            _, _, _, _, _, s, K, N, prec, center, cov = spec
            t, out = srv.submit(fc, s, _cov(cov, fc.shape[2]), K, seed=1000 + K, N=N,
                                precision=prec, center=center)
            assert out.is_cuda != host_io
            tickets.append((t, out))
        srv.drain(timeout=60.0)
        stats = srv.stats()
        for spec, (t, out), (ref, n_ref) in zip(MIX, tickets, alone):
            st = srv.poll(t)
            assert st["state"] == "done", (spec, st)
            assert st["N_used"] == n_ref, spec
            got = out if not host_io else out.to(DEV)
            assert torch.equal(got, ref), (spec, float((got - ref).abs().max()))
        assert stats["completed"] == len(MIX) and stats["failed"] == 0
        assert stats["rounds"] >= 4
        # the cost model's scale, measured from the rounds' device time
        assert 0.05 <= stats["model_scale"] <= 20.0 and stats["model_scale"] != 1.0, stats


def test_split_precision_served_equals_standalone():
    # the split FP32 mode's batched instances (d = 3, R = 18, 21, 24, 30): several
    # requests per launch, term ranges resumed across rounds, each result
    # the bits of bf_vec_ex; an unsupported radius is refused at submit
    specs = [(96, 70, 7.0), (64, 100, 8.0), (80, 96, 10.0), (64, 64, 10.0)]
    imgs = [torch.from_numpy(voronoi_image(H, W, 3, 5, 0.0, 1.0, 0.02, seed=500 + i)).to(DEV)
            for i, (H, W, _) in enumerate(specs)]
    C = 0.1 ** 2 * np.eye(3)
    with P.Server(arena_bytes=1 << 28, quantum_us=5.0) as srv:
        ts = []
        for i, ((H, W, s), f) in enumerate(zip(specs, imgs)):
            for k in (5, 40):
                t, out = srv.submit(f, s, C, k, seed=i * 10 + k, precision="fp32_split")
                ts.append((f, s, k, i, t, out))
        with pytest.raises(P.BfError) as e:
            srv.submit(imgs[0], 2.0, C, 4, 1, precision="fp32_split")
        assert e.value.code == B.BF_EUNSUPPORTED
        srv.drain(timeout=60.0)
        for f, s, k, i, t, out in ts:
            assert srv.poll(t)["state"] == "done"
            ref, _ = P.bf_vec_ex(f, s, C, k, seed=i * 10 + k, precision="fp32_split")
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (s, k, i)
