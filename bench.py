#!/usr/bin/env python3
"""Benchmark of the MCSF hot path on one MI355X.

A step is one whole call of the filter (bf_vec_ex: min/max reduction, order
rule, whitening, term draws, term upload, fused kernel) over the
4096x4096x3 sigma_s=10 K=256 workload, input resident in HBM.  Prints one
JSON line with Mpix/s, the fused kernel's roofline position (HIP events around
each launch), the FP64 oracle's rate on the host as a CPU baseline, and the
serving run: a stream of mixed requests through the continuous-batching
server, first all at once (sustained capacity), then as Poisson arrivals at a
fraction of that capacity (p50/p99 latency).
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s at 4096^2x3 σs=10 K=256 (FP32 vs FP16) + p50/p99 serving latency"
PEAK_FP32_VALU = 157.3      # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
PEAK_FP32_NONPACKED = 78.6  # TFLOP/s: the same without packed-FP32 issue


# HBM bytes per launch of the benchmark's fused kernel, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same
# counters read for a 1 GiB device copy (FETCH_SIZE 524,313.375 KiB: factor
# 1.99988; WRITE_SIZE 1,048,576 KiB: factor 1.0), with the executed VALU and
# matrix-core flops of the same launches (rocprofv3 --pmc
# SQ_INSTS_VALU_FLOPS_* x 64 lanes, SQ_INSTS_VALU_MFMA_MOPS_* x 512).  Valid only for the kernel
# sources they were taken on (TRAFFIC_SOURCES hash); otherwise reported null.
TRAFFIC_SOURCES = ["paper_1605_02164_amd/csrc/mcsf_fused_dev.h",
                   "paper_1605_02164_amd/csrc/mcsf_common.h",
                   "paper_1605_02164_amd/csrc/mcsf_fused.hip"]
TRAFFIC = {
    "sha256": "da6c486fd86f1c5303c2a3bd0b07aa347fad04d42cecc7b01c6459efadd2c97d",
    "fetch_factor": 1048576 / 524313.5625,
    "write_factor": 1048576 / 1048576.0,
    "fp32": {"fetch_kib": 78210137.5, "write_kib": 67108864.0, "valu_flops": 318634459136.0, "mfma_flops": 10771777978368.0},
    "fp16": {"fetch_kib": 97799809.1875, "write_kib": 67108715.8125, "valu_flops": 505198673920.0, "mfma_flops": 20615843020800.0},
}
COUNTERS_PROFILE = "profiles/mcsf_fused_voronoi4096_d3_s10_K256.md"


def _counters(prec):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sha256"] or prec not in TRAFFIC:
        return None
    return TRAFFIC[prec]


def measured_traffic(prec):
    """HBM bytes per launch for the current kernel sources, or None."""
    t = _counters(prec)
    if t is None:
        return None
    return (t["fetch_kib"] * TRAFFIC["fetch_factor"] + t["write_kib"] * TRAFFIC["write_factor"]) * 1024


def kernel_name(d, R, prec, tile_w, mf):
    """The fused-kernel instance a launch ran: mcsf_fused<d, R, storage,
    FP64-phase path, strip width, matrix-core passes>."""
    return f"mcsf_fused<{d}, {R}, {prec}, p64=0, TW={tile_w}, MF={int(bool(mf))}>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops_per_pixel(d, R, K):
    """Per output pixel: K x [4d (phase + modulation) + 8(d+1)(2R+1) (two
    separable passes over 2(d+1) real channels) + 4(d+1) (demodulation)]."""
    return K * (4 * d + 8 * (d + 1) * (2 * R + 1) + 4 * (d + 1))


def _cpu_info():
    """(CPU model, logical CPUs of the machine, CPUs this process may use)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(f, C, sigma_s, K, seed, N, gpu_outs=None, crop=1024, direct_crop=192,
                 n_acc_pixels=1024):
    """The FP64 oracle on the host cores (CPU baseline leg).

    1. O3, the separable MCSF of Algorithm 1 (the oracle as it stands), on a
       centred crop: the K terms are split over the worker threads (numpy
       releases the GIL inside its array operations; each worker's BLAS is
       limited to one thread), each worker filters the crop with its share of
       the terms, and the numerators and normalisers are summed (both are
       sums over terms).  A bounded sample of the terms is run (six per
       worker, about 10-20 s) and the rate scaled to all K.
    2. O1, the direct filter of eqs. (BF)/(normal) with the exact Gaussian
       range kernel (the paper's comparison method), on a smaller centred
       crop, pixels split over the workers.
    3. The GPU outputs (gpu_outs: mode -> ((H, W, d) tensor, spatial
       filter: 0 Gaussian, 3 three boxes)) against O2, the direct filter with
       the same sampled kernel and spatial filter, at seeded pixels: max and
       mean error as a fraction of each channel's range.
    """
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from oracle import mcsf as O
    model, nproc, usable = _cpu_info()
    workers = max(1, min(16, usable))   # at most 16 host threads per GPU
    H, W, d = f.shape
    f64 = f.astype(np.float64)
    Wm = O.whiten(C)
    _, w = O.sample_terms(C, N, K, seed, W=Wm)
    y0, x0 = (H - crop) // 2, (W - crop) // 2
    sub = f64[y0:y0 + crop, x0:x0 + crop]
    k_run = min(K, 6 * workers)
    shares = [s for s in np.array_split(np.arange(k_run), workers) if len(s)]

    def o3_share(idx):
        _, num, Z = O.mcsf_separable(sub, sigma_s, w[idx])
        return num, Z

    with threadpool_limits(limits=1), ThreadPoolExecutor(workers) as ex:
        t0 = time.perf_counter()
        parts = list(ex.map(o3_share, shares))
        num = sum(p[0] for p in parts)
        Z = sum(p[1] for p in parts)
        _ = num / Z[..., None]
        dt = time.perf_counter() - t0
    rate = crop * crop * (k_run / K) / dt / 1e6
    rec = {"value": rate, "unit": "Mpix/s", "cores": len(shares), "kind": "oracle",
           "sample": f"separable FP64 oracle (Algorithm 1) on the {crop}x{crop} centre crop, "
                     f"the first {k_run} of the {K} terms split over {len(shares)} threads "
                     f"({dt:.1f} s), rate scaled to {K} terms",
           "cpu_model": model, "nproc": nproc, "usable_cpus": usable}
    # O1 on a smaller crop
    yd, xd = (H - direct_crop) // 2, (W - direct_crop) // 2
    dsub = f64[yd:yd + direct_crop, xd:xd + direct_crop]
    pix = np.stack(np.meshgrid(np.arange(direct_crop), np.arange(direct_crop), indexing="ij"),
                   axis=-1).reshape(-1, 2)
    with threadpool_limits(limits=1), ThreadPoolExecutor(workers) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda c: O.direct_exact(dsub, sigma_s, C, pixels=c),
                    np.array_split(pix, 8 * workers)))
        dt1 = time.perf_counter() - t0
    rec["direct_o1"] = {"value": direct_crop ** 2 / dt1 / 1e6, "unit": "Mpix/s",
                        "cores": workers,
                        "sample": f"direct FP64 filter, exact Gaussian range kernel, "
                                  f"{direct_crop}x{direct_crop} centre crop, pixels split over "
                                  f"{workers} threads ({dt1:.1f} s)"}
    if gpu_outs:
        rng = np.random.default_rng(17)
        n = n_acc_pixels
        pts = np.stack([rng.integers(0, H, n), rng.integers(0, W, n)], axis=1)
        corners = np.array([[0, 0], [0, W - 1], [H - 1, 0], [H - 1, W - 1]])
        pts = np.unique(np.concatenate([pts, corners]), axis=0)
        refs, dt2 = {}, 0.0
        for sp in sorted({v[1] for v in gpu_outs.values()}):
            with threadpool_limits(limits=1), ThreadPoolExecutor(workers) as ex:
                t0 = time.perf_counter()
                res = list(ex.map(lambda c: O.direct_sampled(f64, sigma_s, w, pixels=c,
                                                             spatial=sp),
                                  np.array_split(pts, 8 * workers)))
                dt2 += time.perf_counter() - t0
            refs[sp] = np.concatenate([r[0] for r in res])
        span = f64.reshape(-1, d).max(0) - f64.reshape(-1, d).min(0)
        span[span == 0] = 1.0
        acc = {}
        for mode, (out, sp) in gpu_outs.items():
            # out: a device tensor of the GPU run; only the sampled pixels come back
            g = out[pts[:, 0], pts[:, 1]].double().cpu().numpy()
            e = np.abs(g - refs[sp]) / span
            acc[mode] = {"max_err": float(e.max()), "mean_err": float(e.mean())}
        rec["accuracy_vs_oracle"] = {
            "reference": "O2: direct filter with the same K sampled terms and the mode's "
                         "spatial filter (FP64)",
            "pixels": int(len(pts)), "unit": "fraction of each channel's range",
            "oracle_s": dt2, "modes": acc}
    return rec


def serving_run(args, P, torch, log_fn, policy="share", graph_rounds=False, autotune=False,
                host_io=False, n=None, rate=None):
    """Serving workload: requests with square sides log-uniform in
    [256, 2048], d in {3, 6}, sigma_s in {2..8}, C = sigma_r^2 I with sigma_r
    ~ U[0.05, 0.2], K in {64, 128, 256}, FP16 storage.  Images are crops (at
    request-seeded offsets, row pitch 2048) of two resident 2048^2 images:
    Voronoi colour (d = 3) and colour plus correlated channels (d = 6).  With
    host_io the pools and the results are in pinned host memory and the
    server uploads each crop and downloads each result (inside the latency).
    policy / graph_rounds / autotune: the server's round policy, graph-captured
    rounds, and strip heights measured per size class (warm-up covers every
    class, so no measurement falls in the timed runs).  rate: Poisson arrival
    rate in requests/s (default: args.serve_load x this run's capacity)."""
    import numpy as np
    from synth import serving_requests, voronoi_image, feature_image
    dev = torch.device("cuda:0")
    n = n or args.serve_requests
    log_fn(f"serving ({policy}, graph_rounds={graph_rounds}, autotune={autotune}, "
           f"host_io={host_io}): generating the 2048^2 image pools")
    pool = {3: torch.from_numpy(voronoi_image(2048, 2048, 3, 64, 0.0, 1.0, 0.02, seed=3003)),
            6: torch.from_numpy(feature_image(2048, 2048, 64, seed=3004, smooth_sigma=32.0))}
    pool = {k: (v.pin_memory() if host_io else v.to(dev)) for k, v in pool.items()}
    reqs = serving_requests(n, seed=5, rate_hz=1.0)
    crops, total_px, outs = [], 0, []
    for q in reqs:
        rng = np.random.Generator(np.random.PCG64(q["image_seed"]))
        s = q["H"]
        oy, ox = (int(v) for v in rng.integers(0, 2048 - s + 1, size=2))
        crops.append(pool[q["d"]][oy:oy + s, ox:ox + s])
        total_px += s * s
    if host_io:
        # results: a ring of pinned buffers of the largest size (requests far
        # apart in the stream share one; only the timing is used here)
        bufs = [torch.empty(2048 * 2048 * 6, dtype=torch.float32).pin_memory() for _ in range(32)]
        for i, q in enumerate(reqs):
            outs.append(bufs[i % len(bufs)][:q["H"] * q["W"] * q["d"]].view(q["H"], q["W"], q["d"]))
    else:
        flat = torch.empty(sum(q["H"] * q["W"] * q["d"] for q in reqs), dtype=torch.float32,
                           device=dev)
        o = 0
        for q in reqs:
            m = q["H"] * q["W"] * q["d"]
            outs.append(flat[o:o + m].view(q["H"], q["W"], q["d"]))
            o += m
    torch.cuda.synchronize()
    srv = P.Server(arena_bytes=args.serve_arena_gib << 30, max_active=args.serve_max_active,
                   quantum_us=args.serve_quantum_us, depth=args.serve_depth,
                   streams=args.serve_streams, policy=policy, graph_rounds=graph_rounds,
                   autotune=autotune)
    dedup = not args.serve_no_dedup

    def submit_all(arrivals):
        ts = []
        for q, f, out, a in zip(reqs, crops, outs, arrivals):
            C = (q["sigma_r"] ** 2) * np.eye(q["d"])
            t, _ = srv.submit(f, q["sigma_s"], C, q["K"], seed=q["term_seed"], out=out,
                              precision="fp16", arrival=a, dedup=dedup)
            ts.append(t)
        return ts

    def collect(ts):
        sts = [srv.poll(t) for t in ts]
        bad = [s for s in sts if s["state"] != "done"]
        if bad:
            raise RuntimeError(f"serving: {len(bad)} requests did not finish: {bad[0]}")
        for t in ts:
            srv.forget(t)
        return sts

    # warm-up: one small request of every kernel instance in the stream; with
    # autotune also one request of every (d, sigma_s, size class) present
    seen = {}
    for i, q in enumerate(reqs):
        seen.setdefault((q["d"], q["sigma_s"]), i)
        if autotune:
            seen.setdefault((q["d"], q["sigma_s"], int(np.floor(2 * np.log2(q["H"]) + 0.5))), i)
    warm = []
    for key, i in seen.items():
        d, sig = key[0], key[1]
        C = (reqs[i]["sigma_r"] ** 2) * np.eye(d)
        f = pool[d][:96, :96] if len(key) == 2 else crops[i]
        t, _ = srv.submit(f, sig, C, 8, seed=1)
        warm.append(t)
    srv.drain(600.0)
    collect(warm)

    # 1. capacity: everything arrives at once
    log_fn(f"serving: {n} requests at once")
    t0 = srv.clock() + 0.5
    ts = submit_all([t0] * n)
    srv.drain(1200.0)
    sts = collect(ts)
    makespan = max(s["done"] for s in sts) - t0
    capacity = n / makespan
    sat = {"makespan_s": makespan, "capacity_rps": capacity, "mpix_s": total_px / makespan / 1e6,
           "p50_ms": 1e3 * float(np.percentile([s["done"] - s["arrival"] for s in sts], 50))}
    log_fn(f"serving: capacity {capacity:.1f} req/s, {sat['mpix_s']:.1f} Mpix/s")

    # 2. latency: Poisson arrivals at args.serve_load x capacity (or the rate given)
    rate = rate or args.serve_load * capacity
    arr = [q["arrival"] / rate for q in reqs]   # the generator's unit-rate arrival times
    log_fn(f"serving: {n} Poisson arrivals at {rate:.1f} req/s")
    t0 = srv.clock() + 0.5
    ts = submit_all([t0 + a for a in arr])
    srv.drain(1200.0)
    sts = collect(ts)
    lat = np.array([s["done"] - s["arrival"] for s in sts]) * 1e3
    span = max(s["done"] for s in sts) - t0
    stats = srv.stats()
    srv.close()
    # slowdown: latency over the request's modelled size (pixels x terms),
    # normalised by the median; shows how the policy treats small and large jobs
    size = np.array([q["H"] * q["W"] * q["K"] for q in reqs], dtype=np.float64)
    # spot check: a few requests equal the same filter run alone, bit for bit
    same = None
    if not host_io:
        same = True
        for i in (0, n // 2, n - 1):
            q = reqs[i]
            ref, _ = P.bf_vec_ex(crops[i].contiguous(), q["sigma_s"],
                                 (q["sigma_r"] ** 2) * np.eye(q["d"]), q["K"],
                                 seed=q["term_seed"], precision="fp16", dedup=dedup)
            torch.cuda.synchronize()
            same = same and bool(torch.equal(ref, outs[i]))
    small = size <= np.percentile(size, 50)
    rec = {
        "requests": n, "precision": "fp16", "load": args.serve_load, "rate_rps": rate,
        "policy": policy, "graph_rounds": graph_rounds, "autotune": autotune,
        "host_io": host_io,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()), "mean_ms": float(lat.mean()),
        "p99_small_half_ms": float(np.percentile(lat[small], 99)),
        "p99_large_half_ms": float(np.percentile(lat[~small], 99)),
        "mpix_s": total_px / span / 1e6, "total_mpix": total_px / 1e6,
        "saturated": sat, "quantum_us": args.serve_quantum_us, "depth": args.serve_depth,
        "streams": args.serve_streams, "dedup": dedup,
        "max_active": args.serve_max_active, "rounds": stats["rounds"],
        "launches": stats["launches"], "arena_peak_gib": stats["arena_peak"] / 2**30,
        "model_scale": stats["model_scale"],
        "spot_check_bitwise_equal_alone": same,
    }
    log_fn(f"serving: p50 {rec['p50_ms']:.1f} ms, p99 {rec['p99_ms']:.1f} ms "
           f"(small half {rec['p99_small_half_ms']:.1f}, large half "
           f"{rec['p99_large_half_ms']:.1f}), {rec['mpix_s']:.1f} Mpix/s")
    return rec


def serving_variants(args, P, torch, log_fn, rate):
    """The serving run under each scheduler option, one at a time against the
    default (processor sharing, direct launches, occupancy-model strips,
    device-resident images), and with host-resident images and results; the
    Poisson phase of every variant runs at the same arrival rate (the
    default's), so the latencies compare like for like."""
    out = []
    for kw in (dict(policy="shortest"), dict(graph_rounds=True), dict(autotune=True),
               dict(host_io=True, n=min(args.serve_requests, 1000))):
        out.append(serving_run(args, P, torch, log_fn, rate=rate, **kw))
    return out


def plan_run(P, torch, log_fn, reps=200):
    """Fixed-shape plans against bf_vec_ex on serving-sized images (d = 3,
    FP16 storage, centring on, N = 20, Voronoi colour images): the latency of
    one image (call + device synchronisation; median and p99 of `reps`), and
    the rate of `reps` images queued back to back (bf_vec_ex waits for each
    image's min/max on the host; a plan's execution waits for nothing)."""
    import numpy as np
    from synth import voronoi_image
    dev = torch.device("cuda:0")
    res = []
    for side, sigma_s, K in ((256, 2.0, 64), (512, 4.0, 64), (1024, 8.0, 128)):
        f = torch.from_numpy(voronoi_image(side, side, 3, 24, 0.0, 1.0, 0.02, seed=side)).to(dev)
        C = 0.1 ** 2 * np.eye(3)
        o1, o2 = torch.empty_like(f), torch.empty_like(f)
        kw = dict(N=20, precision="fp16")
        plan = P.Plan(side, side, 3, sigma_s, C, K, 7, **kw)

        def eager():
            P.bf_vec_ex(f, sigma_s, C, K, 7, out=o1, **kw)

        def graph():
            plan(f, o2)

        row = {"side": side, "sigma_s": sigma_s, "K": K}
        for name, fn in (("bf_vec_ex", eager), ("plan", graph)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            lat = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                lat.append(1e3 * (time.perf_counter() - t0))
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            rate = reps / (time.perf_counter() - t0)
            row[name] = {"p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "images_s": rate}
        row["bitwise_equal"] = bool(torch.equal(o1, o2))
        plan.close()
        log_fn(f"plan {side}^2 K={K}: latency p50 {row['bf_vec_ex']['p50_ms']:.3f} ms -> "
               f"{row['plan']['p50_ms']:.3f} ms, back-to-back {row['bf_vec_ex']['images_s']:.0f}"
               f" -> {row['plan']['images_s']:.0f} images/s, equal {row['bitwise_equal']}")
        res.append(row)
    return res


def _timed(fn, reps):
    """Median wall time (ms) of fn() followed by a device synchronisation."""
    import numpy as np
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts))


def mse_db(a, b):
    """10 log10 of the mean squared difference over pixels and channels
    (eq. (MSE)), images on a [0, 255] scale."""
    import math
    import torch
    m = float(torch.mean((a.double() - b.double()) ** 2))
    return 10 * math.log10(m) if m > 0 else float("-inf")


def study_table1(P, torch, log_fn):
    """Runtime against sigma_s (the paper's Table 1 setting on a synthetic
    stand-in for its 512x512 colour image): direct filter (eq. (BF), exact
    Gaussian range kernel) against MCSF with N = 10, T = 300 terms, sigma_r =
    40 on a [0, 255] scale; both on this GPU."""
    import numpy as np
    from synth import voronoi_image
    f = torch.from_numpy(voronoi_image(512, 512, 3, 64, 0.0, 255.0, 5.0, seed=7001)).cuda()
    C = 40.0 ** 2 * np.eye(3)
    rows = []
    for s in (1, 2, 3, 4, 5, 10):
        ref = torch.empty_like(f)
        t_direct = _timed(lambda: P.bf_direct(f, s, C, out=ref), 3)
        rec = {"sigma_s": s, "direct_ms": t_direct}
        for prec in ("fp32", "fp16"):
            out = torch.empty_like(f)
            rec[f"mcsf_{prec}_ms"] = _timed(
                lambda: P.bf_vec_ex(f, s, C, 300, 11, out=out, N=10, precision=prec), 5)
            rec[f"mcsf_{prec}_mse_db"] = mse_db(out, ref)
        log_fn(f"table1 sigma_s={s}: " + ", ".join(f"{k} {v:.3g}" for k, v in rec.items()
                                                   if k != "sigma_s"))
        rows.append(rec)
    return {"study": "runtime_vs_sigma_s", "image": "512x512x3 Voronoi [0,255]",
            "sigma_r": 40, "N": 10, "K": 300, "rows": rows}


def _radius(sigma_s, n):
    """Window radius for reporting: ceil(3 sigma_s) for the Gaussian, n r for
    n boxes with r nearest the root of n((2r+1)^2 - 1)/12 = sigma_s^2."""
    if n == 0:
        return int(math.ceil(3 * sigma_s))
    return n * int(math.floor((math.sqrt(12 * sigma_s ** 2 / n + 1) - 1) / 2 + 0.5))


def study_spatial(P, torch, log_fn):
    """Kernel time against sigma_s for the Gaussian and the three-box spatial
    filter (the paper's O(1)-in-sigma_s remark): 2048^2 x 3 Voronoi image,
    K = 64, N = 37, C = 0.08^2 I.  FP32: Gaussian and three boxes with FIR
    passes, and three boxes with the running-sum vertical pass
    ("box3+runsum"); FP16 storage: FIR passes.  Times are HIP events around
    the fused kernel (median of 5)."""
    import numpy as np
    from synth import voronoi_image
    f = torch.from_numpy(voronoi_image(2048, 2048, 3, 128, 0.0, 1.0, 0.02, seed=7101)).cuda()
    C = 0.08 ** 2 * np.eye(3)
    out = torch.empty_like(f)
    rows = []
    for s_ in (1.0, 2.0, 4.0, 6.0, 8.0, 10.0, 12.0):
        rec = {"sigma_s": s_}
        for prec, sp in (("fp32", "gauss"), ("fp32", "box3"), ("fp32", "box3+runsum"),
                         ("fp16", "gauss"), ("fp16", "box3")):
            ms = []
            for _ in range(6):
                _, o = P.bf_vec_ex(f, s_, C, 64, 11, out=out, N=37, precision=prec,
                                   spatial=sp, time_kernel=True, return_opts=True)
                ms.append(o.kernel_ms)
            rec[f"{sp}_{prec}_ms"] = float(np.median(ms[1:]))
        rec["R_gauss"] = _radius(s_, 0)
        rec["R_box3"] = _radius(s_, 3)
        log_fn(f"spatial sigma_s={s_}: " + ", ".join(f"{k} {v:.3g}" for k, v in rec.items()
                                                     if k != "sigma_s"))
        rows.append(rec)
    return {"study": "kernel_time_vs_sigma_s_spatial_filter", "image": "2048x2048x3 Voronoi",
            "K": 64, "N": 37, "rows": rows}


def study_mse(P, torch, log_fn, realizations):
    """MSE against the number of terms for N = 10 and N = 20 (the paper's
    error-plot setting on a synthetic stand-in for its 876x584 image):
    sigma_s = 1, sigma_r = 30 on a [0, 255] scale, averaged over
    `realizations` term seeds; reference = the direct filter on this GPU."""
    import numpy as np
    from synth import voronoi_image
    f = torch.from_numpy(voronoi_image(584, 876, 3, 64, 0.0, 255.0, 5.0, seed=7002)).cuda()
    C = 30.0 ** 2 * np.eye(3)
    ref = P.bf_direct(f, 1.0, C)
    torch.cuda.synchronize()
    out = torch.empty_like(f)
    rows = []
    for N in (10, 20):
        for K in (10, 20, 50, 100, 200, 300, 500, 1000):
            acc = 0.0
            for r in range(realizations):
                P.bf_vec_ex(f, 1.0, C, K, 100000 + r, out=out, N=N)
                acc += float(torch.mean((out.double() - ref.double()) ** 2))
            m = acc / realizations
            rows.append({"N": N, "K": K, "mse": m, "mse_db": 10 * math.log10(m)})
            log_fn(f"mse N={N} K={K}: {rows[-1]['mse_db']:.2f} dB")
    return {"study": "mse_vs_terms", "image": "876x584x3 Voronoi [0,255]", "sigma_s": 1,
            "sigma_r": 30, "realizations": realizations, "rows": rows}


def srgb_to_lab(rgb):
    """sRGB in [0, 255] (D65) to CIE-Lab: inverse companding, the sRGB
    primaries' XYZ matrix, then the CIE L*a*b* transform."""
    import numpy as np
    c = np.clip(rgb / 255.0, 0, 1)
    lin = np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)
    M = np.array([[0.4124564, 0.3575761, 0.1804375],
                  [0.2126729, 0.7151522, 0.0721750],
                  [0.0193339, 0.1191920, 0.9503041]])
    xyz = lin @ M.T / np.array([0.95047, 1.0, 1.08883])
    e = 216 / 24389
    k = 24389 / 27
    fx = np.where(xyz > e, np.cbrt(xyz), (k * xyz + 16) / 116)
    return np.stack([116 * fx[..., 1] - 16, 500 * (fx[..., 0] - fx[..., 1]),
                     200 * (fx[..., 1] - fx[..., 2])], axis=-1)


def lab_to_srgb(lab):
    """Inverse of srgb_to_lab, to [0, 255] (clipped)."""
    import numpy as np
    e = 216 / 24389
    k = 24389 / 27
    fy = (lab[..., 0] + 16) / 116
    fx = fy + lab[..., 1] / 500
    fz = fy - lab[..., 2] / 200
    inv = lambda f: np.where(f ** 3 > e, f ** 3, (116 * f - 16) / k)
    xyz = np.stack([inv(fx), inv(fy), inv(fz)], axis=-1) * np.array([0.95047, 1.0, 1.08883])
    Minv = np.linalg.inv(np.array([[0.4124564, 0.3575761, 0.1804375],
                                   [0.2126729, 0.7151522, 0.0721750],
                                   [0.0193339, 0.1191920, 0.9503041]]))
    lin = np.clip(xyz @ Minv.T, 0, 1)
    c = np.where(lin <= 0.0031308, 12.92 * lin, 1.055 * lin ** (1 / 2.4) - 0.055)
    return 255.0 * c


def study_lab(P, torch, log_fn):
    """Filtering in CIE-Lab (the paper's third example: 256x256, sigma_s = 5,
    sigma_r = 90 in Lab units, N = 10, T = 300): RGB -> Lab on the host,
    MCSF and the direct filter on this GPU, back to RGB, MSE in dB on the
    [0, 255] RGB scale; also the same filters applied in RGB."""
    import numpy as np
    from synth import voronoi_image
    rgb = voronoi_image(256, 256, 3, 32, 0.0, 255.0, 5.0, seed=7003).astype(np.float64)
    lab = srgb_to_lab(rgb)
    rows = {}
    for space, img in (("lab", lab), ("rgb", rgb)):
        f = torch.from_numpy(img.astype(np.float32)).cuda()
        C = 90.0 ** 2 * np.eye(3)
        ref = P.bf_direct(f, 5.0, C)
        out, _ = P.bf_vec_ex(f, 5.0, C, 300, 13, N=10)
        torch.cuda.synchronize()
        a, b = ref.cpu().double().numpy(), out.cpu().double().numpy()
        if space == "lab":
            a, b = lab_to_srgb(a), lab_to_srgb(b)
        m = float(np.mean((a - b) ** 2))
        rows[space] = {"mse_db_rgb": 10 * math.log10(m)}
        log_fn(f"lab study: filtered in {space}: MCSF vs direct {rows[space]['mse_db_rgb']:.2f} dB")
    rt = lab_to_srgb(srgb_to_lab(rgb))
    return {"study": "cie_lab_pipeline", "image": "256x256x3 Voronoi sRGB [0,255]",
            "sigma_s": 5, "sigma_r": 90, "N": 10, "K": 300, "rows": rows,
            "round_trip_max_abs": float(np.abs(rt - rgb).max())}


def write_study(path, rec):
    """A study's record as a short markdown file: command, table, raw JSON."""
    rows = rec.get("rows")
    lines = [f"# {rec['study']}", "", f"Command: `{rec['command']}`", ""]
    meta = {k: v for k, v in rec.items() if k not in ("rows", "study", "command")}
    lines += [f"Settings: {json.dumps(meta)}", ""]
    if isinstance(rows, list) and rows:
        keys = list(rows[0].keys())
        lines += ["| " + " | ".join(keys) + " |", "|" + "---|" * len(keys)]
        for r in rows:
            lines.append("| " + " | ".join(f"{r[k]:.4g}" if isinstance(r[k], float) else str(r[k])
                                           for k in keys) + " |")
    elif isinstance(rows, dict):
        for k, v in rows.items():
            lines.append(f"- {k}: {json.dumps(v)}")
    lines += ["", "```json", json.dumps(rec), "```", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="voronoi4096_d3_s10_K256")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "bf16"],
                    help="precision of the headline value; the other modes are reported beside it")
    ap.add_argument("--only", action="store_true", help="time only --precision")
    ap.add_argument("--modes", help="comma-separated modes to time instead of the default set "
                                    "(fp32, fp16, bf16, fp32_split, *_valu, *_dedup, fp32_box3, "
                                    "fp32_box3rs, fp32_box3sl; "
                                    "a _w16 suffix forces 16-column strips); "
                                    "the first is the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-plan", action="store_true",
                    help="skip the fixed-shape plan (HIP graph) latency comparison")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the occupancy model's strip height instead of measuring it")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="Poisson arrival rate as a fraction of the measured capacity")
    ap.add_argument("--serve-quantum-us", type=float, default=2000.0)
    ap.add_argument("--serve-max-active", type=int, default=64)
    ap.add_argument("--serve-arena-gib", type=int, default=16)
    ap.add_argument("--serve-depth", type=int, default=2)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-no-dedup", action="store_true",
                    help="run every drawn term (default: merge equal +-Y draws, exact)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving run (no headline modes, CPU baseline or comparator)")
    ap.add_argument("--serve-variants", action="store_true",
                    help="also run the serving workload under each scheduler option "
                         "(shortest-first, graph rounds, autotune, host I/O)")
    ap.add_argument("--study", choices=["table1", "mse", "lab", "spatial"],
                    help="run one of the paper-study analogues instead of the benchmark and "
                         "print its JSON")
    ap.add_argument("--realizations", type=int, default=400)
    ap.add_argument("--out", help="with --study: also write the result (and the command line) "
                                  "to this markdown file")
    ap.add_argument("--ubench", action="store_true",
                    help="only run the device probes (bf_ubench: matrix, FMA, transcendental, "
                         "LDS and HBM rates) and print their JSON (with --out: also a markdown "
                         "table)")
    ap.add_argument("--copy-kernel-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates the "
                         "FETCH_SIZE/WRITE_SIZE counters against known traffic) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}); "
              "the filter would shard by bands of image rows (R halo rows copied once per "
              "neighbour) or by requests", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1605_02164_amd as P
    from synth import workload

    if args.study:
        rec = (study_table1(P, torch, log) if args.study == "table1"
               else study_lab(P, torch, log) if args.study == "lab"
               else study_spatial(P, torch, log) if args.study == "spatial"
               else study_mse(P, torch, log, args.realizations))
        rec["command"] = "python bench.py " + " ".join(sys.argv[1:])
        print(json.dumps(rec), flush=True)
        if args.out:
            write_study(args.out, rec)
        return

    if args.serve_only:
        rec = {"serving": serving_run(args, P, torch, log)}
        if args.serve_variants:
            rec["serving_variants"] = serving_variants(args, P, torch, log,
                                                       rec["serving"]["rate_rps"])
        print(json.dumps(rec), flush=True)
        return

    if args.ubench:
        rows = []
        for probe, params, unit in (("mfma_f32", (1, 2, 4, 8), "TFLOP/s"),
                                    ("mfma_f32_solo", (1, 2, 4), "TFLOP/s"),
                                    ("mfma_f16", (1, 2, 4, 8), "TFLOP/s"),
                                    ("valu_f32", (1, 2, 4, 8), "TFLOP/s"),
                                    ("trans_f32", (0,), "Top/s"),
                                    ("lds_read", (0,), "TB/s"),
                                    ("hbm_copy", (1024,), "TB/s"),
                                    ("overlap_f32", (0,), "fraction"),
                                    ("overlap_f16", (0,), "fraction")):
            for q in params:
                rows.append({"probe": probe, "param": q, "rate": P.bf_ubench(probe, q),
                             "unit": unit})
                log(f"{probe} param {q}: {rows[-1]['rate']:.2f} {unit}")
        rec = {"ubench": rows, "command": "python bench.py " + " ".join(sys.argv[1:])}
        print(json.dumps(rec), flush=True)
        if args.out:
            with open(args.out, "w") as fh:
                fh.write("# Device probes (bf_ubench), one MI355X\n\n")
                fh.write(f"Command: `{rec['command']}`\n\n")
                fh.write("Each probe: one workgroup of 8 waves (two per SIMD) per compute unit, "
                         "best of three timed launches; param = independent chains per wave "
                         "(matrix) or per lane (FMA), or the copy size in MiB. overlap_*: one "
                         "wave per SIMD runs matrix products, the other FMAs of about the same "
                         "duration; (t_matrix + t_fma - t_both) / min(t_matrix, t_fma), 1 when "
                         "they run side by side, 0 when their times add.\n\n")
                fh.write("| probe | param | rate | unit |\n|---|---|---|---|\n")
                for r in rows:
                    fh.write(f"| {r['probe']} | {r['param']} | {r['rate']:.2f} | {r['unit']} |\n")
        return

    if args.copy_kernel_mib:
        n = args.copy_kernel_mib * (1 << 20) // 4
        a = torch.ones(n, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_kernel_mib} MiB")
        return

    log(f"generating workload {args.workload}")
    f, C, p = workload(args.workload)
    H, W, d = f.shape
    sigma_s, K, seed = p["sigma_s"], p["K"], p["term_seed"]
    R = int(math.ceil(3 * sigma_s))
    dev = torch.device("cuda:0")
    fg = torch.from_numpy(f).to(dev)
    out = torch.empty_like(fg)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(prec, dst, dedup, spatial="gauss", valu=False, tile_w=0):
        _, o = P.bf_vec_ex(fg, sigma_s, C, K, seed, out=dst, precision=prec,
                           stream=stream, time_kernel=True, return_opts=True, dedup=dedup,
                           spatial=spatial, valu_only=valu, tile_w=tile_w)
        return o.N_used, o.kernel_ms, o.K_used, o.tile_h_used, o.tile_w_used, o.mfma_used

    tuned = {}

    def run(mode, dst):
        # fp32_split: FP32 with the vertical pass on FP16 hi + lo pairs
        prec = "fp32_split" if mode.startswith("fp32_split") else mode.split("_")[0]
        dedup = mode.endswith("_dedup")
        tile_w = 16 if mode.endswith("_w16") else 0
        base = mode[:-4] if tile_w else mode
        # box3: FIR passes over the three-box taps; box3rs: FP64 running sums
        # (automatic width); box3sl: sliding sums (32-column strips)
        spatial = ("box3" if base.endswith("_box3") else
                   "box3+runsum" if base.endswith(("_box3rs", "_box3sl")) else "gauss")
        if base.endswith("_box3sl"):
            tile_w = 32
        valu = base.endswith("_valu")
        if not args.no_autotune and prec not in tuned:
            # one-off, untimed: measured strip height for this shape
            tuned[prec] = P.bf_autotune(fg, sigma_s, precision=prec, stream=stream)
            log(f"{prec}: autotuned strip height {tuned[prec][0]}")
        for _ in range(args.warmup):
            step(prec, dst, dedup, spatial, valu, tile_w)
        torch.cuda.synchronize()
        kms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            N, ms, K_used, tile_h, tile_w, mf = step(prec, dst, dedup, spatial, valu, tile_w)
            kms.append(ms)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kernel_ms = float(np.mean(kms))
        # flops of the terms the kernel actually ran (Gaussian FIR passes; the
        # three-box filter is a different filter and reports its rate only)
        flops_run = algorithmic_flops_per_pixel(d, R, K_used) * H * W
        tf = None if spatial != "gauss" else flops_run / (kernel_ms * 1e-3) / 1e12
        rec = {"value": H * W * args.steps / dt / 1e6, "ms_per_step": 1e3 * dt / args.steps,
               "kernel_ms": kernel_ms, "kernel_ms_median": float(np.median(kms)),
               "kernel_ms_min": float(np.min(kms)), "kernel_ms_max": float(np.max(kms)),
               "achieved_tflops": tf,
               "frac_of_fp32_peak": None if tf is None else tf / PEAK_FP32_VALU,
               "N": N, "K_used": K_used, "tile_h": tile_h, "tile_w": tile_w,
               "matrix_core_passes": bool(mf), "spatial": spatial,
               "kernel": kernel_name(d, R, prec, tile_w, mf)}
        log(f"{mode}: N={N} K_used={K_used} step {rec['ms_per_step']:.2f} ms, kernel "
            f"{kernel_ms:.2f} ms, " + ("" if tf is None else f"{tf:.2f} TFLOP/s algorithmic, ")
            + f"{rec['value']:.2f} Mpix/s")
        return rec

    flops = algorithmic_flops_per_pixel(d, R, K) * H * W
    precs = [args.precision] if args.only else [args.precision] + \
        [q for q in ("fp32", "fp16", "bf16") if q != args.precision] + \
        ["fp32_split", "fp32_valu", "fp16_valu", "fp32_dedup", "fp16_dedup", "fp32_split_dedup",
         "fp32_box3", "fp32_box3rs", "fp32_box3sl"]
    if args.modes:
        precs = args.modes.split(",")
        args.precision = precs[0].split("_")[0]
    results, outs = {}, {}
    for prec in precs:
        outs[prec] = torch.empty_like(fg)
        log(f"timing {prec}: {args.warmup} warmup + {args.steps} steps")
        results[prec] = run(prec, outs[prec])
    main_mode = precs[0]
    main_rec = results[main_mode]
    N = main_rec["N"]
    # deviation of the 16-bit modes from the FP32 output (fraction of each
    # channel's range), from the same run's outputs
    if "fp32" in outs:
        span = (fg.reshape(-1, d).amax(0) - fg.reshape(-1, d).amin(0)).clamp_min(1e-30)
        for prec in results:
            if prec != "fp32" and results[prec]["spatial"] == "gauss":
                diff = (outs[prec] - outs["fp32"]).abs().reshape(-1, d) / span
                results[prec]["max_dev_vs_fp32"] = float(diff.max())
                results[prec]["mean_dev_vs_fp32"] = float(diff.mean())
    value, kernel_ms, achieved = main_rec["value"], main_rec["kernel_ms"], main_rec["achieved_tflops"]
    assert main_rec["K_used"] == K
    dt = main_rec["ms_per_step"] * args.steps / 1e3

    # host steps of a call, timed on their own (median of 50 calls each, µs):
    # A1 whitening, A2 the min/max reduction (device, with the copy of 2d
    # floats back) and the order rule, A3 the term draws (with whitening)
    def med_us(fn, n=50):
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts) * 1e6)
    lo, hi = P.bf_minmax(fg)
    host_steps = {"A1_whiten_us": med_us(lambda: P.bf_whiten(C)),
                  "A2_minmax_us": med_us(lambda: P.bf_minmax(fg)),
                  "A2_choose_N_us": med_us(lambda: P.bf_choose_N(C, lo, hi)),
                  "A3_sample_terms_us": med_us(lambda: P.bf_sample_terms(C, N, K, seed))}
    log("host steps: " + ", ".join(f"{k} {v:.1f}" for k, v in host_steps.items()))

    # same-GPU comparator: the direct filter of eq. (BF) with the exact
    # Gaussian range kernel on the same image and window
    direct = None
    if not args.only:
        ref = torch.empty_like(fg)
        ms = _timed(lambda: P.bf_direct(fg, sigma_s, C, out=ref), 2)
        span = (fg.reshape(-1, d).amax(0) - fg.reshape(-1, d).amin(0)).clamp_min(1e-30)
        dev = (outs[main_mode] - ref).abs().reshape(-1, d) / span
        direct = {"ms": ms, "mpix_s": H * W / ms / 1e3,
                  "approx_flops_per_pixel": (2 * R + 1) ** 2 * (2 * d + d * d * 2 + 2 * d + 4),
                  "mcsf_vs_direct": {"max_dev": float(dev.max()), "mean_dev": float(dev.mean()),
                                     "mse_db_255": mse_db(outs[main_mode] * 255.0,
                                                          ref * 255.0)}}
        log(f"direct filter: {ms:.1f} ms, {direct['mpix_s']:.1f} Mpix/s; MCSF deviation from it: "
            f"mean {direct['mcsf_vs_direct']['mean_dev']:.3g}, max "
            f"{direct['mcsf_vs_direct']['max_dev']:.3g} of the range")

    serving = variants = None
    if not args.no_serving:
        serving = serving_run(args, P, torch, log)
        if args.serve_variants:
            variants = serving_variants(args, P, torch, log, serving["rate_rps"])

    plans = None
    if not args.no_plan and not args.only:
        plans = plan_run(P, torch, log)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        sp_code = {"gauss": 0, "box3": 3, "box3+runsum": 3}
        cpu = cpu_baseline(f, C, sigma_s, K, seed, N,
                           gpu_outs={m: (outs[m], sp_code[results[m]["spatial"]])
                                     for m in results})
        log(f"cpu baseline {cpu['value']:.4g} Mpix/s ({cpu['sample']}); direct O1 "
            f"{cpu['direct_o1']['value']:.4g} Mpix/s")
        for m, e in cpu["accuracy_vs_oracle"]["modes"].items():
            results[m]["max_err_vs_oracle"] = e["max_err"]
            results[m]["mean_err_vs_oracle"] = e["mean_err"]
            log(f"{m}: error vs the FP64 oracle max {e['max_err']:.3g}, mean {e['mean_err']:.3g}")

    cnt = _counters(args.precision)
    ex_valu = None if cnt is None else cnt["valu_flops"] / (kernel_ms * 1e-3) / 1e12
    ex_mfma = None if cnt is None else cnt["mfma_flops"] / (kernel_ms * 1e-3) / 1e12
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16 storage, f32 accumulate",
                  "bf16": "bf16 storage, f32 accumulate"}[args.precision],
        "modes": results,
        "data": "synthetic",
        "config": {"workload": args.workload, "H": H, "W": W, "d": d, "sigma_s": sigma_s,
                   "window": 2 * R + 1, "K": K, "N": N, "C": "0.08^2 I" if d == 3 else "SPD",
                   "precision": args.precision},
        "roofline": {
            # FP32: the vertical pass, modulation and demodulation run on the
            # VALU, the horizontal pass (32-column strips, R >= 12) on the
            # FP32 matrix cores; both units peak at 157.3 TFLOP/s
            "bound": "alu",
            "kernel": main_rec["kernel"],
            "units": ("VALU + FP32 matrix cores" if main_rec["matrix_core_passes"] and
                      args.precision == "fp32" else
                      "VALU + 16-bit matrix cores" if main_rec["matrix_core_passes"] else "VALU"),
            "achieved": achieved,
            "peak": PEAK_FP32_VALU,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU,
            "frac_vs_nonpacked_fma": achieved / PEAK_FP32_NONPACKED,
            "algorithmic_flops_per_launch": flops,
            "kernel_ms": kernel_ms,
            "traffic": measured_traffic(args.precision),
            "traffic_unit": "bytes per launch",
            "hbm_tb_s": (None if measured_traffic(args.precision) is None else
                         measured_traffic(args.precision) / (kernel_ms * 1e-3) / 1e12),
            # The fields below come from rocprofv3 --pmc counter runs of this
            # kernel build (COUNTERS_PROFILE), not from this run: executed
            # (not algorithmic) flops per launch, over this run's launch time.
            "counters_source": None if cnt is None else COUNTERS_PROFILE,
            "executed_valu_tflops": ex_valu,
            "executed_valu_frac_of_157_3": None if ex_valu is None else ex_valu / PEAK_FP32_VALU,
            "executed_valu_frac_of_nonpacked_78_6": (None if ex_valu is None else
                                                     ex_valu / PEAK_FP32_NONPACKED),
            "executed_matrix_core_tflops": ex_mfma,
        },
        "cpu_baseline": cpu,
        "host_steps": host_steps,
        "direct_comparator": direct,
        "serving": serving,
        "serving_variants": variants,
        "plan": plans,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
