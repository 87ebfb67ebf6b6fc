"""Shared helpers of the test suite (no filter arithmetic here)."""

import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    """Names of the functions declared in include/bfvec.h."""
    text = open(os.path.join(ROOT, "include", "bfvec.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bf_[A-Za-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def sample_pixels(H, W, n, seed, R=0, seams_y=(), seams_x=()):
    """Seeded pixel coordinates (y, x), sorted and distinct: the four
    corners; n // 4 pixels in each of the four border bands of width R + 1
    (top, bottom, left, right); for every strip seam (a first row or column
    of a strip, from ``seams_y`` / ``seams_x``) the pixel pairs on both sides
    of it at a random position along it; then uniform draws up to at least n
    pixels in all."""
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1)}
    k = max(0, n // 4)
    for _ in range(k):
        pts.add((int(rng.integers(0, min(H, R + 1))), int(rng.integers(0, W))))
        pts.add((int(rng.integers(max(0, H - R - 1), H)), int(rng.integers(0, W))))
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, min(W, R + 1)))))
        pts.add((int(rng.integers(0, H)), int(rng.integers(max(0, W - R - 1), W))))
    for y in seams_y:
        if 0 < y < H:
            x = int(rng.integers(0, W))
            pts.update({(y - 1, x), (y, x)})
    for x in seams_x:
        if 0 < x < W:
            y = int(rng.integers(0, H))
            pts.update({(y, x - 1), (y, x)})
    while len(pts) < n:
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, W))))
    return np.array(sorted(pts), dtype=np.int64)


def corner_blocks(H, W, R):
    """Every pixel within R of an image corner: the four min(R, H) x min(R, W)
    corner blocks."""
    ry, rx = min(R, H), min(R, W)
    ys = list(range(ry)) + list(range(H - ry, H))
    xs = list(range(rx)) + list(range(W - rx, W))
    return np.array(sorted({(y, x) for y in ys for x in xs}), dtype=np.int64).reshape(-1, 2)


def strip_seams(n, size):
    """First rows (or columns) of every strip after the first, for strips of
    ``size`` over an extent of n."""
    return list(range(size, n, size))


def merge_pixels(*sets):
    """Union of (y, x) pixel arrays, sorted."""
    pts = {tuple(int(v) for v in p) for s in sets for p in np.asarray(s).reshape(-1, 2)}
    return np.array(sorted(pts), dtype=np.int64).reshape(-1, 2)


def parallel_pixels(fn, pixels, threads=None):
    """Evaluate fn(pixels_chunk) -> (values, Z) over chunks of the pixel list
    in a thread pool (numpy releases the GIL in its kernels; BLAS limited to
    one thread per worker) and concatenate.  Test-side scheduling only: fn is
    called on disjoint pixel subsets exactly as on the whole list."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    chunks = [c for c in np.array_split(np.asarray(pixels), 4 * threads) if len(c)]
    with threadpool_limits(limits=1), ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(fn, chunks))
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])


def rel_err_per_channel(got, ref, f):
    """max |got - ref| per channel divided by the input's channel range."""
    f = np.asarray(f, dtype=np.float64).reshape(-1, f.shape[-1])
    rng = f.max(axis=0) - f.min(axis=0)
    rng[rng == 0] = 1.0
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    d = d.reshape(-1, d.shape[-1])
    return d.max(axis=0) / rng
