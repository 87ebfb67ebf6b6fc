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


def sample_pixels(H, W, n, seed, R=0):
    """n seeded pixel coordinates (y, x): the four corners, pixels within R of
    the borders, and uniform interior draws."""
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1)}
    k = max(0, n // 4)
    for _ in range(k):
        pts.add((int(rng.integers(0, min(H, R + 1))), int(rng.integers(0, W))))
        pts.add((int(rng.integers(max(0, H - R - 1), H)), int(rng.integers(0, W))))
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, min(W, R + 1)))))
    while len(pts) < n:
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, W))))
    return np.array(sorted(pts), dtype=np.int64)


def rel_err_per_channel(got, ref, f):
    """max |got - ref| per channel divided by the input's channel range."""
    f = np.asarray(f, dtype=np.float64).reshape(-1, f.shape[-1])
    rng = f.max(axis=0) - f.min(axis=0)
    rng[rng == 0] = 1.0
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    d = d.reshape(-1, d.shape[-1])
    return d.max(axis=0) / rng
