"""Synthetic piecewise-smooth vector images and parameter sets.

The paper evaluates on natural 8-bit colour photographs (Dome 876x584,
Peppers 512x512, House 256x256) that are not available here.  These seeded
generators stand in for them with the same structure: piecewise-smooth regions
separated by sharp edges (a Voronoi partition), smooth shading inside regions
(linear gradients), and sensor-like noise.

Voronoi recipe (all draws from numpy's PCG64 seeded by ``seed``):
  * ``n_cells`` sites uniform over the continuous image rectangle; each pixel
    takes the colour of its nearest site (Euclidean distance);
  * each cell has a base value per channel and, when ``gradient`` is set, a
    linear ramp  value = base + <g, p - site>  with
    g ~ U[-1, 1]^2 * 0.25 * (channel range) / sqrt(H W / n_cells);
  * values are clipped to the channel range, then iid Gaussian noise of the
    given standard deviation is added (not clipped).
"""

import math

import numpy as np
from scipy.spatial import cKDTree


def _cells(H, W, n_cells, rng):
    sites = rng.uniform(0.0, 1.0, size=(n_cells, 2)) * np.array([H, W])
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64),
                         np.arange(W, dtype=np.float64), indexing="ij")
    pts = np.stack([yy.ravel(), xx.ravel()], axis=1)
    _, idx = cKDTree(sites).query(pts, k=1)
    return sites, idx.reshape(H, W), yy, xx


def voronoi_image(H, W, d, n_cells, lo, hi, noise, seed, gradient=True):
    """Piecewise-smooth (H, W, d) float32 image; channel m spans [lo[m], hi[m]]
    before noise.  ``lo``/``hi`` may be scalars."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (d,))
    hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (d,))
    sites, idx, yy, xx = _cells(H, W, n_cells, rng)
    base = rng.uniform(lo, hi, size=(n_cells, d))
    img = base[idx]                                       # (H, W, d)
    if gradient:
        scale = 0.25 * (hi - lo) / math.sqrt(H * W / n_cells)
        g = rng.uniform(-1.0, 1.0, size=(n_cells, 2, d)) * scale
        dy = yy - sites[idx, 0]
        dx = xx - sites[idx, 1]
        img = img + dy[..., None] * g[idx, 0, :] + dx[..., None] * g[idx, 1, :]
    img = np.clip(img, lo, hi)
    if noise > 0:
        img = img + rng.normal(0.0, noise, size=img.shape)
    return img.astype(np.float32)


def lab_like_image(H, W, n_cells, seed):
    """CIE-Lab-like 3-channel image: L in [0, 100], a and b in [-60, 60],
    linear gradients, N(0, 1) noise."""
    return voronoi_image(H, W, 3, n_cells, lo=[0.0, -60.0, -60.0],
                         hi=[100.0, 60.0, 60.0], noise=1.0, seed=seed)


def feature_image(H, W, n_cells, seed, smooth_sigma=32.0):
    """Six correlated channels: three colour channels (piecewise-smooth in
    [0, 1], noise 0.02) and three feature maps 0.5*colour_m + 0.5*S_m, where
    S_m is white noise blurred with a Gaussian of ``smooth_sigma`` pixels and
    rescaled to [0, 1]."""
    from scipy.ndimage import gaussian_filter
    colour = voronoi_image(H, W, 3, n_cells, 0.0, 1.0, 0.02, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    feats = []
    for m in range(3):
        S = gaussian_filter(rng.standard_normal((H, W)), smooth_sigma, mode="wrap")
        S = (S - S.min()) / (S.max() - S.min())
        feats.append(0.5 * colour[..., m] + 0.5 * S)
    return np.concatenate([colour, np.stack(feats, axis=-1).astype(np.float32)],
                          axis=-1).astype(np.float32)


def random_spd(d, log10_lo, log10_hi, seed):
    """C = Q diag(10^u) Q^T with u ~ U[log10_lo, log10_hi] and Q from the QR
    factorisation of a d x d standard normal matrix (signs fixed so that the
    triangular factor has a positive diagonal)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((d, d))
    Q, Rm = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(Rm))[None, :]
    ev = 10.0 ** rng.uniform(log10_lo, log10_hi, size=d)
    C = (Q * ev[None, :]) @ Q.T
    return 0.5 * (C + C.T)


# ---------------------------------------------------------------------------
# The workloads (sizes, value distributions and parameters)
# ---------------------------------------------------------------------------

WORKLOADS = {
    "voronoi128_d3_s2_K64": dict(
        H=128, W=128, d=3, sigma_s=2.0, K=64, image_seed=1001, term_seed=2001,
        desc="128x128x3 in [0,1], 16 Voronoi cells, flat colours, noise 0.02, "
             "sigma_s=2, C=0.1^2 I, K=64"),
    "lab1024_d3_s5_K128": dict(
        H=1024, W=1024, d=3, sigma_s=5.0, K=128, image_seed=1002, term_seed=2002,
        desc="1024x1024x3 Lab-like (L in [0,100], a,b in [-60,60]), 64 cells with "
             "gradients, noise N(0,1), sigma_s=5, full SPD C, K=128"),
    "voronoi4096_d3_s10_K256": dict(
        H=4096, W=4096, d=3, sigma_s=10.0, K=256, image_seed=1003, term_seed=2003,
        desc="4096x4096x3 in [0,1], 256 cells with gradients, noise 0.02, "
             "sigma_s=10, C=0.08^2 I, K=256"),
    "feature2048_d6_s4_K256": dict(
        H=2048, W=2048, d=6, sigma_s=4.0, K=256, image_seed=1004, term_seed=2004,
        desc="2048x2048x6 (3 colour + 3 smooth feature maps), sigma_s=4, random "
             "SPD C with log-uniform eigenvalues in [1e-3,1e-1], K=256"),
}


def workload(name, H=None, W=None):
    """Return (f, C, params) for a named workload.  ``H``/``W`` override the
    size (same recipe, cell count scaled with the area, at least 4 cells)."""
    p = dict(WORKLOADS[name])
    H0, W0 = p["H"], p["W"]
    H = H0 if H is None else H
    W = W0 if W is None else W
    area = (H * W) / (H0 * W0)
    s = p["image_seed"]
    if name.startswith("voronoi128"):
        n = max(4, round(16 * area))
        f = voronoi_image(H, W, 3, n, 0.0, 1.0, 0.02, s, gradient=False)
        C = np.eye(3) * 0.1 ** 2
    elif name.startswith("lab1024"):
        n = max(4, round(64 * area))
        f = lab_like_image(H, W, n, s)
        C = np.array([[100.0, 0.0, 0.0], [0.0, 25.0, 12.5], [0.0, 12.5, 25.0]])
    elif name.startswith("voronoi4096"):
        n = max(4, round(256 * area))
        f = voronoi_image(H, W, 3, n, 0.0, 1.0, 0.02, s)
        C = np.eye(3) * 0.08 ** 2
    elif name.startswith("feature2048"):
        n = max(4, round(128 * area))
        f = feature_image(H, W, n, s, smooth_sigma=32.0 * math.sqrt(area) if area < 1 else 32.0)
        C = random_spd(6, -3.0, -1.0, s + 1)
    else:
        raise KeyError(name)
    p.update(H=H, W=W)
    return f, C, p


def serving_requests(n, seed=5, rate_hz=1.0, side_lo=256, side_hi=2048):
    """Request stream for the serving workload: Poisson arrivals at
    ``rate_hz``; square images of side round(exp U[ln side_lo, ln side_hi]);
    d in {3, 6}; sigma_s uniform in {2..8}; C = sigma_r^2 I with
    sigma_r ~ U[0.05, 0.2]; K in {64, 128, 256}.  Images are drawn lazily from
    the per-request seed (cfg3-style for d = 3, cfg4-style for d = 6, with
    max(16, side^2/65536) cells).  Returns a list of dicts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        side = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        d = int(rng.choice([3, 6]))
        sigma_s = float(rng.integers(2, 9))
        sigma_r = float(rng.uniform(0.05, 0.2))
        K = int(rng.choice([64, 128, 256]))
        reqs.append(dict(id=i, arrival=t, H=side, W=side, d=d, sigma_s=sigma_s,
                         sigma_r=sigma_r, K=K, image_seed=100000 + i,
                         term_seed=200000 + i,
                         n_cells=max(16, side * side // 65536)))
    return reqs


def request_image(req):
    """The image of one serving request (see ``serving_requests``)."""
    H, W, n = req["H"], req["W"], req["n_cells"]
    if req["d"] == 3:
        return voronoi_image(H, W, 3, n, 0.0, 1.0, 0.02, req["image_seed"])
    return feature_image(H, W, n, req["image_seed"], smooth_sigma=32.0)
