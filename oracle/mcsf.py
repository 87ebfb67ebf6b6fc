"""Reference (oracle) implementation of the MCSF, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

Paper: Ghosh & Chaudhury, "Fast Bilateral Filtering of Vector-Valued Images",
arXiv 1605.02164.  Equation names below are the paper's labels.

Layout convention: an image ``f`` is an (H, W, d) float64 array, row-major,
channels last.  ``C`` is a (d, d) SPD covariance.  A term table ``w`` is a
(K, d) array of frequency vectors with theta_t(i) = <w_t, f(i)>.

Readings of the paper taken here (the paper is silent or ambiguous):
  * window radius R = ceil(3 sigma_s) (Section 1, square window
    [-3 sigma_s, 3 sigma_s]^2); sigma_s = 0 gives R = 0, the identity;
  * the other spatial filters the paper allows in place of the Gaussian
    (Section 3, remark after Algorithm 1: box or hat filters, any spatial
    filter) are taken as n-fold convolutions of a box of width 2r + 1 (n = 1
    box, n = 2 hat, n = 3 the usual three-box stand-in for a Gaussian), with r
    the integer whose variance n((2r+1)^2 - 1)/12 is nearest sigma_s^2;
  * the spatial kernel is unnormalised (it cancels in the ratio);
  * out-of-domain pixels contribute nothing to numerator or normaliser
    (the sums of eqs. (BF)/(normal) run over i - j in Omega);
  * the estimator keeps the real parts of the complex accumulators P and Z of
    Algorithm 1, i.e. psi_K(D) = (1/K) sum_t cos<w_t, D>;
  * order N is chosen per image by the aliasing rule in ``choose_order`` unless
    given;
  * the Bernoulli bits of X ~ B(N, 1/2) come from Philox4x32-10 (``draw_binomial``).
"""

import math

import numpy as np

from .philox import philox4x32_10

# ---------------------------------------------------------------------------
# Spatial kernel (eq. (kernel), Section 1 window)
# ---------------------------------------------------------------------------


def box_radius(sigma_s, n):
    """Half-width r of the box whose n-fold convolution stands in for the
    Gaussian of standard deviation sigma_s: the variance of one box of width
    2r + 1 is ((2r+1)^2 - 1)/12, so r solves n((2r+1)^2 - 1)/12 = sigma_s^2,
    rounded to the nearest integer (halves up)."""
    x = (math.sqrt(12.0 * float(sigma_s) ** 2 / n + 1.0) - 1.0) / 2.0
    return int(math.floor(x + 0.5))


def window_radius(sigma_s, spatial=0):
    """Gaussian (spatial = 0): R = ceil(3 sigma_s), the sums of eqs.
    (BF)/(normal) are restricted to the square window [-3 sigma_s, 3 sigma_s]^2
    (Section 1).  n-fold box (spatial = n): R = n r, the support of the
    filter."""
    if spatial:
        return spatial * box_radius(sigma_s, spatial)
    if sigma_s == 0:
        return 0
    return int(math.ceil(3.0 * float(sigma_s)))


def spatial_taps(sigma_s, spatial=0):
    """One-dimensional factor omega_1(u), u = -R..R, of the separable spatial
    filter omega(j) = omega_1(j_y) * omega_1(j_x).  Unnormalised.
    spatial = 0: omega_1(u) = exp(-u^2 / (2 sigma_s^2)) (eq. (kernel)).
    spatial = n in {1, 2, 3}: the n-fold convolution of the box of ones of
    width 2r + 1 (r from ``box_radius``): box, hat, three boxes."""
    if spatial:
        r = box_radius(sigma_s, spatial)
        taps = np.ones(1)
        for _ in range(spatial):
            taps = np.convolve(taps, np.ones(2 * r + 1))
        return taps
    R = window_radius(sigma_s)
    if R == 0:
        return np.ones(1)
    u = np.arange(-R, R + 1, dtype=np.float64)
    return np.exp(-(u * u) / (2.0 * float(sigma_s) ** 2))


# ---------------------------------------------------------------------------
# Range-space whitening (eq. (COB), Algorithm 1, diagonalisation step)
# ---------------------------------------------------------------------------


def check_covariance(C):
    """C must be symmetric positive definite (eq. (kernel))."""
    C = np.asarray(C, dtype=np.float64)
    if C.ndim != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("C must be square")
    scale = np.max(np.abs(C))
    if not np.all(np.isfinite(C)) or scale == 0:
        raise ValueError("C must be finite and nonzero")
    if np.max(np.abs(C - C.T)) > 1e-12 * scale:
        raise ValueError("C must be symmetric")
    if np.min(np.linalg.eigvalsh(C)) <= 0:
        raise ValueError("C must be positive definite")
    return C


WHITEN_EIG, WHITEN_CHOL, WHITEN_SYM = 0, 1, 2


def whiten(C, mode=WHITEN_EIG):
    """Whitening W with W^T W = C^{-1}.

    mode = WHITEN_EIG (default) follows eq. (COB), below.  The other two are
    the other standard square roots of C^{-1}: WHITEN_CHOL, W = L^{-1} with
    C = L L^T (L lower triangular with positive diagonal); WHITEN_SYM,
    W = C^{-1/2}, the symmetric positive definite root.  All three give the
    same Gaussian kernel of eq. (kernel); at finite N the product of raised
    cosines of eq. (approx) depends on the choice.

    WHITEN_EIG, following eq. (COB):

    C^{-1} = Q diag(alpha^2) Q^T with Q orthogonal; row k of W is
    alpha_k q_k^T, so that (W x)_k = alpha_k y_k with y = Q^T x.

    The eigen-decomposition is not unique; this project fixes it:
      * a diagonal C (all off-diagonals exactly zero) gives Q = I in channel
        order, alpha_k = C_kk^{-1/2} (the case the paper uses: Section 4,
        isotropic C gives Q = I and alpha_k = 1/sigma_r);
      * otherwise eigenpairs of C are taken in ascending eigenvalue order and
        each eigenvector is signed so that its first component whose magnitude
        exceeds 1e-6 of the vector's largest magnitude is positive.
    """
    C = check_covariance(C)
    d = C.shape[0]
    off = C - np.diag(np.diag(C))
    if not np.any(off):
        return np.diag(1.0 / np.sqrt(np.diag(C)))
    if mode == WHITEN_CHOL:
        L = np.linalg.cholesky(C)
        # W = L^{-1} by forward substitution (L W = I), column by column
        W = np.zeros((d, d))
        for j in range(d):
            for i in range(j, d):
                rhs = (1.0 if i == j else 0.0) - sum(L[i, k] * W[k, j] for k in range(j, i))
                W[i, j] = rhs / L[i, i]
        return W
    lam, V = np.linalg.eigh(C)          # ascending eigenvalues
    if mode == WHITEN_SYM:
        return (V / np.sqrt(lam)) @ V.T
    if mode != WHITEN_EIG:
        raise ValueError("unknown whitening mode")
    W = np.empty((d, d))
    for k in range(d):
        v = V[:, k].copy()
        big = np.abs(v) > 1e-6 * np.max(np.abs(v))
        first = int(np.argmax(big))
        if v[first] < 0:
            v = -v
        W[k, :] = v / math.sqrt(lam[k])
    return W


# ---------------------------------------------------------------------------
# Order N (eq. (approx)); the paper picks N by hand
# ---------------------------------------------------------------------------


def choose_order(f, W, n_min=10):
    """Order rule used when N is not given.

    cos(z / sqrt(N))^N approximates exp(-z^2/2) (Proposition 1) only for
    |z| < pi sqrt(N); at z = pi sqrt(N) it aliases back to magnitude one.  The
    whitened difference z = W (f(i-j) - f(i)) satisfies
    |z_k| <= T_k = sum_m |W_km| (hi_m - lo_m), with lo/hi the per-channel
    extrema of the image.  N is the smallest order with
    pi sqrt(N) >= max_k T_k + 4 (alias lobe suppressed to exp(-8) over the data
    range), and at least ``n_min`` (the paper's N = 10).
    """
    f = np.asarray(f, dtype=np.float64)
    d = f.shape[-1]
    flat = f.reshape(-1, d)
    span = flat.max(axis=0) - flat.min(axis=0)
    T = float(np.max(np.abs(W) @ span))
    return max(int(n_min), int(math.ceil(((T + 4.0) / math.pi) ** 2)))


# ---------------------------------------------------------------------------
# Monte Carlo draws (Proposition 2, eq. (finalApproxY), Algorithm 1, draw step)
# ---------------------------------------------------------------------------


def draw_binomial(seed, K, d, N):
    """X[t, m] ~ B(N, 1/2), independent over (t, m) (Proposition 2).

    X[t, m] is the number of set bits among the first N bits of the Philox
    stream for (t, m): bit i of the stream is bit (i mod 32) of word
    (i div 32); word q is output lane (q mod 4) of
    Philox4x32-10(counter = (t, m, q div 4, 0), key = (seed lo32, seed hi32)).
    """
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = (seed & 0xFFFFFFFF, seed >> 32)
    nwords = (N + 31) // 32
    nblocks = (nwords + 3) // 4
    t, m, b = np.meshgrid(np.arange(K), np.arange(d), np.arange(nblocks),
                          indexing="ij")
    ctr = np.stack([t.ravel(), m.ravel(), b.ravel(), np.zeros(t.size, np.int64)],
                   axis=1).astype(np.uint32)
    words = philox4x32_10(ctr, key).reshape(K, d, nblocks * 4)[:, :, :nwords]
    rem = N - 32 * (nwords - 1)             # bits used from the last word
    words = words.astype(np.uint64)
    if rem < 32:
        words[:, :, -1] &= np.uint64((1 << rem) - 1)
    X = np.zeros((K, d), dtype=np.int64)
    for bit in range(32):
        X += ((words >> np.uint64(bit)) & np.uint64(1)).sum(axis=2).astype(np.int64)
    return X


def sample_terms(C, N, K, seed, W=None):
    """Y[t] = N - 2 X[t] (eq. (finalApproxY)) and the frequency vectors
    w_t = W^T Y_t / sqrt(N), so that
    <w_t, f(i)> = sum_k Y_k gamma_k g_k(i) with g = Q^T f, gamma_k = alpha_k/sqrt(N)
    (Proposition 2, eqs. (Ht), (bigExp))."""
    if W is None:
        W = whiten(C)
    d = W.shape[0]
    X = draw_binomial(seed, K, d, N)
    Y = N - 2 * X
    w = (Y.astype(np.float64) @ W) / math.sqrt(N)
    return Y, w


# ---------------------------------------------------------------------------
# Range kernels
# ---------------------------------------------------------------------------


def psi_gauss(Delta, C):
    """phi(x) = exp(-x^T C^{-1} x / 2), eq. (kernel); C^{-1} by a linear solve,
    independent of the whitening."""
    C = np.asarray(C, dtype=np.float64)
    sol = np.linalg.solve(C, Delta.reshape(-1, C.shape[0]).T).T
    q = np.sum(Delta.reshape(-1, C.shape[0]) * sol, axis=1)
    return np.exp(-0.5 * q).reshape(Delta.shape[:-1])


def psi_raised_cosine(Delta, W, N):
    """Order-N kernel of eq. (approx): prod_k cos((W Delta)_k / sqrt(N))^N."""
    z = Delta @ W.T
    return np.prod(np.cos(z / math.sqrt(N)) ** N, axis=-1)


def psi_sampled(Delta, w, weights=None):
    """Real part of the Monte Carlo kernel of eq. (finalApproxY):
    (1/K) sum_t cos<w_t, Delta> (or the weighted mean with ``weights``)."""
    c = np.cos(Delta @ w.T)
    if weights is None:
        return c.mean(axis=-1)
    weights = np.asarray(weights, dtype=np.float64)
    return (c @ weights) / weights.sum()


# ---------------------------------------------------------------------------
# Direct evaluation of eqs. (BF)/(normal) with a given range kernel
# ---------------------------------------------------------------------------


def _direct(f, sigma_s, kernel, pixels=None, spatial=0):
    """out(i) = sum_j omega(j) k(f(i-j) - f(i)) f(i-j) / sum_j omega(j) k(...),
    the sums running over j in [-R, R]^2 with i - j inside the image
    (eqs. (BF), (normal), Section 1 window).  ``kernel`` maps an (..., d) array
    of differences to weights.  Returns (out, Z) for the listed pixels (an
    (n, 2) integer array of (y, x)), or for all pixels as (H, W, d), (H, W)."""
    f = np.asarray(f, dtype=np.float64)
    H, Wd, d = f.shape
    R = window_radius(sigma_s, spatial)
    w1 = spatial_taps(sigma_s, spatial)
    if pixels is None:
        pix = np.stack(np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij"),
                       axis=-1).reshape(-1, 2)
    else:
        pix = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    out = np.empty((len(pix), d))
    Z = np.empty(len(pix))
    for n, (y, x) in enumerate(pix):
        y0, y1 = max(0, y - R), min(H, y + R + 1)
        x0, x1 = max(0, x - R), min(Wd, x + R + 1)
        win = f[y0:y1, x0:x1, :]
        sw = np.outer(w1[y0 - y + R:y1 - y + R], w1[x0 - x + R:x1 - x + R])
        wt = sw * kernel(win - f[y, x, :])
        Z[n] = wt.sum()
        out[n] = np.tensordot(wt, win, axes=([0, 1], [0, 1])) / Z[n]
    if pixels is None:
        return out.reshape(H, Wd, d), Z.reshape(H, Wd)
    return out, Z


def direct_exact(f, sigma_s, C, pixels=None, spatial=0):
    """O1: the bilateral filter of eqs. (BF)/(normal) with the Gaussian range
    kernel of eq. (kernel), evaluated directly (O(sigma_s^2) per pixel)."""
    C = check_covariance(C)
    return _direct(f, sigma_s, lambda D: psi_gauss(D, C), pixels, spatial)


def direct_sampled(f, sigma_s, w, pixels=None, weights=None, spatial=0):
    """O2: eqs. (BF)/(normal) with phi replaced by the sampled kernel
    psi_K(D) = (1/K) sum_t cos<w_t, D> (eqs. (finalApproxY), (bigExp))."""
    w = np.asarray(w, dtype=np.float64)
    return _direct(f, sigma_s, lambda D: psi_sampled(D, w, weights), pixels, spatial)


def direct_raised_cosine(f, sigma_s, W, N, pixels=None):
    """O4 (closed form): eqs. (BF)/(normal) with the order-N product of raised
    cosines of eq. (approx) in whitened coordinates."""
    return _direct(f, sigma_s, lambda D: psi_raised_cosine(D, W, N), pixels)


# ---------------------------------------------------------------------------
# The MCSF itself (Algorithm 1, eqs. (Ht), (numerator), (denom))
# ---------------------------------------------------------------------------


def _gauss_sep(U, w1):
    """Truncated separable Gaussian omega * U over the last two axes of U,
    with zero contribution from outside the image: first along x, then along
    y (separability of omega, eq. (kernel))."""
    R = (len(w1) - 1) // 2
    if R == 0:
        return U * (w1[0] * w1[0])
    Hh, Ww = U.shape[-2:]
    P = np.zeros(U.shape[:-2] + (Hh + 2 * R, Ww + 2 * R))
    P[..., R:R + Hh, R:R + Ww] = U
    V = np.zeros(U.shape[:-2] + (Hh + 2 * R, Ww))
    for u in range(2 * R + 1):
        V += w1[u] * P[..., :, u:u + Ww]
    A = np.zeros(U.shape)
    for u in range(2 * R + 1):
        A += w1[u] * V[..., u:u + Hh, :]
    return A


def mcsf_separable(f, sigma_s, w, weights=None, spatial=0):
    """O3: Algorithm 1 with the term draws given as the table ``w`` (K, d).

    For each term t (Algorithm 1 loop over t):
      H(i) = exp(i <w_t, f(i)>)            (eq. (Ht), with Q and gamma folded into w_t)
      G(i) = H(i) f(i)
      Gbar = omega * G, Hbar = omega * H  (separable, truncated, zero outside Omega)
      P += conj(H) Gbar,  Z += conj(H) Hbar
    and finally out = P / Z (Algorithm 1 last step), keeping real parts:
    Re(conj(H) Gbar) = cos*(omega * cos f) + sin*(omega * sin f).
    A weighted table multiplies term t's contribution by weights[t];
    ``spatial`` selects omega as in ``spatial_taps``.
    Returns (out (H, W, d), num (H, W, d), Z (H, W)).
    """
    f = np.asarray(f, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64).reshape(-1, f.shape[-1])
    H, Wd, d = f.shape
    w1 = spatial_taps(sigma_s, spatial)
    ft = np.moveaxis(f, -1, 0)                      # (d, H, W)
    num = np.zeros((d, H, Wd))
    Z = np.zeros((H, Wd))
    for t in range(w.shape[0]):
        theta = np.tensordot(w[t], ft, axes=(0, 0))  # <w_t, f(i)>
        c, s = np.cos(theta), np.sin(theta)
        U = np.concatenate([c[None], s[None], c[None] * ft, s[None] * ft], axis=0)
        A = _gauss_sep(U, w1)
        wt = 1.0 if weights is None else float(weights[t])
        Z += wt * (c * A[0] + s * A[1])
        num += wt * (c[None] * A[2:2 + d] + s[None] * A[2 + d:])
    out = num / Z[None]
    return np.moveaxis(out, 0, -1), np.moveaxis(num, 0, -1), Z


def full_expansion_terms(W, N):
    """O4 (enumeration): every Y in {-N, -N+2, ..., N}^d with its probability
    prod_k binom(N, (N - Y_k)/2) / 2^N (eqs. (expansion), (exp)); returns the
    frequency table w = Y W / sqrt(N) and the weights."""
    d = W.shape[0]
    n = np.arange(N + 1)
    p1 = np.array([math.comb(N, int(k)) for k in n], dtype=np.float64) / 2.0 ** N
    grids = np.meshgrid(*([n] * d), indexing="ij")
    Xs = np.stack([g.ravel() for g in grids], axis=1)
    Y = N - 2 * Xs
    weights = np.prod(p1[Xs], axis=1)
    w = (Y.astype(np.float64) @ W) / math.sqrt(N)
    return w, weights


def mcsf(f, sigma_s, C, K, seed, N=None):
    """The whole method (Algorithm 1): whiten C, pick N, draw K terms with the
    seed, run the separable filter.  Returns (out, N, Y, w)."""
    W = whiten(C)
    if N is None:
        N = choose_order(f, W)
    Y, w = sample_terms(C, N, K, seed, W=W)
    out, _, _ = mcsf_separable(f, sigma_s, w)
    return out, N, Y, w


# ---------------------------------------------------------------------------
# Accuracy metric (eq. (MSE))
# ---------------------------------------------------------------------------


def mse(a, b):
    """eq. (MSE): mean over channels and pixels of the squared difference."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.mean((a - b) ** 2))


def mse_db(a, b, scale=1.0):
    """10 log10(MSE) of the images multiplied by ``scale`` (255 for [0, 1]
    images, to compare with the paper's 8-bit dB figures)."""
    return 10.0 * math.log10(mse(scale * np.asarray(a), scale * np.asarray(b)))
