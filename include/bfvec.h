/*
 * bfvec.h -- C ABI of the MI355X (gfx950) Monte Carlo Shiftable Filter.
 *
 * The filter is the fast vector-valued bilateral filter of Ghosh & Chaudhury,
 * "Fast Bilateral Filtering of Vector-Valued Images" (arXiv 1605.02164):
 * the Gaussian range kernel phi(x) = exp(-x^T C^{-1} x / 2) of eq. (kernel) is
 * whitened (eq. (COB)), replaced by a product of order-N raised cosines
 * (eq. (approx)), expanded stochastically (Proposition 2) and estimated with K
 * Monte Carlo terms (eq. (finalApproxY)); each term modulates the image,
 * filters d+1 complex channels with the truncated separable Gaussian omega of
 * eq. (kernel), and demodulates into a numerator and normaliser
 * (eqs. (numerator), (denom)); one division ends Algorithm 1.
 *
 * Conventions for every entry point
 *   - Images are float32, row-major, channels last ("HWC"): element (y, x, m)
 *     sits at index (y*W + x)*d + m.  Image pointers named f/out are DEVICE
 *     pointers owned by the caller; out must not overlap f.
 *   - C is a HOST pointer to a d x d float64 row-major symmetric positive
 *     definite covariance.
 *   - Window radius R = ceil(3*sigma_s) (square window [-3 sigma_s, 3 sigma_s]^2
 *     of the paper's Section 1); sigma_s = 0 is the identity filter.
 *   - Pixels outside the image contribute nothing to numerator or normaliser.
 *   - The estimator keeps real parts: out = Re(P) / Re(Z) (Algorithm 1, last
 *     step), which is the paper's estimator on the symmetric sample {+Y, -Y}.
 *   - Every call returns a status (BF_OK = 0).  On failure nothing has been
 *     written to out, and bf_last_error() gives a message (thread-local).
 *     Argument errors are detected before any device work.  HIP failures
 *     return BF_EDEVICE.
 *   - The library allocates only small per-call device buffers (term table,
 *     taps, reduction partials) in stream order; the caller owns images.
 *   - Limits: 1 <= H, W <= 65536; 1 <= d <= 8; 0 <= sigma_s <= 32 (R <= 96);
 *     1 <= K <= 65536; 1 <= N <= 65536.
 */
#ifndef BFVEC_H
#define BFVEC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BF_OK = 0,
  BF_EINVAL = 1,        /* bad argument (size, pointer, range)            */
  BF_ENOTSPD = 2,       /* C not symmetric positive definite               */
  BF_ENOMEM = 3,        /* device or host allocation failed                */
  BF_EDEVICE = 4,       /* HIP runtime error                               */
  BF_EUNSUPPORTED = 5,  /* option not supported for these sizes            */
  BF_EBUSY = 6          /* serving queue full                              */
};

/* Storage type of the modulated channels and of the horizontal-pass
 * intermediates.  Accumulation of both passes and of num/Z is FP32 always. */
enum { BF_FP32 = 0, BF_FP16 = 1, BF_BF16 = 2 };

typedef struct bf_opts {
  int N;           /* raised-cosine order (eq. (approx)); 0 = automatic rule  */
  int precision;   /* BF_FP32 (default), BF_FP16, BF_BF16                      */
  int center;      /* 1 (default): phase taken on f - c with c the per-channel
                      midpoint (exact in arithmetic: the filter commutes with
                      constant shifts); 0: phase on f itself                   */
  int tile_h;      /* strip height in rows; 0 = automatic                      */
  void* stream;    /* hipStream_t for all device work; NULL = null stream      */
  float* num_out;  /* optional DEVICE H*W*d numerator Re(P), or NULL           */
  float* z_out;    /* optional DEVICE H*W normaliser Re(Z), or NULL            */
  int N_used;      /* OUT: the order actually used                             */
  int time_kernel; /* 1: time the fused kernel with HIP events on `stream` and
                      wait for it (fills kernel_ms); 0 (default): no timing      */
  float kernel_ms; /* OUT: fused-kernel duration in ms when time_kernel = 1     */
  int reserved[5];
} bf_opts;

/* Fill *o with the defaults (N auto, FP32, centring on, automatic tiles,
 * null stream, no debug outputs). */
void bf_opts_init(bf_opts* o);

/* The filter, synchronous.  Algorithm 1 with the K terms drawn from `seed`
 * and the order N chosen by the automatic rule (see bf_choose_N).
 * f, out: device HWC float32.  C: host d x d float64.  Returns when out is
 * complete. */
int bf_vec(const float* f, int H, int W, int d, double sigma_s,
           const double* C, int K, uint64_t seed, float* out);

/* Same, with options.  All device work is queued on o->stream.  When N is
 * automatic or centring is on, the call first reduces per-channel min/max on
 * the device and waits for that reduction (a few tens of microseconds);
 * otherwise it returns without waiting.  o->N_used is written. */
int bf_vec_ex(const float* f, int H, int W, int d, double sigma_s,
              const double* C, int K, uint64_t seed, float* out, bf_opts* o);

/* The filter with an explicit term table instead of drawn terms:
 * w: HOST K x d float64 frequency vectors (radians per unit of f), so term t
 * modulates by exp(i <w_t, f(i)>) (eqs. (Ht), (bigExp)); weights: HOST K
 * float64 nonnegative term weights, or NULL for equal weights.  With the full
 * binomially weighted table this evaluates the unsampled expansion of
 * eq. (expansion).  o may be NULL (defaults). */
int bf_vec_terms(const float* f, int H, int W, int d, double sigma_s,
                 const double* w, const double* weights, int K, float* out,
                 bf_opts* o);

/* Whitening of eq. (COB), host only: W (d x d row-major, host) with
 * W^T W = C^{-1}; row k is alpha_k q_k^T.  Diagonal C gives
 * W = diag(C_kk^{-1/2}); otherwise eigenpairs of C in ascending eigenvalue
 * order, each eigenvector signed so that its first component larger than
 * 1e-6 of its largest magnitude is positive.  BF_ENOTSPD if C is not
 * symmetric (to 1e-12 relative) or not positive definite. */
int bf_whiten(int d, const double* C, double* W);

/* Monte Carlo draws of Proposition 2, host only.  X[t][m] ~ B(N, 1/2) is the
 * number of set bits among the first N bits of the Philox4x32-10 stream with
 * key (seed lo32, seed hi32) and counters (t, m, q, 0), q = 0, 1, ...; word
 * 4q + l of the stream is output lane l of counter q; bit i of the stream is
 * bit (i mod 32) of word (i div 32).  Y = N - 2X (eq. (finalApproxY));
 * w[t] = W^T Y[t] / sqrt(N) with W from bf_whiten.  Y (K x d int32) and w
 * (K x d float64) are host arrays; either may be NULL. */
int bf_sample_terms(int d, const double* C, int N, int K, uint64_t seed,
                    int32_t* Y, double* w);

/* Order rule, host only: with spans s_m = hi[m] - lo[m] and T = max_k
 * sum_m |W_km| s_m (the largest whitened difference in the image), N is the
 * smallest integer with pi*sqrt(N) >= T + 4, and at least 10.  lo/hi are host
 * arrays of d floats.  BF_EUNSUPPORTED if that N exceeds 65536. */
int bf_choose_N(int d, const double* W, const float* lo, const float* hi, int* N);

/* Per-channel minimum and maximum of a device HWC image, written to host
 * arrays lo/hi (d floats each).  Synchronous on `stream` (NULL = null
 * stream).  BF_EINVAL if the image holds a NaN or infinity. */
int bf_minmax(const float* f, int H, int W, int d, float* lo, float* hi,
              void* stream);

/* Direct evaluation of eqs. (BF)/(normal) on the GPU with the exact Gaussian
 * range kernel (O(sigma_s^2) work per pixel; the paper's comparison method).
 * Same layout, window and boundary rules as bf_vec.  Synchronous. */
int bf_direct(const float* f, int H, int W, int d, double sigma_s,
              const double* C, float* out);

/* Message for the last failing call on this thread ("" if none). */
const char* bf_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int bf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BFVEC_H */
