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
 *   - Limits: 1 <= H, W <= 65536; 1 <= d <= 8; 1 <= K <= 65536;
 *     1 <= N <= 65536; the fused filter takes window radii R <= 40
 *     (sigma_s <= 13.33) and images with H*W*(d+1) below 2^30 elements
 *     (BF_EUNSUPPORTED otherwise); bf_direct takes R <= 96.
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
  BF_EBUSY = 6,         /* serving queue full                              */
  BF_ETIMEDOUT = 7      /* a wait ended before the request finished        */
};

/* Storage type of the modulated channels and of the horizontal-pass
 * intermediates.  Accumulation of both passes and of num/Z is FP32 always.
 * BF_FP32_SPLIT: FP32 channels and horizontal pass, with the horizontal-pass
 * rows kept as FP16 pairs hi + lo (about 22 significant bits; hi = the value
 * rounded to FP16, lo = the remainder rounded) and the vertical pass as exact
 * FP16 products hi.hi + lo.hi + hi.lo on the matrix cores, so that it leaves
 * the FP32 datapath the horizontal pass and the modulation use.  Errors
 * against the FP64 reference measure the same as BF_FP32's.  Exists for
 * d = 3, window radius 18, 21, 24 or 30 (the Gaussian's sigma_s 6, 7, 8, 10) and
 * W >= 32 (else BF_EUNSUPPORTED), not with valu_only; its FP16 halves need
 * the FP16 range rule of BF_FP16 (checked where the image's range is known:
 * bf_vec_ex and the server, not plans, as for BF_FP16).  (3 and 4 are not
 * precisions.) */
enum { BF_FP32 = 0, BF_FP16 = 1, BF_BF16 = 2, BF_FP32_SPLIT = 5 };

/* Whitening W with W^T W = C^{-1} (eq. (COB) fixes W only up to that): the
 * eigen-decomposition of eq. (COB) (default, see bf_whiten), W = L^{-1} with
 * C = L L^T (Cholesky), or the symmetric root W = C^{-1/2}.  The three give
 * the same Gaussian range kernel; at finite N the product of raised cosines
 * of eq. (approx) is not rotation invariant, so the filters differ slightly.
 * All three coincide for diagonal C. */
enum { BF_WHITEN_EIG = 0, BF_WHITEN_CHOL = 1, BF_WHITEN_SYM = 2 };

/* Spatial filter omega (separable, unnormalised).  The paper's eq. (kernel)
 * Gaussian by default; Section 3 allows any spatial filter in its place, such
 * as a box or a hat.  BF_SPATIAL_BOX / HAT / BOX3 are the 1-, 2- and 3-fold
 * convolutions of a box of 2r+1 ones per axis, with r the integer nearest the
 * root of n((2r+1)^2 - 1)/12 = sigma_s^2 (n boxes have variance sigma_s^2),
 * window radius R = n r.  Both passes run as FIR passes over these taps.
 * BF_SPATIAL_RUNSUM (or-ed into a box value, BF_FP32 only) runs the vertical
 * pass as exact running sums instead, whose cost does not depend on sigma_s
 * (the paper's O(1) remark): FP64 running sums in 16-column strips, or, for
 * BF_SPATIAL_BOX3 at d = 3 with tile_w = 32 at a compile-time radius, three
 * cascaded sliding box sums with the horizontal pass on the matrix cores.
 * On MI355X both are slower than the FIR pass for every supported window
 * (R <= 40), so neither is the default. */
enum { BF_SPATIAL_GAUSS = 0, BF_SPATIAL_BOX = 1, BF_SPATIAL_HAT = 2, BF_SPATIAL_BOX3 = 3,
       BF_SPATIAL_RUNSUM = 16 };

typedef struct bf_opts {
  int N;           /* raised-cosine order (eq. (approx)); 0 = automatic rule  */
  int precision;   /* BF_FP32 (default), BF_FP16, BF_BF16, BF_FP32_SPLIT       */
  int center;      /* 1 (default): phase taken on f - c with c the per-channel
                      midpoint (exact in arithmetic: the filter commutes with
                      constant shifts); 0: phase on f itself                   */
  int tile_h;      /* strip height in rows; 0 = automatic.  Rounded up to a
                      multiple of 8 rows; tile_h_used reports what ran        */
  void* stream;    /* hipStream_t for all device work; NULL = null stream      */
  float* num_out;  /* optional DEVICE H*W*d numerator Re(P), or NULL           */
  float* z_out;    /* optional DEVICE H*W normaliser Re(Z), or NULL            */
  int N_used;      /* OUT: the order actually used                             */
  int time_kernel; /* 1: time the fused kernel with HIP events on `stream` and
                      wait for it (fills kernel_ms); 0 (default): no timing      */
  float kernel_ms; /* OUT: fused-kernel duration in ms when time_kernel = 1     */
  int dedup;       /* 1: merge draws with equal Y or equal -Y into one weighted
                      term before filtering (bf_vec_ex only).  Exact in
                      arithmetic: a term's real part is even in Y, so the sum
                      over the K draws equals the multiplicity-weighted sum over
                      the distinct +-Y.  0 (default): K terms as drawn          */
  int K_used;      /* OUT: terms the kernel ran (K, or the distinct +-Y count)  */
  int tile_h_used; /* OUT: strip height the fused kernel ran with              */
  int spatial;     /* BF_SPATIAL_* (default BF_SPATIAL_GAUSS), optionally
                      | BF_SPATIAL_RUNSUM with a box filter and BF_FP32       */
  int whiten;      /* BF_WHITEN_* (default BF_WHITEN_EIG)                      */
  int tile_w;      /* strip width in columns: 0 = automatic (default), 16, or
                      32.  32 needs d = 3, a window radius with a compile-time
                      kernel (6, 9, 12, 15, 18, 21, 24 or 30: the Gaussian's
                      3 sigma_s), BF_FP32/FP16/BF16 (with BF_SPATIAL_RUNSUM:
                      BF_SPATIAL_BOX3 and a radius that is a multiple of 3),
                      and W >= 32 (else BF_EUNSUPPORTED); automatic picks 32
                      there unless it cuts resident waves per CU below 3/4 or
                      the image is too small to fill the GPU (fewer than two
                      16-column, 8-row strips per compute unit);
                      BF_FP32_SPLIT runs 32 only.  At these
                      radii the passes run as banded matrix products on the
                      matrix cores: both with FP16/BF16 storage (either
                      width), and for FP32 in 32-column strips the horizontal
                      one from a radius of 12 up and both from 21 up; these
                      sum the taps in another order than 16-column strips, so
                      FP32 results there differ between widths by rounding
                      only.  Otherwise the
                      width changes no output bit.  bf_vec_ex, plans and the
                      server agree bit for bit at equal width.                */
  int tile_w_used; /* OUT: strip width the fused kernel ran with (16 or 32)   */
  int valu_only;   /* 1: run both separable passes on the vector ALUs (FMA /
                      v_dot2 sliding windows), never on the matrix cores; 0
                      (default): matrix-core passes where tile_w describes
                      them.  16-bit results are the same bits either way only
                      up to rounding of the pass sums                       */
  int mfma_used;   /* OUT: 1 if a pass ran on the matrix cores, else 0        */
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

/* Size of the device scratch array of bf_vec_static (per GPU, held for the
 * life of the process). */
#define BF_STATIC_SCRATCH_BYTES (64u << 20)

/* bf_vec_ex without any device allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, options, results (the
 * same bits as bf_vec_ex) and errors, except:
 *   - the min/max partials, the term table and the accumulators live in one
 *     library-owned static device array of BF_STATIC_SCRATCH_BYTES per GPU;
 *     a call whose accumulators ((d+1) x padded rows x padded columns floats)
 *     plus term table exceed it returns BF_EUNSUPPORTED before any kernel
 *     runs (2^24 floats: about 4 million padded pixels at d = 3, 2.3 million
 *     at d = 6; strips pad the image to whole strips of 16 or 32 columns);
 *   - every call on one GPU shares that GPU's array: calls that overlap on
 *     the device (different streams, or threads without ordering) race and
 *     give undefined results.  Calls queued on one stream are ordered and
 *     safe.  The array keeps the last call's contents; nothing in it needs
 *     to start at zero (the kernels write before they read);
 *   - o->time_kernel must be 0 (BF_EINVAL).
 * The caller still provides f and out (and num_out / z_out if wanted). */
int bf_vec_static(const float* f, int H, int W, int d, double sigma_s,
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

/* The same for any BF_WHITEN_* mode: BF_WHITEN_CHOL gives the lower-triangular
 * L^{-1} (C = L L^T), BF_WHITEN_SYM the symmetric C^{-1/2}.  Errors as
 * bf_whiten, and BF_EINVAL for an unknown mode.  Host only. */
int bf_whiten_mode(int d, const double* C, int mode, double* W);

/* Monte Carlo draws of Proposition 2, host only.  X[t][m] ~ B(N, 1/2) is the
 * number of set bits among the first N bits of the Philox4x32-10 stream with
 * key (seed lo32, seed hi32) and counters (t, m, q, 0), q = 0, 1, ...; word
 * 4q + l of the stream is output lane l of counter q; bit i of the stream is
 * bit (i mod 32) of word (i div 32).  Y = N - 2X (eq. (finalApproxY));
 * w[t] = W^T Y[t] / sqrt(N) with W = bf_whiten_mode(C, whiten), so these are
 * exactly the terms bf_vec_ex draws with the same seed, N and opts.whiten.
 * Y (K x d int32) and w (K x d float64) are host arrays; either may be NULL.
 * BF_EINVAL for N or K outside [1, 65536] or an unknown whitening mode;
 * BF_ENOTSPD as bf_whiten. */
int bf_sample_terms(int d, const double* C, int N, int K, uint64_t seed, int whiten,
                    int32_t* Y, double* w);

/* Order rule, host only.  The raised cosine cos(z/sqrt(N))^N of eq. (approx)
 * approximates exp(-z^2/2) (Proposition 1) only for |z| < pi sqrt(N): at
 * z = pi sqrt(N) it aliases back to magnitude one.  With W =
 * bf_whiten_mode(C, whiten), spans s_m = hi[m] - lo[m] and T = max_k sum_m
 * |W_km| s_m (the largest whitened difference between two pixels of the
 * image), N is the smallest integer with pi*sqrt(N) >= T + 4 (the alias lobe
 * stays below exp(-8) over the data range), and at least 10, the paper's
 * order.  lo/hi: host arrays of d floats (finite, lo <= hi), as bf_minmax
 * returns them.  BF_EINVAL for bad arguments, BF_ENOTSPD as bf_whiten,
 * BF_EUNSUPPORTED if that N exceeds 65536. */
int bf_choose_N(int d, const double* C, const float* lo, const float* hi, int whiten, int* N);

/* Per-channel minimum and maximum of a device HWC image, written to host
 * arrays lo/hi (d floats each).  Synchronous on `stream` (NULL = null
 * stream).  BF_EINVAL if the image holds a NaN or infinity. */
int bf_minmax(const float* f, int H, int W, int d, float* lo, float* hi,
              void* stream);

/* Autotuner of the fused kernel's strip height (rows of output per
 * workgroup; the strip width is fixed at 16 columns).  Times the fused kernel
 * with a few probe terms on the device image f (read only) for candidate
 * heights around the occupancy model's choice, and records the fastest in a
 * process-wide table keyed by the current device, d, the window radius,
 * precision and (H, W); later bf_vec_ex / bf_vec_terms calls with
 * tile_h = 0, and server requests of that shape, use it.  Synchronous on
 * `stream`.  Writes the chosen height to *tile_h and its probe time per term
 * in ms to *ms_per_term (either may be NULL).  Errors as bf_vec_ex. */
int bf_autotune(const float* f, int H, int W, int d, double sigma_s,
                int precision, void* stream, int* tile_h, float* ms_per_term);

/* Direct evaluation of eqs. (BF)/(normal) on the GPU with the exact Gaussian
 * range kernel (O(sigma_s^2) work per pixel; the paper's comparison method).
 * Same layout, window and boundary rules as bf_vec.  Synchronous. */
int bf_direct(const float* f, int H, int W, int d, double sigma_s,
              const double* C, float* out);

/* ------------------------------------------------------------------------
 * Fixed-shape plans: Algorithm 1 for a stream of images that share shape,
 * sigma_s, C, K, seed and options.
 *
 * bf_plan_create does the host work of bf_vec_ex once: whitening (eq. (COB)),
 * the draws of Proposition 2, the term and tap table and its upload, the
 * strip geometry, and the device allocations (accumulators, table, min/max
 * partials), all owned by the plan.  bf_plan_execute then queues one HIP
 * graph on `stream` (NULL = null stream) and returns without waiting: the
 * per-channel min/max (centring on only), the fused term loop and the final
 * division of Algorithm 1.  With centring the kernels read the centre from
 * the device min/max result, formed as bf_vec_ex forms it on the host, so
 * out is bit-identical to bf_vec_ex with the same arguments and options.
 * The image's range is unknown when a graph is captured, so plans always
 * run the kernel instance that can reduce large phases in FP64 (about 2%
 * slower than the one bf_vec_ex picks for phases below 2^8 turns; results
 * are the same bits).
 * ------------------------------------------------------------------------ */
typedef struct bf_plan bf_plan;   /* opaque */

/* Create a plan for H x W x d images.  o (NULL = defaults) selects
 * precision, center, tile_h and dedup as for bf_vec_ex; o->N must be explicit
 * (1..65536: the automatic rule needs each image's range on the host), and
 * num_out, z_out and time_kernel must be unset.  o->N_used, o->K_used and
 * o->tile_h_used are written.  Synchronous (uploads the table).  Errors as
 * bf_vec_ex; *plan is NULL on failure. */
int bf_plan_create(int H, int W, int d, double sigma_s, const double* C,
                   int K, uint64_t seed, bf_opts* o, bf_plan** plan);

/* Filter device image f (H x W x d, contiguous) into out (same layout, not
 * overlapping f), queued on `stream`.  The graph of each (f, out) pair is
 * captured on first use; the plan keeps the four most recently used.  f is
 * not checked for NaN or infinity (the output is then unspecified).
 * Executions of one plan share its accumulators: queue them on one stream,
 * or order them, and do not overlap them. */
int bf_plan_execute(bf_plan* plan, const float* f, float* out, void* stream);

/* Wait for the device, then free the plan's graphs and memory.  NULL is a
 * no-op. */
int bf_plan_destroy(bf_plan* plan);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of many filter requests on one GPU.
 *
 * A server owns a device arena (accumulators, term tables, reduction
 * partials), a few HIP streams of default priority and one scheduler thread.
 * Requests are admitted in arrival order while their device footprint fits
 * the arena and fewer than max_active are admitted.  Each scheduling round
 * gives every admitted request the next chunk of its terms -- about
 * quantum_us of modelled device time, so a request smaller than that
 * finishes in its first round while a large one advances a quantum per round
 * -- and packs the chunks of requests that share a kernel instance (d, window
 * radius, precision) into one launch of the batched kernel.  Instances map to
 * streams, so different instances run concurrently.  Rounds are queued at
 * most `depth` ahead of the device.  A result is bit-identical to bf_vec_ex
 * with the same arguments: chunking only splits Algorithm 1's term loop,
 * whose accumulators sit in device memory between terms in both paths.
 *
 * Threading: every bf_server_* call is thread-safe; the scheduler runs on its
 * own thread.  The server binds to the HIP device current at creation.
 *
 * Errors: a launch the runtime refuses (arguments, resources) fails only the
 * requests packed into it, with BF_EDEVICE, after their earlier work has
 * drained; the server keeps serving.  A device error reported later (an
 * event or synchronisation) fails every request, and later submits return it.
 * Test hook: with BF_FAULT_INJECT=launch:<n> in the environment at
 * bf_server_create, the server's n-th batched launch is refused that way
 * without running anything on the device.
 * ---------------------------------------------------------------------- */
typedef struct bf_server bf_server;   /* opaque */

typedef struct bf_server_config {
  uint64_t arena_bytes; /* device arena; 0 = 8 GiB                                */
  int max_active;       /* admitted requests at once; 0 = 64                       */
  int max_queued;       /* submitted, not yet admitted; 0 = unlimited, else submit
                           returns BF_EBUSY beyond it                              */
  int streams;          /* HIP streams for the rounds, 1..16; 0 = 4               */
  int depth;            /* rounds queued on the device at once, >= 1; 0 = 2        */
  double quantum_us;    /* modelled device time per request per round; 0 = 2000   */
  int policy;           /* BF_POLICY_SHARE (0, default): every admitted request
                           advances by one quantum per round (processor
                           sharing); BF_POLICY_SHORTEST_FIRST: a round's budget
                           of quantum x admitted requests goes to the requests
                           with the least modelled work left, each taking all it
                           needs in that order                                   */
  int autotune;         /* 1: the first request of each (d, window radius,
                           precision, strip width, half-octave size class of H
                           and of W) measures its strip height with bf_autotune's
                           probes at submit (the submitting thread waits, a few
                           ms); later requests of the class use the measured
                           strip count.  0 (default): occupancy model, or a
                           height bf_autotune recorded for the exact shape       */
  int graph_rounds;     /* 1: each round's launches on a stream are captured in a
                           HIP graph and launched as one graph; 0 (default):
                           launched directly                                     */
  int reserved[5];
} bf_server_config;

enum { BF_POLICY_SHARE = 0, BF_POLICY_SHORTEST_FIRST = 1 };

typedef struct bf_request {
  const float* f;       /* DEVICE image, H x W x d floats; pixel (y, x) starts at
                           f + (y*pitch + x)*d.  Must hold its final contents at
                           submit and stay unchanged until the request ends.      */
  float* out;           /* DEVICE output, H x W x d contiguous; written when the
                           request ends; must not overlap f                        */
  int H, W, d;
  int pitch;            /* pixels per row of f, >= W; 0 = W                       */
  double sigma_s;
  const double* C;      /* HOST d x d covariance, copied at submit                */
  int K;                /* Monte Carlo terms                                      */
  int N;                /* raised-cosine order; 0 = automatic rule                */
  uint64_t seed;        /* term draws, as in bf_vec_ex                            */
  int precision;        /* BF_FP32, BF_FP16, BF_BF16, BF_FP32_SPLIT               */
  int center;           /* as bf_opts.center                                      */
  double arrival;       /* server clock (s, see bf_server_clock) at which the
                           request arrives; <= 0: at submit.  Latency is measured
                           from it; a request is not admitted before it.          */
  int dedup;            /* as bf_opts.dedup: merge equal +-Y draws (exact)        */
  int spatial;          /* as bf_opts.spatial: BF_SPATIAL_*                        */
  int whiten;           /* as bf_opts.whiten: BF_WHITEN_*                          */
  int reserved[1];
  const float* f_host;  /* HOST image instead of f (f = NULL): H rows of W*d floats,
                           pixel (y, x) at f_host + (y*pitch + x)*d; copied to the
                           device by the server after admission (latency includes
                           the upload).  Pinned memory (hipHostMalloc) keeps the
                           copy asynchronous; must stay unchanged until the
                           request ends                                           */
  float* out_host;      /* HOST H*W*d output: written by a device-to-host copy
                           before the request is reported done (latency includes
                           it); out may then be NULL (the device result lives in
                           the server's arena).  Pinned memory recommended      */
} bf_request;

enum {
  BF_REQ_QUEUED = 0,    /* submitted, not admitted                               */
  BF_REQ_PREPARING = 1, /* admitted: min/max reduction and term table in flight  */
  BF_REQ_RUNNING = 2,   /* in the rounds                                          */
  BF_REQ_DONE = 3,      /* out is complete                                        */
  BF_REQ_FAILED = 4,    /* see error / message                                    */
  BF_REQ_CANCELLED = 5  /* never admitted: server destroyed first                 */
};

typedef struct bf_request_status {
  int state;            /* BF_REQ_*                                               */
  int error;            /* BF_* code when failed                                  */
  int N_used;           /* order used (once the term table is built)              */
  int chunks;           /* rounds that advanced this request                      */
  double arrival;       /* server clock, s                                        */
  double admitted;      /* 0 until admitted                                       */
  double started;       /* first chunk queued; 0 before                           */
  double done;          /* completion observed by the scheduler; 0 before         */
  char message[128];    /* failure message, "" otherwise                          */
} bf_request_status;

typedef struct bf_server_stats {
  uint64_t submitted, completed, failed;
  uint64_t rounds;      /* scheduling rounds queued                               */
  uint64_t launches;    /* batched kernel launches                                */
  uint64_t workgroups;  /* workgroups over all launches                           */
  uint64_t arena_bytes, arena_peak;
  int admitted;         /* requests admitted now                                  */
  int queued;           /* requests waiting for admission now                     */
  float model_scale;    /* measured device time / modelled time of the rounds so
                           far (running average; the round planner multiplies the
                           modelled cost of a term by it, so quantum_us is in
                           measured microseconds); 1 before the first round     */
  int reserved[5];
} bf_server_stats;

/* Fill *cfg with the defaults (all zero fields mean "default"). */
void bf_server_config_init(bf_server_config* cfg);
/* Fill *req with defaults: pitch 0, N 0 (auto), BF_FP16, centring on,
 * arrival 0 (at submit); pointers null. */
void bf_request_init(bf_request* req);

/* Create a server on the current device (cfg may be NULL for defaults).
 * Allocates the arena and starts the scheduler thread.  BF_ENOMEM if the
 * arena cannot be allocated. */
int bf_server_create(const bf_server_config* cfg, bf_server** srv);

/* Queue a request.  Arguments are validated as in bf_vec_ex before anything
 * is queued (BF_EINVAL, BF_ENOTSPD, BF_EUNSUPPORTED); BF_ENOMEM if its
 * footprint exceeds the whole arena, BF_EBUSY past max_queued.  *ticket names
 * it in later calls. */
int bf_server_submit(bf_server* srv, const bf_request* req, uint64_t* ticket);

/* Current status of a request (BF_EINVAL for an unknown ticket). */
int bf_server_poll(bf_server* srv, uint64_t ticket, bf_request_status* st);

/* Wait until the request is done, failed or cancelled, at most timeout_s
 * seconds (< 0: no limit).  BF_ETIMEDOUT if still in flight; st (optional)
 * receives the status either way. */
int bf_server_wait(bf_server* srv, uint64_t ticket, double timeout_s, bf_request_status* st);

/* Wait until every submitted request has ended (timeout as bf_server_wait). */
int bf_server_drain(bf_server* srv, double timeout_s);

/* Drop the record of an ended request (BF_EBUSY if it has not ended). */
int bf_server_forget(bf_server* srv, uint64_t ticket);

/* Counters since creation. */
int bf_server_get_stats(bf_server* srv, bf_server_stats* s);

/* Seconds since the server was created (steady clock). */
double bf_server_clock(const bf_server* srv);

/* Cancel requests not yet admitted, let admitted ones finish, stop the
 * scheduler and free the server's device and host memory. */
int bf_server_destroy(bf_server* srv);

/* ---- Device probes ---------------------------------------------------------
 * The rates a roofline of the fused kernel is read against, measured on the
 * current device (not part of the filter).  Each
 * probe launches one small kernel per repetition on the null stream, one
 * workgroup of 8 waves (two per SIMD) per compute unit, and reports the best
 * of three timed launches in *rate:
 *   BF_UB_MFMA_F32   16x16x4 FP32 matrix products; param independent
 *                    accumulator chains per wave (1, 2, 4 or 8); TFLOP/s
 *   BF_UB_MFMA_F16   16x16x32 FP16 matrix products, likewise; TFLOP/s
 *   BF_UB_VALU_F32   FP32 FMAs (packed FP32 issue is disabled in this build),
 *                    param chains per lane; TFLOP/s
 *   BF_UB_TRANS_F32  v_sin_f32, 8 chains per lane; tera-operations/s
 *   BF_UB_LDS_READ   conflict-free 128-bit LDS reads; TB/s over all CUs
 *   BF_UB_HBM_COPY   a device copy of param MiB (1..16384), read + write
 *                    bytes over time; TB/s (allocates 2 param MiB)
 *   BF_UB_MFMA_F32_SOLO  as BF_UB_MFMA_F32 with one wave per SIMD (4 waves
 *                    per compute unit): a wave's dependent chain alone
 *   BF_UB_OVERLAP_F32  overlap of matrix and vector work on one SIMD: one
 *                    wave runs two chains of 16x16x4 FP32 products, the
 *                    other wave of the SIMD FP32 FMAs of about the same
 *                    duration; *rate = (t_matrix + t_fma - t_both) /
 *                    min(t_matrix, t_fma): 1 when they run side by side, 0
 *                    when their times add (param ignored, pass 0)
 *   BF_UB_OVERLAP_F16  the same with 16x16x32 FP16 products
 * Synchronous.  BF_EINVAL for an unknown probe, a bad param or rate NULL
 * (before any device work); BF_EDEVICE on a HIP error. */
enum { BF_UB_MFMA_F32 = 0, BF_UB_MFMA_F16 = 1, BF_UB_VALU_F32 = 2, BF_UB_TRANS_F32 = 3,
       BF_UB_LDS_READ = 4, BF_UB_HBM_COPY = 5, BF_UB_MFMA_F32_SOLO = 6,
       BF_UB_OVERLAP_F32 = 7, BF_UB_OVERLAP_F16 = 8 };
int bf_ubench(int probe, int param, double* rate);

/* Message for the last failing call on this thread ("" if none). */
const char* bf_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int bf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BFVEC_H */
