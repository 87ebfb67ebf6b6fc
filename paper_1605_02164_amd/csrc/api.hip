// C entry points of libbfvec that touch the device: bf_vec, bf_vec_ex,
// bf_vec_terms, bf_minmax, bf_direct; plus the min/max reduction and the
// direct-filter kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bfvec.h"
#include "host.h"
#include "mcsf_common.h"

namespace bfvec {

namespace {


int hip_fail(hipError_t e, const char* what) {
  return fail(BF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                         \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// ---------------------------------------------------------------------------
// Per-channel min/max (used by the order rule and for centring).
// ---------------------------------------------------------------------------

constexpr int kMMThreads = 256;

__global__ __launch_bounds__(kMMThreads) void minmax_partial(const float* f, size_t npx, int W,
                                                             int pitch, int d, float* part) {
  __shared__ float s_lo[8][kMMThreads], s_hi[8][kMMThreads];
  __shared__ int s_bad[kMMThreads];
  float lo[8], hi[8];
  for (int m = 0; m < 8; ++m) {
    lo[m] = INFINITY;
    hi[m] = -INFINITY;
  }
  int bad = 0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
    const size_t y = p / (size_t)W, q = (y * (size_t)pitch + (p - y * (size_t)W)) * (size_t)d;
    for (int m = 0; m < d; ++m) {
      const float v = f[q + m];
      bad |= !isfinite(v);
      lo[m] = fminf(lo[m], v);
      hi[m] = fmaxf(hi[m], v);
    }
  }
  for (int m = 0; m < 8; ++m) {
    s_lo[m][threadIdx.x] = lo[m];
    s_hi[m][threadIdx.x] = hi[m];
  }
  s_bad[threadIdx.x] = bad;
  __syncthreads();
  for (int w = kMMThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int m = 0; m < 8; ++m) {
        s_lo[m][threadIdx.x] = fminf(s_lo[m][threadIdx.x], s_lo[m][threadIdx.x + w]);
        s_hi[m][threadIdx.x] = fmaxf(s_hi[m][threadIdx.x], s_hi[m][threadIdx.x + w]);
      }
      s_bad[threadIdx.x] |= s_bad[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float* o = part + (size_t)blockIdx.x * 17;
    for (int m = 0; m < 8; ++m) {
      o[m] = s_lo[m][0];
      o[8 + m] = s_hi[m][0];
    }
    o[16] = (float)s_bad[0];
  }
}

__global__ __launch_bounds__(64) void minmax_final(const float* part, int nparts, int d,
                                                   float* res) {
  // one wave: lane m < 8 reduces minima of channel m, lanes 8..15 maxima,
  // lane 16 the non-finite flag; lanes m < d then form the midpoints
  const int l = threadIdx.x;
  float v = l < 8 ? INFINITY : (l < 16 ? -INFINITY : 0.0f);
  if (l < 17) {
    for (int i = 0; i < nparts; ++i) {
      const float x = part[(size_t)i * 17 + l];
      v = l < 8 ? fminf(v, x) : (l < 16 ? fmaxf(v, x) : fmaxf(v, x));
    }
    res[l] = v;
  }
  const float hi = __shfl_down(v, 8);
  if (l < 8) res[17 + l] = l < d ? (float)(0.5 * ((double)v + (double)hi)) : 0.0f;
}

}  // namespace

int minmax_parts(size_t npx) {
  return (int)std::min<size_t>(1024, (npx + kMMThreads - 1) / kMMThreads);
}

hipError_t launch_minmax(const float* f, int H, int W, int pitch, int d, float* part, int nparts,
                         float* res, hipStream_t st) {
  const size_t npx = (size_t)H * W;
  hipLaunchKernelGGL(minmax_partial, dim3(nparts), dim3(kMMThreads), 0, st, f, npx, W, pitch, d,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(minmax_final, dim3(1), dim3(64), 0, st, part, nparts, d, res);
  return hipGetLastError();
}

namespace {

// Per-channel extrema on the host.  work: device buffer of at least
// minmax_floats(H*W) floats, or null to allocate one in stream order.
int run_minmax(const float* f, int H, int W, int d, float* lo, float* hi, hipStream_t st,
               float* work = nullptr) {
  const int nparts = minmax_parts((size_t)H * W);
  float* dbuf = work;
  if (!work)
    HIP_TRY(hipMallocAsync((void**)&dbuf, ((size_t)nparts * 17 + kMMResult) * sizeof(float), st),
            "hipMallocAsync(minmax)");
  float* res = dbuf + (size_t)nparts * 17;
  hipError_t e = launch_minmax(f, H, W, W, d, dbuf, nparts, res, st);
  float h[17];
  if (e == hipSuccess) e = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, st);
  if (!work) {
    hipError_t e2 = hipFreeAsync(dbuf, st);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "min/max reduction");
  if (h[16] != 0.0f) return fail(BF_EINVAL, "f contains NaN or infinity");
  for (int m = 0; m < d; ++m) {
    lo[m] = h[m];
    hi[m] = h[8 + m];
  }
  return BF_OK;
}

}  // namespace

namespace {

int check_opts(const bf_opts* o) {
  if (o->N < 0 || o->N > 65536) return fail(BF_EINVAL, "opts.N must be 0 (auto) or in [1, 65536]");
  if (o->precision != BF_FP32 && o->precision != BF_FP16 && o->precision != BF_BF16 &&
      o->precision != BF_FP32_SPLIT)
    return fail(BF_EINVAL, "opts.precision must be BF_FP32, BF_FP16, BF_BF16 or BF_FP32_SPLIT");
  if (o->center != 0 && o->center != 1) return fail(BF_EINVAL, "opts.center must be 0 or 1");
  if (o->tile_h < 0) return fail(BF_EINVAL, "opts.tile_h must be >= 0");
  if (o->tile_w != 0 && o->tile_w != kTW && o->tile_w != kTWMax)
    return fail(BF_EINVAL, "opts.tile_w must be 0 (auto), 16 or 32");
  if (o->dedup != 0 && o->dedup != 1) return fail(BF_EINVAL, "opts.dedup must be 0 or 1");
  if (o->whiten < BF_WHITEN_EIG || o->whiten > BF_WHITEN_SYM)
    return fail(BF_EINVAL, "opts.whiten must be BF_WHITEN_EIG, _CHOL or _SYM");
  if (o->valu_only != 0 && o->valu_only != 1) return fail(BF_EINVAL, "opts.valu_only must be 0 or 1");
  if (o->precision == BF_FP32_SPLIT && o->valu_only)
    return fail(BF_EUNSUPPORTED, "BF_FP32_SPLIT runs its passes on the matrix cores (valu_only = 0)");
  return check_spatial(o->spatial, o->precision);
}

}  // namespace

int phase64_flag(int d, const float* wmax, const float* cen, const float* lo, const float* hi) {
  if (!lo || !hi) return 1;
  float bound = 0.0f;
  for (int m = 0; m < d; ++m) bound = std::fmaf(wmax[m], std::fmax(hi[m] - cen[m], cen[m] - lo[m]), bound);
  return bound <= kPhaseBound ? 0 : 1;
}

void table_wmax(int d, int K, const float* tab, float* wmax) {
  for (int m = 0; m < 8; ++m) wmax[m] = 0.0f;
  for (int t = 0; t < K; ++t)
    for (int m = 0; m < d; ++m) wmax[m] = std::fmax(wmax[m], std::fabs(tab[(size_t)t * (d + 1) + m]));
}

int check_spatial(int spatial, int precision) {
  if ((spatial & ~(3 | BF_SPATIAL_RUNSUM)) != 0)
    return fail(BF_EINVAL, "spatial must be a BF_SPATIAL_* value");
  if (spatial_runsum(spatial) && spatial_boxes(spatial) == 0)
    return fail(BF_EINVAL, "BF_SPATIAL_RUNSUM applies to the box filters only");
  if (spatial_runsum(spatial) && precision != BF_FP32)
    return fail(BF_EUNSUPPORTED, "BF_SPATIAL_RUNSUM needs BF_FP32");
  return BF_OK;
}

int check_fused_size(int H, int W, int pitch, int d, int R) {
  if (R > kRMax) return fail(BF_EUNSUPPORTED, "sigma_s too large: window radius above 40");
  // the kernels address f and the accumulators with 32-bit byte offsets
  // (buffer loads): each must stay below 2^30 floats
  const double elems = (double)(H + 2 * kB) * (double)(W + kTWMax) * (double)(d + 1);
  const double felems = (double)H * (double)pitch * (double)d;
  if (elems >= 1073741824.0 - 65536.0 || felems >= 1073741824.0 - 65536.0)
    return fail(BF_EUNSUPPORTED, "image too large: H*W*(d+1) must stay below 2^30 elements");
  return BF_OK;
}

void fused_geometry(FusedArgs& a, int H, int W, int R, int prec, int TH, int vbox, int TW) {
  // The kernel prefetches accumulators two steps ahead, which needs at least
  // two steps per term: with no look-ahead rows (R = 0) strips are >= 16 rows.
  if (lag_steps(R) + TH / kB < 2) TH = 2 * kB;
  a.H = H;
  a.W = W;
  a.R = R;
  a.TH = TH;
  a.TWc = TW;
  a.nsx = (W + TW - 1) / TW;
  a.nsy = (H + TH - 1) / TH;
  a.SW = (prec == 1 || prec == 2) ? stage_width16(R, TW) : stage_width(R, TW);
  a.lag = lag_steps(R);
  a.RSB = ring_steps(R, vbox);
  a.vbox = vbox;
  a.CRB = a.lag + 2;
  a.steps = a.lag + TH / kB;
  a.Hp = a.nsy * TH;
}

size_t fused_acc_floats(const FusedArgs& a, int d) {
  return (size_t)(d + 1) * a.Hp * a.nsx * a.TWc;
}

int check_acc_size(const FusedArgs& a, int d) {
  // the kernels form accumulator offsets as 32-bit byte offsets
  if ((double)(d + 1) * (double)a.Hp * (double)a.nsx * (double)a.TWc >= 1073741824.0 - 65536.0)
    return fail(BF_EUNSUPPORTED,
                "accumulators too large: (d+1) x padded rows x padded columns must stay below 2^30");
  return BF_OK;
}


std::vector<float> term_table(int d, int K, const double* w, const double* weights,
                              double sigma_s, size_t* off_weights, size_t* off_taps, int spatial) {
  const int NP = d + 1;
  const int ntaps = 2 * window_radius(sigma_s, spatial) + 1;
  const double two_pi = 6.283185307179586476925286766559;
  const size_t n_terms = (size_t)K * NP, n_w = weights ? (size_t)K : 0;
  std::vector<float> h(2 * n_terms + n_w + (size_t)ntaps, 0.0f);
  for (int t = 0; t < K; ++t)
    for (int m = 0; m < d; ++m) {
      const double x = w[(size_t)t * d + m] / two_pi;
      const float hi = (float)x;
      h[(size_t)t * NP + m] = hi;
      h[n_terms + (size_t)t * NP + m] = (float)(x - (double)hi);
    }
  if (weights)
    for (int t = 0; t < K; ++t) h[2 * n_terms + t] = (float)weights[t];
  const std::vector<double> taps = spatial_taps(sigma_s, spatial);
  for (int u = 0; u < ntaps; ++u) h[2 * n_terms + n_w + u] = (float)taps[u];
  *off_weights = weights ? 2 * n_terms : (size_t)-1;
  *off_taps = 2 * n_terms + n_w;
  return h;
}

void frequency_table(int d, const double* Wm, int N, int K, uint64_t seed, double* w) {
  const double sqn = std::sqrt((double)N);
  for (int t = 0; t < K; ++t) {
    int Y[8];
    for (int m = 0; m < d; ++m) Y[m] = N - 2 * binomial_draw(seed, t, m, N);
    for (int j = 0; j < d; ++j) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += (double)Y[k] * Wm[k * d + j];
      w[(size_t)t * d + j] = s / sqn;
    }
  }
}

void distinct_terms(int d, const double* Wm, int N, int K, uint64_t seed, std::vector<double>* w,
                    std::vector<double>* weight) {
  // key: Y with the sign of its first nonzero entry made positive
  std::map<std::array<int, 8>, size_t> index;
  std::vector<std::array<int, 8>> keys;
  w->clear();
  weight->clear();
  for (int t = 0; t < K; ++t) {
    std::array<int, 8> Y{};
    for (int m = 0; m < d; ++m) Y[m] = N - 2 * binomial_draw(seed, t, m, N);
    int s = 0;
    for (int m = 0; m < d && s == 0; ++m) s = Y[m] > 0 ? 1 : (Y[m] < 0 ? -1 : 0);
    if (s < 0)
      for (int m = 0; m < d; ++m) Y[m] = -Y[m];
    auto it = index.find(Y);
    if (it != index.end()) {
      (*weight)[it->second] += 1.0;
      continue;
    }
    index.emplace(Y, keys.size());
    keys.push_back(Y);
    weight->push_back(1.0);
  }
  const double sqn = std::sqrt((double)N);
  w->resize(keys.size() * d);
  for (size_t u = 0; u < keys.size(); ++u)
    for (int j = 0; j < d; ++j) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += (double)keys[u][k] * Wm[k * d + j];
      (*w)[u * d + j] = s / sqn;
    }
}

namespace {

// Checks that need no device work: window size, precision, strip height.
int plan_fused(int H, int W, int d, double sigma_s, const bf_opts* o, int* TH, int* TW) {
  const int R = window_radius(sigma_s, spatial_boxes(o->spatial));
  int rc = check_fused_size(H, W, W, d, R);
  if (rc) return rc;
  const int v = select_variant(d, R, o->precision, o->spatial, W, o->tile_w, o->valu_only);
  if ((rc = choose_strip_width(d, R, v, H, W, o->tile_w, TW))) return rc;
  if ((rc = choose_strip_height(d, R, v, H, W, o->tile_h, TH, *TW, o->valu_only))) return rc;
  FusedArgs g{};   // the padded accumulators of this geometry must fit 32-bit offsets
  fused_geometry(g, H, W, R, v, *TH, v == 3 ? spatial_boxes(o->spatial) : 0, *TW);
  return check_acc_size(g, d);
}

// Launch the fused filter for a host FP64 term table (radians per unit).
// lo/hi: per-channel extrema when known (min/max ran), else null.
// work: device buffer of work_floats floats for the accumulators and the
// term table (the call fails with BF_EUNSUPPORTED if they do not fit), or
// null to allocate them in stream order.
int run_terms(const float* f, int H, int W, int d, double sigma_s, const double* w,
              const double* weights, int K, float* out, bf_opts* o, const float* lo,
              const float* hi, int TH, int TW, float* work = nullptr, size_t work_floats = 0) {
  hipStream_t st = (hipStream_t)o->stream;
  const int R = window_radius(sigma_s, spatial_boxes(o->spatial));
  const int variant = select_variant(d, R, o->precision, o->spatial, W, o->tile_w, o->valu_only);
  size_t off_w = 0, off_taps = 0;
  const std::vector<float> hbuf =
      term_table(d, K, w, weights, sigma_s, &off_w, &off_taps, spatial_boxes(o->spatial));

  FusedArgs a{};
  a.f = f;
  for (int m = 0; m < 8; ++m)
    a.cen[m] = (o->center && lo && m < d) ? (float)(0.5 * ((double)lo[m] + (double)hi[m])) : 0.0f;
  table_wmax(d, K, hbuf.data(), a.wmax);
  a.p64 = phase64_flag(d, a.wmax, a.cen, lo, hi);
  fused_geometry(a, H, W, R, variant, TH, variant == 3 ? spatial_boxes(o->spatial) : 0, TW);
  a.fpitch = W;
  a.t0 = 0;
  a.t1 = K;
  a.valu = o->valu_only;
  int rc = check_acc_size(a, d);
  if (rc) return rc;
  if (o->precision == BF_FP16 || o->precision == BF_FP32_SPLIT) {
    if (!lo) return fail(BF_EINVAL, "FP16 storage needs the image range (internal)");
    if ((rc = check_fp16_range(d, sigma_s, spatial_boxes(o->spatial), lo, hi, a.cen))) return rc;
  }
  o->tile_h_used = a.TH;
  o->tile_w_used = a.TWc;
  o->mfma_used = fused_uses_mf(d, R, variant, a.TWc, a.valu);

  // one buffer: accumulators | terms | weights | taps
  const size_t n_acc = fused_acc_floats(a, d);
  float* dbuf = work;
  if (work && n_acc + hbuf.size() > work_floats)
    return fail(BF_EUNSUPPORTED,
                "accumulators and term table need " +
                    std::to_string((n_acc + hbuf.size()) * sizeof(float)) +
                    " bytes, above the static scratch of " +
                    std::to_string(work_floats * sizeof(float)) + " bytes");
  if (!work)
    HIP_TRY(hipMallocAsync((void**)&dbuf, (n_acc + hbuf.size()) * sizeof(float), st),
            "hipMallocAsync(accumulators)");
  a.acc = dbuf;
  float* dterms = dbuf + n_acc;
  hipError_t e = hipMemcpyAsync(dterms, hbuf.data(), hbuf.size() * sizeof(float),
                                hipMemcpyHostToDevice, st);
  a.terms = dterms;
  a.terms_lo = dterms + (size_t)K * (d + 1);
  a.weights = weights ? dterms + off_w : nullptr;
  a.taps = dterms + off_taps;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess && o->time_kernel) {
    e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e == hipSuccess) e = hipEventRecord(ev0, st);
  }
  if (e == hipSuccess) e = launch_fused(d, variant, a, st);
  if (e == hipSuccess && o->time_kernel) e = hipEventRecord(ev1, st);
  if (e == hipSuccess) {
    FinalizeArgs fa{};
    fa.acc = a.acc;
    fa.out = out;
    fa.num_out = o->num_out;
    fa.z_out = o->z_out;
    for (int m = 0; m < 8; ++m) fa.cen[m] = a.cen[m];
    fa.H = H;
    fa.W = W;
    fa.Hp = a.Hp;
    fa.Wp = a.nsx * a.TWc;
    e = launch_finalize(d, fa, st);
  }
  if (e == hipSuccess && o->time_kernel) {
    e = hipEventSynchronize(ev1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    o->kernel_ms = ms;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (!work) {
    hipError_t e2 = hipFreeAsync(dbuf, st);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return hip_fail(e, "fused MCSF launch");
  return BF_OK;
}

// ---------------------------------------------------------------------------
// Direct evaluation of eqs. (BF)/(normal) with the Gaussian range kernel.
// One thread per output pixel; neighbours read through the cache hierarchy.
// ---------------------------------------------------------------------------

struct DirectArgs {
  const float* f;
  float* out;
  float Wm[64];     // whitening, row-major d x d
  float taps[96 * 2 + 1];
  int H, W, R;
};

template <int D>
__global__ __launch_bounds__(256) void direct_bf(DirectArgs a) {
  const int x = blockIdx.x * 16 + (threadIdx.x % 16);
  const int y = blockIdx.y * 16 + (threadIdx.x / 16);
  if (x >= a.W || y >= a.H) return;
  float fi[D];
  for (int m = 0; m < D; ++m) fi[m] = a.f[((size_t)y * a.W + x) * D + m];
  float num[D];
  for (int m = 0; m < D; ++m) num[m] = 0.0f;
  float Z = 0.0f;
  for (int jy = -a.R; jy <= a.R; ++jy) {
    const int yy = y - jy;
    if (yy < 0 || yy >= a.H) continue;
    const float wy = a.taps[jy + a.R];
    for (int jx = -a.R; jx <= a.R; ++jx) {
      const int xx = x - jx;
      if (xx < 0 || xx >= a.W) continue;
      const float* fj = a.f + ((size_t)yy * a.W + xx) * D;
      float v[D], dl[D];
      for (int m = 0; m < D; ++m) {
        v[m] = fj[m];
        dl[m] = v[m] - fi[m];
      }
      float q = 0.0f;
      for (int k = 0; k < D; ++k) {
        float z = 0.0f;
        for (int m = 0; m < D; ++m) z = fmaf(a.Wm[k * D + m], dl[m], z);
        q = fmaf(z, z, q);
      }
      const float wgt = wy * a.taps[jx + a.R] * expf(-0.5f * q);
      Z += wgt;
      for (int m = 0; m < D; ++m) num[m] = fmaf(wgt, v[m], num[m]);
    }
  }
  for (int m = 0; m < D; ++m) a.out[((size_t)y * a.W + x) * D + m] = num[m] / Z;
}

template <int D>
hipError_t launch_direct(const DirectArgs& a, hipStream_t st) {
  dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
  hipLaunchKernelGGL(direct_bf<D>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free variant (bf_vec_static): every device buffer the call needs
// (min/max partials, term table, accumulators) lives in one file-scope device
// array per GPU.  Host code must not use the array's name as a device
// address: its per-device address comes from hipGetSymbolAddress, taken once
// per device with that device current.
// ---------------------------------------------------------------------------

constexpr size_t kScratchFloats = (size_t)BF_STATIC_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (resolved on the first call there).
int scratch_for_current_device(float** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(BF_EDEVICE, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(BF_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *ptr = g_scratch_ptr[dev];
  return BF_OK;
}

}  // namespace
}  // namespace bfvec

using namespace bfvec;

extern "C" {

int bf_vec_static(const float* f, int H, int W, int d, double sigma_s, const double* C, int K,
                  uint64_t seed, float* out, bf_opts* o) {
  clear_error();
  bf_opts def;
  if (!o) {
    bf_opts_init(&def);
    o = &def;
  }
  int rc = check_common(f, H, W, d, sigma_s, out);
  if (rc) return rc;
  if (K < 1 || K > 65536) return fail(BF_EINVAL, "K must be in [1, 65536]");
  if (!C) return fail(BF_EINVAL, "C must be non-null");
  if ((rc = check_opts(o))) return rc;
  if (o->time_kernel) return fail(BF_EINVAL, "bf_vec_static takes no time_kernel (events)");
  double Wm[64];
  if ((rc = whiten(d, C, Wm, o->whiten))) return rc;
  int TH = 0, TW = 0;
  if ((rc = plan_fused(H, W, d, sigma_s, o, &TH, &TW))) return rc;
  // the min/max partials fit the scratch at any size (at most 1024 x 17 +
  // kMMResult floats); the accumulators and the table are checked by run_terms
  float* work = nullptr;
  if ((rc = scratch_for_current_device(&work))) return rc;
  float lo[8] = {0}, hi[8] = {0};
  const bool have_range = o->N == 0 || o->center || o->precision == BF_FP16 ||
                          o->precision == BF_FP32_SPLIT;
  if (have_range && (rc = run_minmax(f, H, W, d, lo, hi, (hipStream_t)o->stream, work))) return rc;
  int N = o->N;
  if (N == 0 && (rc = choose_order(d, Wm, lo, hi, &N))) return rc;
  o->N_used = N;
  std::vector<double> w, weight;
  if (o->dedup) {
    distinct_terms(d, Wm, N, K, seed, &w, &weight);
    o->K_used = (int)weight.size();
  } else {
    w.resize((size_t)K * d);
    frequency_table(d, Wm, N, K, seed, w.data());
    o->K_used = K;
  }
  return run_terms(f, H, W, d, sigma_s, w.data(), o->dedup ? weight.data() : nullptr, o->K_used,
                   out, o, have_range ? lo : nullptr, have_range ? hi : nullptr, TH, TW, work,
                   kScratchFloats);
}

int bf_vec_ex(const float* f, int H, int W, int d, double sigma_s, const double* C, int K,
              uint64_t seed, float* out, bf_opts* o) {
  clear_error();
  bf_opts def;
  if (!o) {
    bf_opts_init(&def);
    o = &def;
  }
  int rc = check_common(f, H, W, d, sigma_s, out);
  if (rc) return rc;
  if (K < 1 || K > 65536) return fail(BF_EINVAL, "K must be in [1, 65536]");
  if (!C) return fail(BF_EINVAL, "C must be non-null");
  if ((rc = check_opts(o))) return rc;
  double Wm[64];
  if ((rc = whiten(d, C, Wm, o->whiten))) return rc;
  int TH = 0, TW = 0;
  if ((rc = plan_fused(H, W, d, sigma_s, o, &TH, &TW))) return rc;
  float lo[8] = {0}, hi[8] = {0};
  // the order rule, centring and the FP16 range check need the extrema
  const bool have_range = o->N == 0 || o->center || o->precision == BF_FP16 ||
                          o->precision == BF_FP32_SPLIT;
  if (have_range) {
    if ((rc = run_minmax(f, H, W, d, lo, hi, (hipStream_t)o->stream))) return rc;
  }
  int N = o->N;
  if (N == 0 && (rc = choose_order(d, Wm, lo, hi, &N))) return rc;
  o->N_used = N;
  if (o->dedup) {
    std::vector<double> w, weight;
    distinct_terms(d, Wm, N, K, seed, &w, &weight);
    o->K_used = (int)weight.size();
    return run_terms(f, H, W, d, sigma_s, w.data(), weight.data(), o->K_used, out, o,
                     have_range ? lo : nullptr, have_range ? hi : nullptr, TH, TW);
  }
  std::vector<double> w((size_t)K * d);
  frequency_table(d, Wm, N, K, seed, w.data());
  o->K_used = K;
  return run_terms(f, H, W, d, sigma_s, w.data(), nullptr, K, out, o,
                   have_range ? lo : nullptr, have_range ? hi : nullptr, TH, TW);
}

int bf_vec(const float* f, int H, int W, int d, double sigma_s, const double* C, int K,
           uint64_t seed, float* out) {
  bf_opts o;
  bf_opts_init(&o);
  int rc = bf_vec_ex(f, H, W, d, sigma_s, C, K, seed, out, &o);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return BF_OK;
}

int bf_vec_terms(const float* f, int H, int W, int d, double sigma_s, const double* w,
                 const double* weights, int K, float* out, bf_opts* o) {
  clear_error();
  bf_opts def;
  if (!o) {
    bf_opts_init(&def);
    o = &def;
  }
  int rc = check_common(f, H, W, d, sigma_s, out);
  if (rc) return rc;
  if (K < 1 || K > (1 << 24)) return fail(BF_EINVAL, "K must be in [1, 2^24]");
  if (!w) return fail(BF_EINVAL, "w must be non-null");
  if ((rc = check_opts(o))) return rc;
  for (size_t i = 0; i < (size_t)K * d; ++i)
    if (!std::isfinite(w[i])) return fail(BF_EINVAL, "w must be finite");
  if (weights)
    for (int t = 0; t < K; ++t)
      if (!(weights[t] >= 0.0) || !std::isfinite(weights[t]))
        return fail(BF_EINVAL, "weights must be finite and nonnegative");
  int TH = 0, TW = 0;
  if ((rc = plan_fused(H, W, d, sigma_s, o, &TH, &TW))) return rc;
  float lo[8] = {0}, hi[8] = {0};
  const bool have_range = o->center || o->precision == BF_FP16 ||
                          o->precision == BF_FP32_SPLIT;
  if (have_range && (rc = run_minmax(f, H, W, d, lo, hi, (hipStream_t)o->stream))) return rc;
  o->N_used = o->N;
  o->K_used = K;
  return run_terms(f, H, W, d, sigma_s, w, weights, K, out, o, have_range ? lo : nullptr,
                   have_range ? hi : nullptr, TH, TW);
}

int bf_autotune(const float* f, int H, int W, int d, double sigma_s, int precision, void* stream,
                int* tile_h, float* ms_per_term) {
  clear_error();
  // f is read only; a distinct dummy output pointer passes the common checks
  int rc = check_common(f, H, W, d, sigma_s, (const char*)f + (size_t)H * W * d * sizeof(float));
  if (rc) return rc;
  if (precision != BF_FP32 && precision != BF_FP16 && precision != BF_BF16 &&
      precision != BF_FP32_SPLIT)
    return fail(BF_EINVAL, "precision must be BF_FP32, BF_FP16, BF_BF16 or BF_FP32_SPLIT");
  return autotune_strip_height(f, H, W, W, d, sigma_s, precision, (hipStream_t)stream, tile_h,
                               ms_per_term);
}

}  // extern "C"

namespace bfvec {

int autotune_strip_height(const float* f, int H, int W, int pitch, int d, double sigma_s,
                          int precision, hipStream_t stream, int* tile_h, float* ms_per_term) {
  int rc = BF_OK;
  const int R = window_radius(sigma_s);
  if ((rc = check_fused_size(H, W, pitch, d, R))) return rc;
  int TH0 = 0;   // validates the window against the LDS budget
  if ((rc = choose_strip_height(d, R, precision, H, W, 0, &TH0))) return rc;
  (void)TH0;
  int TW = kTW;   // the probes run at the automatic strip width
  if ((rc = choose_strip_width(d, R, precision, H, W, 0, &TW))) return rc;
  // every height as the launch runs it (fused_geometry may round it up)
  auto effective = [&](int th) {
    FusedArgs g{};
    fused_geometry(g, H, W, R, precision, th, 0, TW);
    return g.TH;
  };
  const int model = effective(model_strip_height(d, R, precision, H, W, TW));
  // candidate strip counts down the image around the model's
  const int nsy0 = (H + model - 1) / model, nmax = (H + kB - 1) / kB;
  std::vector<int> ths;
  auto acc_fits = [&](int th) {   // check_acc_size's rule, without setting an error
    FusedArgs g{};
    fused_geometry(g, H, W, R, precision, th, 0, TW);
    return (double)fused_acc_floats(g, d) < 1073741824.0 - 65536.0;
  };
  if (!acc_fits(model)) {
    FusedArgs g{};
    fused_geometry(g, H, W, R, precision, model, 0, TW);
    return check_acc_size(g, d);
  }
  const int mult = strip_row_multiple(d, R, precision, TW, 0);
  for (int f10 : {3, 5, 7, 10, 13, 15, 20, 30, 40}) {
    const int nsy = std::min(nmax, std::max(1, (nsy0 * f10 + 5) / 10));
    const int th = effective(((H + nsy - 1) / nsy + mult - 1) / mult * mult);
    if (acc_fits(th) && std::find(ths.begin(), ths.end(), th) == ths.end()) ths.push_back(th);
  }
  // probe terms: a few fixed frequencies (the cost does not depend on them)
  constexpr int KP = 4;
  std::vector<double> w((size_t)KP * d);
  for (int t = 0; t < KP; ++t)
    for (int m = 0; m < d; ++m) w[(size_t)t * d + m] = 0.7 + 0.3 * t + 0.1 * m;
  size_t off_w = 0, off_taps = 0;
  const std::vector<float> tab = term_table(d, KP, w.data(), nullptr, sigma_s, &off_w, &off_taps);
  size_t n_acc = 0;
  for (int th : ths) {
    FusedArgs a{};
    fused_geometry(a, H, W, R, precision, th, 0, TW);
    n_acc = std::max(n_acc, fused_acc_floats(a, d));
  }
  hipStream_t st = (hipStream_t)stream;
  float* dbuf = nullptr;
  HIP_TRY(hipMallocAsync((void**)&dbuf, (n_acc + tab.size()) * sizeof(float), st),
          "hipMallocAsync(autotune)");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemcpyAsync(dbuf + n_acc, tab.data(), tab.size() * sizeof(float),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // The model's own height is timed too; another candidate replaces it only
  // when it is at least 2% faster (probe timings vary by about 1%).
  if (std::find(ths.begin(), ths.end(), model) == ths.end()) ths.push_back(model);
  int best_th = model;
  float best = -1.0f, model_ms = -1.0f;
  for (size_t i = 0; i < ths.size() && e == hipSuccess; ++i) {
    FusedArgs a{};
    a.f = f;
    a.acc = dbuf;
    a.terms = dbuf + n_acc;
    a.terms_lo = a.terms + (size_t)KP * (d + 1);
    a.taps = dbuf + n_acc + off_taps;
    a.p64 = 0;   // probe phases are small
    fused_geometry(a, H, W, R, precision, ths[i], 0, TW);
    a.fpitch = pitch;
    a.t0 = 0;
    a.t1 = KP;
    e = launch_fused(d, precision, a, st);   // warm-up
    float ms = -1.0f;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {   // fastest of three probes
      float m = 0.0f;
      e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = launch_fused(d, precision, a, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
      if (e == hipSuccess && (ms < 0.0f || m < ms)) ms = m;
    }
    if (e != hipSuccess) break;
    if (ths[i] == model) model_ms = ms;
    if (best < 0.0f || ms < best) {
      best = ms;
      best_th = ths[i];
    }
  }
  if (e == hipSuccess && model_ms > 0.0f && best > 0.98f * model_ms) {
    best_th = model;
    best = model_ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t e2 = hipFreeAsync(dbuf, st);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "autotune");
  record_tuned_height(d, R, precision, H, W, best_th, TW);
  if (tile_h) *tile_h = best_th;
  if (ms_per_term) *ms_per_term = best / KP;
  return BF_OK;
}

}  // namespace bfvec

extern "C" {

int bf_minmax(const float* f, int H, int W, int d, float* lo, float* hi, void* stream) {
  clear_error();
  if (!f || !lo || !hi) return fail(BF_EINVAL, "null argument");
  if (H < 1 || W < 1 || d < 1 || d > 8) return fail(BF_EINVAL, "bad image shape");
  return run_minmax(f, H, W, d, lo, hi, (hipStream_t)stream);
}

int bf_direct(const float* f, int H, int W, int d, double sigma_s, const double* C, float* out) {
  clear_error();
  int rc = check_common(f, H, W, d, sigma_s, out);
  if (rc) return rc;
  if (!C) return fail(BF_EINVAL, "C must be non-null");
  double Wm[64];
  if ((rc = whiten(d, C, Wm))) return rc;
  const int R = window_radius(sigma_s);
  if (R > 96) return fail(BF_EUNSUPPORTED, "window radius above 96");
  DirectArgs a{};
  a.f = f;
  a.out = out;
  for (int i = 0; i < d * d; ++i) a.Wm[i] = (float)Wm[i];
  const std::vector<double> taps = spatial_taps(sigma_s);
  for (int u = 0; u < 2 * R + 1; ++u) a.taps[u] = (float)taps[u];
  a.H = H;
  a.W = W;
  a.R = R;
  hipError_t e;
  switch (d) {
    case 1: e = launch_direct<1>(a, nullptr); break;
    case 2: e = launch_direct<2>(a, nullptr); break;
    case 3: e = launch_direct<3>(a, nullptr); break;
    case 4: e = launch_direct<4>(a, nullptr); break;
    case 5: e = launch_direct<5>(a, nullptr); break;
    case 6: e = launch_direct<6>(a, nullptr); break;
    case 7: e = launch_direct<7>(a, nullptr); break;
    default: e = launch_direct<8>(a, nullptr); break;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "direct filter");
  return BF_OK;
}

}  // extern "C"
