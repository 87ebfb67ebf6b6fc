// Fixed-shape execution plans: the bf_plan_* entry points.
//
// A plan is created once per (shape, sigma_s, C, K, seed, options).  The host
// work of a bf_vec_ex call -- whitening, the Monte Carlo draws of
// Proposition 2, the term/tap table and its upload, the strip geometry, the
// device allocations -- happens at creation.  Each execution is then one HIP
// graph launch of the device steps of Algorithm 1: the per-channel min/max
// (only with centring on), the fused term loop and the final division.  The
// centre is read by the kernels from the min/max result on the device, so no
// execution waits for the host.
//
// A graph embeds the f and out pointers of the launches it was captured with,
// so a plan keeps a small cache of instantiated graphs keyed by (f, out): a
// caller that cycles through a few buffers captures each pair once.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "bfvec.h"
#include "host.h"
#include "mcsf_common.h"

struct bf_plan {
  int H = 0, W = 0, d = 0, variant = 0, center = 0;   // variant: kernel_variant()
  bfvec::FusedArgs a{};        // geometry, tables and accumulators (no f)
  float* dev = nullptr;        // accumulators | term table | min/max partials | result
  int nparts = 0;
  float* part = nullptr;
  float* res = nullptr;
  hipStream_t cap = nullptr;   // private stream the graphs are captured on
  struct Entry {
    const float* f;
    float* out;
    hipGraphExec_t exec;
    uint64_t used;
  };
  std::vector<Entry> cache;
  uint64_t tick = 0;
  std::mutex mu;               // executions of one plan are serialised
};

namespace bfvec {
namespace {

constexpr size_t kPlanGraphs = 4;   // instantiated graphs kept per plan

int plan_hip_fail(hipError_t e, const char* what) {
  return fail(BF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void free_plan(bf_plan* p) {
  for (auto& c : p->cache) (void)hipGraphExecDestroy(c.exec);
  p->cache.clear();
  if (p->dev) (void)hipFree(p->dev);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

// Records the device steps of one execution on p->cap (in capture mode).
hipError_t record_steps(bf_plan* p, const float* f, float* out) {
  hipError_t e = hipSuccess;
  const float* cen = nullptr;
  if (p->center) {
    e = launch_minmax(f, p->H, p->W, p->W, p->d, p->part, p->nparts, p->res, p->cap);
    cen = p->res + 17;
  }
  FusedArgs a = p->a;
  a.f = f;
  a.cen_dev = cen;
  if (e == hipSuccess) e = launch_fused(p->d, p->variant, a, p->cap);
  if (e == hipSuccess) {
    FinalizeArgs fa{};
    fa.acc = a.acc;
    fa.out = out;
    fa.cen_dev = cen;
    fa.H = p->H;
    fa.W = p->W;
    fa.Hp = a.Hp;
    fa.Wp = a.nsx * a.TWc;
    e = launch_finalize(p->d, fa, p->cap);
  }
  return e;
}

// Captures and instantiates the graph of one (f, out) pair.
int capture(bf_plan* p, const float* f, float* out, hipGraphExec_t* exec) {
  hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return plan_hip_fail(e, "hipStreamBeginCapture");
  const hipError_t e_rec = record_steps(p, f, out);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(p->cap, &g);   // always leave capture mode
  if (e_rec != hipSuccess) e = e_rec;
  if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return plan_hip_fail(e, "plan graph capture");
  return BF_OK;
}

}  // namespace
}  // namespace bfvec

using namespace bfvec;

extern "C" {

int bf_plan_create(int H, int W, int d, double sigma_s, const double* C, int K, uint64_t seed,
                   bf_opts* o, bf_plan** plan) {
  clear_error();
  if (!plan) return fail(BF_EINVAL, "plan must be non-null");
  *plan = nullptr;
  bf_opts def;
  if (!o) {
    bf_opts_init(&def);
    o = &def;
  }
  // the shape rules of bf_vec_ex (the images come with each execution)
  if (H < 1 || W < 1 || H > 65536 || W > 65536)
    return fail(BF_EINVAL, "H and W must be in [1, 65536]");
  if (d < 1 || d > 8) return fail(BF_EINVAL, "d must be in [1, 8]");
  if (!std::isfinite(sigma_s) || sigma_s < 0.0 || sigma_s > 32.0)
    return fail(BF_EINVAL, "sigma_s must be finite and in [0, 32]");
  int rc = BF_OK;
  if (K < 1 || K > 65536) return fail(BF_EINVAL, "K must be in [1, 65536]");
  if (!C) return fail(BF_EINVAL, "C must be non-null");
  if (o->N < 1 || o->N > 65536)
    return fail(BF_EINVAL, "plans need an explicit order: opts.N in [1, 65536]");
  if (o->precision != BF_FP32 && o->precision != BF_FP16 && o->precision != BF_BF16 &&
      o->precision != BF_FP32_SPLIT)
    return fail(BF_EINVAL, "opts.precision must be BF_FP32, BF_FP16, BF_BF16 or BF_FP32_SPLIT");
  if (o->center != 0 && o->center != 1) return fail(BF_EINVAL, "opts.center must be 0 or 1");
  if (o->tile_h < 0) return fail(BF_EINVAL, "opts.tile_h must be >= 0");
  if (o->dedup != 0 && o->dedup != 1) return fail(BF_EINVAL, "opts.dedup must be 0 or 1");
  if (int rs = check_spatial(o->spatial, o->precision)) return rs;
  if (o->whiten < BF_WHITEN_EIG || o->whiten > BF_WHITEN_SYM)
    return fail(BF_EINVAL, "opts.whiten must be BF_WHITEN_EIG, _CHOL or _SYM");
  if (o->num_out || o->z_out || o->time_kernel)
    return fail(BF_EINVAL, "plans take no num_out, z_out or time_kernel");
  if (o->valu_only != 0 && o->valu_only != 1) return fail(BF_EINVAL, "opts.valu_only must be 0 or 1");
  if (o->precision == BF_FP32_SPLIT && o->valu_only)
    return fail(BF_EUNSUPPORTED, "BF_FP32_SPLIT runs its passes on the matrix cores (valu_only = 0)");
  double Wm[64];
  if ((rc = whiten(d, C, Wm, o->whiten))) return rc;
  const int R = window_radius(sigma_s, spatial_boxes(o->spatial));
  const int variant = select_variant(d, R, o->precision, o->spatial, W, o->tile_w, o->valu_only);
  if ((rc = check_fused_size(H, W, W, d, R))) return rc;
  int TH = 0, TW = 0;
  if ((rc = choose_strip_width(d, R, variant, H, W, o->tile_w, &TW))) return rc;
  if ((rc = choose_strip_height(d, R, variant, H, W, o->tile_h, &TH, TW, o->valu_only))) return rc;
  {
    FusedArgs g{};
    fused_geometry(g, H, W, R, variant, TH, variant == 3 ? spatial_boxes(o->spatial) : 0, TW);
    if ((rc = check_acc_size(g, d))) return rc;
  }

  // the terms, exactly as bf_vec_ex draws them
  const int N = o->N;
  std::vector<double> w, weight;
  int Kr = K;
  if (o->dedup) {
    distinct_terms(d, Wm, N, K, seed, &w, &weight);
    Kr = (int)weight.size();
  } else {
    w.resize((size_t)K * d);
    frequency_table(d, Wm, N, K, seed, w.data());
  }
  size_t off_w = 0, off_taps = 0;
  const std::vector<float> tab = term_table(d, Kr, w.data(), o->dedup ? weight.data() : nullptr,
                                            sigma_s, &off_w, &off_taps,
                                            spatial_boxes(o->spatial));

  bf_plan* p = new bf_plan;
  p->H = H;
  p->W = W;
  p->d = d;
  p->variant = variant;
  p->center = o->center;
  FusedArgs& a = p->a;
  fused_geometry(a, H, W, R, variant, TH, variant == 3 ? spatial_boxes(o->spatial) : 0, TW);
  a.fpitch = W;
  a.t0 = 0;
  a.t1 = Kr;
  a.valu = o->valu_only;
  const size_t n_acc = fused_acc_floats(a, d);
  p->nparts = minmax_parts((size_t)H * W);
  const size_t n_mm = o->center ? (size_t)p->nparts * 17 + kMMResult : 0;
  const size_t n_tab = (tab.size() + 63) / 64 * 64;   // keep the partials 256-byte aligned
  hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void**)&p->dev, (n_acc + n_tab + n_mm) * sizeof(float));
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->dev + n_acc, tab.data(), tab.size() * sizeof(float),
                       hipMemcpyHostToDevice, p->cap);
  if (e == hipSuccess) e = hipStreamSynchronize(p->cap);
  if (e != hipSuccess) {
    free_plan(p);
    return plan_hip_fail(e, "plan creation");
  }
  a.acc = p->dev;
  a.terms = p->dev + n_acc;
  a.terms_lo = a.terms + (size_t)Kr * (d + 1);
  table_wmax(d, Kr, tab.data(), a.wmax);
  a.p64 = 1;   // the image's range is not known when the graph is captured
  a.weights = o->dedup ? a.terms + off_w : nullptr;
  a.taps = a.terms + off_taps;
  if (o->center) {
    p->part = p->dev + n_acc + n_tab;
    p->res = p->part + (size_t)p->nparts * 17;
  }
  o->N_used = N;
  o->K_used = Kr;
  o->tile_h_used = a.TH;
  o->tile_w_used = a.TWc;
  o->mfma_used = fused_uses_mf(d, R, variant, a.TWc, a.valu);
  *plan = p;
  return BF_OK;
}

int bf_plan_execute(bf_plan* p, const float* f, float* out, void* stream) {
  clear_error();
  if (!p) return fail(BF_EINVAL, "plan must be non-null");
  int rc = check_common(f, p->H, p->W, p->d, 0.0, out);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(p->mu);
  bf_plan::Entry* hit = nullptr;
  for (auto& c : p->cache)
    if (c.f == f && c.out == out) hit = &c;
  if (!hit) {
    hipGraphExec_t exec = nullptr;
    if ((rc = capture(p, f, out, &exec))) return rc;
    if (p->cache.size() == kPlanGraphs) {   // replace the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < p->cache.size(); ++i)
        if (p->cache[i].used < p->cache[lru].used) lru = i;
      (void)hipGraphExecDestroy(p->cache[lru].exec);
      p->cache[lru] = {f, out, exec, 0};
      hit = &p->cache[lru];
    } else {
      p->cache.push_back({f, out, exec, 0});
      hit = &p->cache.back();
    }
  }
  hit->used = ++p->tick;
  const hipError_t e = hipGraphLaunch(hit->exec, (hipStream_t)stream);
  if (e != hipSuccess) return plan_hip_fail(e, "hipGraphLaunch");
  return BF_OK;
}

int bf_plan_destroy(bf_plan* p) {
  clear_error();
  if (!p) return BF_OK;
  // executions may still be queued on the caller's streams
  const hipError_t e = hipDeviceSynchronize();
  free_plan(p);
  if (e != hipSuccess) return plan_hip_fail(e, "hipDeviceSynchronize");
  return BF_OK;
}

}  // extern "C"
