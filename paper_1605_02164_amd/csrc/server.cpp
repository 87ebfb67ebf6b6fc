// Continuous-batching server of the MCSF filter: the bf_server_* entry points.
//
// One scheduler thread per server drives the device:
//   admission  -- requests whose arrival time has passed are admitted in
//                 arrival order while their footprint (accumulators, term
//                 table, reduction partials) fits the device arena and fewer
//                 than max_active are admitted;
//   preparation-- per-channel min/max on an auxiliary stream when the order
//                 rule or centring needs it, then the host draws the K terms
//                 (Proposition 2, as bf_vec_ex does) and uploads the table;
//   rounds     -- every admitted request gets its next chunk of terms (a
//                 quantum of modelled device time) and chunks of one kernel
//                 instance go into one batched launch; at most `depth` rounds
//                 are queued ahead of the device;
//   completion -- after its last chunk a request's finalize kernel (the
//                 division of Algorithm 1) and a completion event follow on
//                 the same stream; the scheduler frees its arena block when
//                 the event has passed.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "bfvec.h"
#include "host.h"
#include "mcsf_common.h"
#include "scheduler.h"

namespace bfvec {
namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr int kMMFloats = 17;  // min/max partial block: 8 minima, 8 maxima, flag

// Modelled device cost of one term of a planned request, in microseconds:
// executed flops of all its workgroup steps (modulation of the haloed rows,
// both passes; the 16-bit passes do two taps per instruction, the running-sum
// vertical passes of variants 3 and 4 about eight operations per output) at a
// nominal 50 TFLOP/s.  The server scales it by the measured device time of
// its rounds over their modelled time (Server::model_scale), so the nominal
// rate only sets the first rounds.
double model_term_us(const FusedArgs& a, int d, int prec) {
  const double NC = 2.0 * (d + 1), taps = 2.0 * a.R + 1.0;
  const double mod = (double)kB * (a.TWc + 2 * a.R) * (4.0 * d + 2.0);
  const double one = (double)kB * NC * a.TWc * taps * 2.0;   // one FIR pass, FP32
  // variants 3 and 4: the running-sum vertical pass; 5: FP32 with the
  // vertical pass on FP16 products (measured ~0.78 of FP32's time)
  const double pass = (prec == 3 || prec == 4) ? one + (double)kB * NC * a.TWc * 8.0
                      : 2.0 * one * (prec == BF_FP32 ? 1.0 : prec == 5 ? 0.75 : 0.5);
  const double per_step = mod + pass;
  const double flops = per_step * a.steps * (double)a.nsx * a.nsy;
  return flops / 50e12 * 1e6;
}

struct Req {
  uint64_t ticket = 0;
  bf_request in{};
  double Cm[64] = {0};
  double Wm[64] = {0};
  int R = 0, variant = 0, stream = 0;   // variant: the server's instance id (d, R, kvar, p64, TW)
  int kvar = 0;                         // kernel variant (precision, running-sum box pass)
  FusedArgs a{};
  size_t n_acc = 0, n_tab = 0, off_w = 0, off_taps = 0;
  int nparts = 0;
  size_t dev_bytes = 0, pin_bytes = 0, dev_off = 0, pin_off = 0;
  bool has_dev = false, has_pin = false, need_minmax = false;
  float* part = nullptr;  // device reduction partials (nparts*17) then result (17)
  size_t n_part = 0, n_img = 0, n_out = 0;   // floats: partials, uploaded image, device output
  float* dev_img = nullptr;   // arena copy of a host image (f_host), or null
  float* dev_out = nullptr;   // arena output when the caller gives only out_host
  float* pin = nullptr;   // pinned: min/max result (17, padded to 32) then term table
  double cost_term = 0.0;
  int next_t = 0;
  int K_run = 0;          // kernel terms: K, or the distinct +-Y count
  hipEvent_t ev_mm = nullptr, ev_done = nullptr;
  // shared with callers (guarded by the server mutex)
  int state = BF_REQ_QUEUED, error = 0, N_used = 0, chunks = 0;
  std::string msg;
  double t_arrival = 0, t_admit = 0, t_start = 0, t_done = 0;
};

struct Round {
  std::vector<hipEvent_t> evs;         // end of the round's work on each stream it used
  std::vector<hipEvent_t> starts;      // its start on that stream (timing events)
  std::vector<double> model_us;        // modelled device time of its launches there
  std::vector<hipGraphExec_t> execs;   // graph rounds: freed when the round has passed
  std::vector<hipGraph_t> graphs;
};

}  // namespace

struct Server {
  bf_server_config cfg{};
  int device = 0;
  Clock::time_point epoch;
  char* dev_base = nullptr;
  char* pin_base = nullptr;
  Arena dev_arena, pin_arena;
  std::vector<hipStream_t> streams;
  hipStream_t aux = nullptr;
  hipStream_t tune_stream = nullptr;   // autotune probes at submit (cfg.autotune)
  std::mutex tune_mu;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::deque<Req*> incoming;
  // (d, R, kernel variant, p64, strip width) -> id
  std::map<std::tuple<int, int, int, int, int>, int> variants;
  uint64_t next_ticket = 1;
  bool stop = false;
  int queued = 0, admitted = 0;
  bf_server_stats stats{};

  // scheduler-thread state
  std::multimap<std::pair<double, uint64_t>, Req*> pending;
  std::vector<Req*> preparing, active, finishing;
  std::deque<Round> rounds;
  std::vector<hipEvent_t> event_pool, tevent_pool;
  int fatal = 0;
  std::string fatal_msg;
  std::thread worker;
  uint64_t fault_at = 0, launch_count = 0;   // BF_FAULT_INJECT=launch:<n> (test hook)

  double now() const {
    return std::chrono::duration<double>(Clock::now() - epoch).count();
  }

  hipEvent_t take_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
  void give_event(hipEvent_t& e) {
    if (e) event_pool.push_back(e);
    e = nullptr;
  }
  // timing-enabled events: the start and end of a round on each stream
  hipEvent_t take_tevent() {
    if (!tevent_pool.empty()) {
      hipEvent_t e = tevent_pool.back();
      tevent_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void give_tevent(hipEvent_t& e) {
    if (e) tevent_pool.push_back(e);
    e = nullptr;
  }
  // Measured device time of the rounds over their modelled time, a running
  // average over rounds (each stream of a round one sample; concurrent
  // streams share the device, so a sample measures the time its work took
  // there, which is what a round's length is made of).
  double model_scale = 1.0;
  // event polling interval of the scheduler thread while the device is busy
  static constexpr int kPollMinUs = 20, kPollMaxUs = 160;
  int poll_us = kPollMinUs;
  void calibrate(const Round& rd) {
    for (size_t i = 0; i < rd.starts.size() && i < rd.evs.size(); ++i) {
      float ms = 0.0f;
      if (!rd.starts[i] || !rd.evs[i] || rd.model_us[i] <= 0.0 ||
          hipEventElapsedTime(&ms, rd.starts[i], rd.evs[i]) != hipSuccess)
        continue;
      const double ratio = std::min(20.0, std::max(0.05, 1e3 * ms / rd.model_us[i]));
      model_scale += 0.2 * (ratio - model_scale);
    }
    std::lock_guard<std::mutex> lk(mu);
    stats.model_scale = (float)model_scale;
  }

  void release(Req* r) {
    if (r->has_dev) dev_arena.release(r->dev_off);
    if (r->has_pin) pin_arena.release(r->pin_off);
    r->has_dev = r->has_pin = false;
    give_event(r->ev_mm);
    give_event(r->ev_done);
  }

  // Record the end of a request (caller holds no lock).
  void finish(Req* r, int state, int error, const std::string& msg) {
    release(r);
    std::lock_guard<std::mutex> lk(mu);
    r->state = state;
    r->error = error;
    r->msg = msg;
    r->t_done = now();
    --admitted;
    if (state == BF_REQ_DONE) ++stats.completed;
    else ++stats.failed;
    cv_done.notify_all();
  }

  // First device error: the server fails every request from then on.  Only
  // the scheduler thread writes these; submit reads them under the mutex.
  void set_fatal(hipError_t e, const char* what) {
    std::lock_guard<std::mutex> lk(mu);
    if (fatal) return;
    fatal = BF_EDEVICE;
    fatal_msg = std::string(what) + ": " + hipGetErrorString(e);
  }

  // ---- preparation ----------------------------------------------------------
  bool prepare_terms(Req* r, const float* lo, const float* hi) {
    const int d = r->in.d;
    int N = r->in.N;
    if (N == 0 && choose_order(d, r->Wm, lo, hi, &N) != BF_OK) {
      finish(r, BF_REQ_FAILED, BF_EUNSUPPORTED, bf_last_error());
      return false;
    }
    std::vector<double> w, weight;
    if (r->in.dedup) {
      distinct_terms(d, r->Wm, N, r->in.K, r->in.seed, &w, &weight);
    } else {
      w.resize((size_t)r->in.K * d);
      frequency_table(d, r->Wm, N, r->in.K, r->in.seed, w.data());
    }
    const int K = r->in.dedup ? (int)weight.size() : r->in.K;
    size_t off_w = 0, off_taps = 0;
    const std::vector<float> tab = term_table(d, K, w.data(), r->in.dedup ? weight.data() : nullptr,
                                              r->in.sigma_s, &off_w, &off_taps,
                                              spatial_boxes(r->in.spatial));
    for (int m = 0; m < 8; ++m)
      r->a.cen[m] = (r->in.center && m < d) ? (float)(0.5 * ((double)lo[m] + (double)hi[m])) : 0.0f;
    if ((r->in.precision == BF_FP16 || r->in.precision == BF_FP32_SPLIT) &&
        check_fp16_range(d, r->in.sigma_s, spatial_boxes(r->in.spatial), lo, hi, r->a.cen) != BF_OK) {
      finish(r, BF_REQ_FAILED, BF_EUNSUPPORTED, bf_last_error());
      return false;
    }
    // the extrema are known when the min/max ran (order rule, centring, FP16)
    table_wmax(d, K, tab.data(), r->a.wmax);
    r->a.p64 = phase64_flag(d, r->a.wmax, r->a.cen, r->need_minmax ? lo : nullptr,
                            r->need_minmax ? hi : nullptr);
    {  // kernel instance (d, R, variant, FP64-phase path, strip width): its id picks the stream
      std::lock_guard<std::mutex> lk(mu);
      const auto key = std::make_tuple(d, r->R, r->kvar, r->a.p64, r->a.TWc);
      auto it = variants.find(key);
      if (it == variants.end()) it = variants.emplace(key, (int)variants.size()).first;
      r->variant = it->second;
      r->stream = r->variant % cfg.streams;
    }
    float* ptab = r->pin + 32;
    std::memcpy(ptab, tab.data(), tab.size() * sizeof(float));
    float* dtab = reinterpret_cast<float*>(dev_base + r->dev_off) + r->n_acc;
    hipError_t e = hipMemcpyAsync(dtab, ptab, tab.size() * sizeof(float), hipMemcpyHostToDevice,
                                  streams[r->stream]);
    if (e != hipSuccess) {
      set_fatal(e, "term table upload");
      finish(r, BF_REQ_FAILED, BF_EDEVICE, fatal_msg);
      return false;
    }
    r->a.terms = dtab;
    r->a.terms_lo = dtab + (size_t)K * (d + 1);
    r->a.weights = r->in.dedup ? dtab + off_w : nullptr;
    r->a.taps = dtab + off_taps;
    r->K_run = K;
    std::lock_guard<std::mutex> lk(mu);
    r->N_used = N;
    r->state = BF_REQ_RUNNING;
    active.push_back(r);
    return true;
  }

  bool admit() {
    bool progress = false;
    const double t = now();
    while (!pending.empty() && !fatal) {
      Req* r = pending.begin()->second;
      if (r->t_arrival > t || admitted >= cfg.max_active) break;
      size_t doff = 0, poff = 0;
      if (!dev_arena.alloc(r->dev_bytes, &doff)) break;  // arrival order: no overtaking
      if (!pin_arena.alloc(r->pin_bytes, &poff)) {
        dev_arena.release(doff);
        break;
      }
      pending.erase(pending.begin());
      r->dev_off = doff;
      r->pin_off = poff;
      r->has_dev = r->has_pin = true;
      float* dev = reinterpret_cast<float*>(dev_base + doff);
      r->a.acc = dev;
      {
        const size_t b_part = Arena::round_up((r->n_acc + r->n_tab) * sizeof(float), kAlign);
        const size_t b_img = b_part + Arena::round_up(r->n_part * sizeof(float), kAlign);
        const size_t b_out = b_img + Arena::round_up(r->n_img * sizeof(float), kAlign);
        r->part = reinterpret_cast<float*>(dev_base + doff + b_part);
        r->dev_img = r->n_img ? reinterpret_cast<float*>(dev_base + doff + b_img) : nullptr;
        r->dev_out = r->n_out ? reinterpret_cast<float*>(dev_base + doff + b_out) : nullptr;
      }
      r->pin = reinterpret_cast<float*>(pin_base + poff);
      r->ev_done = take_event();
      {
        std::lock_guard<std::mutex> lk(mu);
        --queued;
        ++admitted;
        r->state = BF_REQ_PREPARING;
        r->t_admit = t;
      }
      progress = true;
      if (!r->ev_done) {
        finish(r, BF_REQ_FAILED, BF_EDEVICE, "hipEventCreate failed");
        continue;
      }
      if (r->need_minmax) {
        r->ev_mm = take_event();
        float* res = r->part + (size_t)r->nparts * kMMFloats;
        hipError_t e = r->ev_mm ? hipSuccess : hipErrorOutOfMemory;
        if (e == hipSuccess && r->dev_img) {
          // host image: upload it first (its pitch kept on the host side)
          const size_t row = (size_t)r->in.W * r->in.d * sizeof(float);
          e = hipMemcpy2DAsync(r->dev_img, row, r->in.f_host,
                               (size_t)r->in.pitch * r->in.d * sizeof(float), row, r->in.H,
                               hipMemcpyHostToDevice, aux);
          r->a.f = r->dev_img;
          r->a.fpitch = r->in.W;
        }
        if (e == hipSuccess)
          e = launch_minmax(r->a.f, r->in.H, r->in.W, r->a.fpitch, r->in.d, r->part, r->nparts,
                            res, aux);
        if (e == hipSuccess)
          e = hipMemcpyAsync(r->pin, res, kMMFloats * sizeof(float), hipMemcpyDeviceToHost, aux);
        if (e == hipSuccess) e = hipEventRecord(r->ev_mm, aux);
        if (e != hipSuccess) {
          set_fatal(e, "min/max reduction");
          finish(r, BF_REQ_FAILED, BF_EDEVICE, fatal_msg);
          continue;
        }
        preparing.push_back(r);
      } else {
        const float zero[8] = {0};
        prepare_terms(r, zero, zero);
      }
    }
    return progress;
  }

  bool finish_preparing() {
    bool progress = false;
    for (size_t i = 0; i < preparing.size();) {
      Req* r = preparing[i];
      const hipError_t q = hipEventQuery(r->ev_mm);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      preparing.erase(preparing.begin() + i);
      progress = true;
      if (q != hipSuccess) {
        set_fatal(q, "min/max reduction");
        finish(r, BF_REQ_FAILED, BF_EDEVICE, fatal_msg);
        continue;
      }
      const float* h = r->pin;
      if (h[16] != 0.0f) {
        finish(r, BF_REQ_FAILED, BF_EINVAL, "f contains NaN or infinity");
        continue;
      }
      prepare_terms(r, h, h + 8);
    }
    return progress;
  }

  // ---- rounds ---------------------------------------------------------------
  bool enqueue_round() {
    if (active.empty() || (int)rounds.size() >= cfg.depth || fatal) return false;
    std::vector<PlanJob> jobs;
    jobs.reserve(active.size());
    for (size_t i = 0; i < active.size(); ++i)
      jobs.push_back(PlanJob{(int)i, active[i]->variant, active[i]->next_t, active[i]->K_run,
                             active[i]->cost_term * model_scale});
    const std::vector<PlanLaunch> plan = plan_round(jobs, cfg.quantum_us, kMaxBatch, cfg.policy);
    Round rd;
    std::map<int, bool> capturing;   // graph rounds: streams being captured
    auto begin_capture = [&](int si) -> hipError_t {
      if (!cfg.graph_rounds || capturing.count(si)) return hipSuccess;
      capturing[si] = true;
      return hipStreamBeginCapture(streams[si], hipStreamCaptureModeRelaxed);
    };
    // a device error while streams are being captured: end the captures
    // (their graphs are discarded) before the error path touches the streams
    auto abort_captures = [&] {
      for (auto& kv : capturing) {
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(streams[kv.first], &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      }
      capturing.clear();
      // and the round's start events go back to the pool (the round is dropped)
      for (hipEvent_t& ev : rd.starts) give_tevent(ev);
      rd.starts.clear();
      rd.model_us.clear();
    };
    std::map<int, size_t> stream_slot;   // stream -> index into rd.starts / rd.model_us
    std::vector<Req*> ended;
    std::set<Req*> failed;
    std::string failed_msg;
    size_t n_failed_launches = 0;
    const double t = now();
    uint64_t wgs = 0;
    for (const PlanLaunch& L : plan) {
      BatchArgs b{};
      b.n = (int)L.items.size();
      b.first[0] = 0;
      Req* r0 = active[L.items[0].job];
      for (int k = 0; k < b.n; ++k) {
        Req* r = active[L.items[k].job];
        b.req[k] = r->a;
        b.req[k].t0 = L.items[k].t0;
        b.req[k].t1 = L.items[k].t1;
        b.first[k + 1] = b.first[k] + r->a.nsx * r->a.nsy;
      }
      hipStream_t st = streams[r0->stream];
      const bool injected = fault_at != 0 && ++launch_count == fault_at;
      if (!stream_slot.count(r0->stream)) {
        // the round's start on this stream (outside any capture)
        hipEvent_t ev = take_tevent();
        if (!ev || hipEventRecord(ev, st) != hipSuccess) {
          give_tevent(ev);
          set_fatal(hipErrorUnknown, "round start event");
          abort_captures();
          return true;
        }
        stream_slot[r0->stream] = rd.starts.size();
        rd.starts.push_back(ev);
        rd.model_us.push_back(0.0);
      }
      hipError_t e = begin_capture(r0->stream);
      if (e != hipSuccess) {
        set_fatal(e, "round capture");
        abort_captures();
        return true;
      }
      e = injected ? hipErrorLaunchFailure : launch_fused_batch(r0->in.d, r0->R, r0->kvar, b, st);
      if (e != hipSuccess && cfg.graph_rounds && !injected) {
        set_fatal(e, "batched fused launch under capture");
        abort_captures();
        return true;
      }
      if (e != hipSuccess) {
        // Refused at launch (arguments, resources, or the injected fault):
        // nothing of it runs and the device stays usable, so only this
        // launch's requests fail, once their earlier chunks on the stream
        // have drained (their arena blocks are then free to reuse).
        (void)hipGetLastError();
        if (cfg.graph_rounds) {   // no stream drain while capturing: the server fails
          abort_captures();
          set_fatal(e, "batched fused launch refused in a graph round");
          return true;
        }
        failed_msg = std::string(injected ? "injected fault: " : "") +
                     "batched fused launch: " + hipGetErrorString(e);
        const hipError_t q = hipStreamSynchronize(st);
        if (q != hipSuccess) {
          set_fatal(q, "stream drain after a refused launch");
          abort_captures();
          return true;
        }
        for (const PlanItem& it : L.items) failed.insert(active[it.job]);
        ++n_failed_launches;
        continue;
      }
      wgs += (uint64_t)b.first[b.n];
      for (const PlanItem& it : L.items)
        rd.model_us[stream_slot[r0->stream]] += (it.t1 - it.t0) * active[it.job]->cost_term;
      for (const PlanItem& it : L.items) {
        Req* r = active[it.job];
        r->next_t = it.t1;
        if (r->next_t < r->K_run) continue;
        FinalizeArgs fa{};
        fa.acc = r->a.acc;
        fa.out = r->in.out ? r->in.out : r->dev_out;
        for (int m = 0; m < 8; ++m) fa.cen[m] = r->a.cen[m];
        fa.H = r->in.H;
        fa.W = r->in.W;
        fa.Hp = r->a.Hp;
        fa.Wp = r->a.nsx * r->a.TWc;
        e = launch_finalize(r->in.d, fa, st);
        if (e == hipSuccess && r->in.out_host)
          e = hipMemcpyAsync(r->in.out_host, fa.out,
                             (size_t)r->in.H * r->in.W * r->in.d * sizeof(float),
                             hipMemcpyDeviceToHost, st);
        // the completion event follows the stream's graph in graph rounds
        if (e == hipSuccess && !cfg.graph_rounds) e = hipEventRecord(r->ev_done, st);
        if (e != hipSuccess) {
          set_fatal(e, "finalize launch");
          abort_captures();
          return true;
        }
        ended.push_back(r);
      }
    }
    // graph rounds: end each stream's capture and launch its graph; then the
    // completion events of the requests that ended on it
    for (auto& kv : capturing) {
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      hipError_t e = hipStreamEndCapture(streams[kv.first], &g);
      if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (e == hipSuccess) e = hipGraphLaunch(x, streams[kv.first]);
      if (g) rd.graphs.push_back(g);
      if (x) rd.execs.push_back(x);
      if (e != hipSuccess) {
        set_fatal(e, "graph round");
        rounds.push_back(std::move(rd));
        return true;
      }
    }
    if (cfg.graph_rounds)
      for (Req* r : ended)
        if (hipEventRecord(r->ev_done, streams[r->stream]) != hipSuccess) {
          set_fatal(hipErrorUnknown, "completion event");
          rounds.push_back(std::move(rd));
          return true;
        }
    // the round's end on every stream it started on, in the order of
    // rd.starts (a stream whose launches were all refused ends at once)
    std::vector<hipEvent_t> ends(rd.starts.size(), nullptr);
    for (const auto& kv : stream_slot) {
      hipEvent_t ev = take_tevent();
      if (!ev || hipEventRecord(ev, streams[kv.first]) != hipSuccess) {
        set_fatal(hipErrorUnknown, "round event");
        give_tevent(ev);
        break;
      }
      ends[kv.second] = ev;
    }
    for (size_t i = 0; i < ends.size(); ++i) {
      if (ends[i]) continue;   // fatal above: keep the lists aligned for the cleanup
      ends[i] = rd.starts[i];
      rd.starts[i] = nullptr;
    }
    rd.evs = std::move(ends);
    rounds.push_back(std::move(rd));
    {
      std::lock_guard<std::mutex> lk(mu);
      for (const PlanLaunch& L : plan)
        for (const PlanItem& it : L.items) {
          Req* r = active[it.job];
          if (failed.count(r)) continue;
          ++r->chunks;
          if (r->t_start == 0.0) r->t_start = t;
        }
      ++stats.rounds;
      stats.launches += plan.size() - n_failed_launches;
      stats.workgroups += wgs;
    }
    for (Req* r : ended) finishing.push_back(r);
    std::vector<Req*> still;
    still.reserve(active.size());
    for (Req* r : active)
      if (!failed.count(r) && r->next_t < r->K_run) still.push_back(r);
    active.swap(still);
    for (Req* r : failed) finish(r, BF_REQ_FAILED, BF_EDEVICE, failed_msg);
    return true;
  }

  bool reap_rounds() {
    bool progress = false;
    while (!rounds.empty()) {
      Round& rd = rounds.front();
      bool done = true;
      for (hipEvent_t ev : rd.evs) {
        const hipError_t q = hipEventQuery(ev);
        if (q == hipErrorNotReady) {
          done = false;
          break;
        }
        if (q != hipSuccess) set_fatal(q, "round");
      }
      if (!done) break;
      calibrate(rd);
      for (hipEvent_t& ev : rd.evs) give_tevent(ev);
      for (hipEvent_t& ev : rd.starts) give_tevent(ev);
      for (hipGraphExec_t x : rd.execs) (void)hipGraphExecDestroy(x);
      for (hipGraph_t g : rd.graphs) (void)hipGraphDestroy(g);
      rounds.pop_front();
      progress = true;
    }
    return progress;
  }

  bool reap_done() {
    bool progress = false;
    for (size_t i = 0; i < finishing.size();) {
      Req* r = finishing[i];
      const hipError_t q = hipEventQuery(r->ev_done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      finishing.erase(finishing.begin() + i);
      progress = true;
      if (q != hipSuccess) {
        set_fatal(q, "request completion");
        finish(r, BF_REQ_FAILED, BF_EDEVICE, fatal_msg);
      } else {
        finish(r, BF_REQ_DONE, BF_OK, "");
      }
    }
    return progress;
  }

  // After a device error: wait for what was queued, then fail everything.
  void fail_all() {
    for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(aux);
    for (Round& rd : rounds) {
      for (hipEvent_t& ev : rd.evs) give_tevent(ev);
      for (hipEvent_t& ev : rd.starts) give_tevent(ev);
      for (hipGraphExec_t x : rd.execs) (void)hipGraphExecDestroy(x);
      for (hipGraph_t g : rd.graphs) (void)hipGraphDestroy(g);
    }
    rounds.clear();
    std::vector<Req*> all;
    for (auto* v : {&preparing, &active, &finishing}) {
      all.insert(all.end(), v->begin(), v->end());
      v->clear();
    }
    for (Req* r : all) finish(r, BF_REQ_FAILED, fatal, fatal_msg);
    for (auto& kv : pending) {
      std::lock_guard<std::mutex> lk(mu);
      Req* r = kv.second;
      r->state = BF_REQ_FAILED;
      r->error = fatal;
      r->msg = fatal_msg;
      --queued;
      ++stats.failed;
    }
    pending.clear();
    std::lock_guard<std::mutex> lk(mu);
    cv_done.notify_all();
  }

  void run() {
    (void)hipSetDevice(device);
    for (;;) {
      bool stopping;
      {
        std::lock_guard<std::mutex> lk(mu);
        while (!incoming.empty()) {
          Req* r = incoming.front();
          incoming.pop_front();
          pending.emplace(std::make_pair(r->t_arrival, r->ticket), r);
        }
        stopping = stop;
      }
      if (stopping && !pending.empty()) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : pending) {
          kv.second->state = BF_REQ_CANCELLED;
          --queued;
        }
        pending.clear();
        cv_done.notify_all();
      }
      if (fatal) fail_all();
      const bool busy = !preparing.empty() || !active.empty() || !finishing.empty() ||
                        !rounds.empty();
      if (stopping && !busy) break;
      bool progress = reap_done();
      progress |= reap_rounds();
      progress |= finish_preparing();
      progress |= admit();
      progress |= enqueue_round();
      if (progress) {
        poll_us = kPollMinUs;
        continue;
      }
      if (busy) {
        // device work in flight and nothing to do until some of it ends:
        // poll its events with a backoff (doubling up to kPollMaxUs while
        // nothing changes), woken at once by a submission
        std::unique_lock<std::mutex> lk(mu);
        if (incoming.empty() && !stop) cv_work.wait_for(lk, std::chrono::microseconds(poll_us));
        poll_us = std::min(2 * poll_us, kPollMaxUs);
        continue;
      }
      // idle: sleep until a submission, the next arrival, or stop
      std::unique_lock<std::mutex> lk(mu);
      if (!incoming.empty() || stop) continue;
      if (pending.empty()) {
        cv_work.wait(lk, [&] { return !incoming.empty() || stop; });
      } else {
        const double wait_s = pending.begin()->first.first - now();
        if (wait_s > 0)
          cv_work.wait_for(lk, std::chrono::duration<double>(std::min(wait_s, 1.0)));
      }
    }
  }

  void fill_status(const Req* r, bf_request_status* st) const {
    std::memset(st, 0, sizeof(*st));
    st->state = r->state;
    st->error = r->error;
    st->N_used = r->N_used;
    st->chunks = r->chunks;
    st->arrival = r->t_arrival;
    st->admitted = r->t_admit;
    st->started = r->t_start;
    st->done = r->t_done;
    std::strncpy(st->message, r->msg.c_str(), sizeof(st->message) - 1);
  }
};

namespace {

bool ended(int state) {
  return state == BF_REQ_DONE || state == BF_REQ_FAILED || state == BF_REQ_CANCELLED;
}

int hip_err(hipError_t e, const char* what) {
  return fail(BF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Validate a request and plan its launch geometry and footprint.
int plan_request(Server* s, const bf_request* q, Req* r) {
  if (!q) return fail(BF_EINVAL, "req must be non-null");
  r->in = *q;
  bf_request& in = r->in;
  if (in.pitch == 0) in.pitch = in.W;
  if ((in.f != nullptr) == (in.f_host != nullptr))
    return fail(BF_EINVAL, "give exactly one of f (device) and f_host (host)");
  if (!in.out && !in.out_host) return fail(BF_EINVAL, "give out (device) or out_host (host)");
  if (in.H < 1 || in.W < 1 || in.H > 65536 || in.W > 65536)
    return fail(BF_EINVAL, "H and W must be in [1, 65536]");
  if (in.d < 1 || in.d > 8) return fail(BF_EINVAL, "d must be in [1, 8]");
  if (in.pitch < in.W) return fail(BF_EINVAL, "pitch must be 0 or >= W");
  if (!std::isfinite(in.sigma_s) || in.sigma_s < 0.0 || in.sigma_s > 32.0)
    return fail(BF_EINVAL, "sigma_s must be finite and in [0, 32]");
  if (in.K < 1 || in.K > 65536) return fail(BF_EINVAL, "K must be in [1, 65536]");
  if (in.N < 0 || in.N > 65536) return fail(BF_EINVAL, "N must be 0 (auto) or in [1, 65536]");
  if (in.precision != BF_FP32 && in.precision != BF_FP16 && in.precision != BF_BF16 &&
      in.precision != BF_FP32_SPLIT)
    return fail(BF_EINVAL, "precision must be BF_FP32, BF_FP16, BF_BF16 or BF_FP32_SPLIT");
  if (in.center != 0 && in.center != 1) return fail(BF_EINVAL, "center must be 0 or 1");
  if (in.dedup != 0 && in.dedup != 1) return fail(BF_EINVAL, "dedup must be 0 or 1");
  if (int rs = check_spatial(in.spatial, in.precision)) return rs;
  if (!in.C) return fail(BF_EINVAL, "C must be non-null");
  if (!std::isfinite(in.arrival)) return fail(BF_EINVAL, "arrival must be finite");
  {
    const size_t fbytes = (((size_t)in.H - 1) * in.pitch + in.W) * in.d * sizeof(float);
    const size_t obytes = (size_t)in.H * in.W * in.d * sizeof(float);
    const char* a = (const char*)in.f;
    const char* b = (const char*)in.out;
    if (a && b && a < b + obytes && b < a + fbytes) return fail(BF_EINVAL, "out must not overlap f");
    const char* ah = (const char*)in.f_host;
    const char* bh = (const char*)in.out_host;
    if (ah && bh && ah < bh + obytes && bh < ah + fbytes)
      return fail(BF_EINVAL, "out_host must not overlap f_host");
  }
  std::memcpy(r->Cm, in.C, sizeof(double) * in.d * in.d);
  in.C = r->Cm;
  int rc = whiten(in.d, r->Cm, r->Wm, in.whiten);
  if (rc) return rc;
  r->R = window_radius(in.sigma_s, spatial_boxes(in.spatial));
  r->kvar = select_variant(in.d, r->R, in.precision, in.spatial, in.W, 0, 0);
  if ((rc = check_fused_size(in.H, in.W, in.pitch, in.d, r->R))) return rc;
  int TH = 0, TW = 0;
  {
    // occupancy queries need the server's device current on this thread
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != s->device) e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_err(e, "hipSetDevice");
    rc = choose_strip_width(in.d, r->R, r->kvar, in.H, in.W, 0, &TW);
    // autotune: measure this size class once, on the request's own image
    if (!rc && s->cfg.autotune && in.f && r->kvar <= 2 && spatial_boxes(in.spatial) == 0 &&
        !tuned_class_known(in.d, r->R, r->kvar, in.H, in.W, TW)) {
      std::lock_guard<std::mutex> tk(s->tune_mu);
      if (!tuned_class_known(in.d, r->R, r->kvar, in.H, in.W, TW))
        rc = autotune_strip_height(in.f, in.H, in.W, in.pitch, in.d, in.sigma_s, in.precision,
                                   s->tune_stream, nullptr, nullptr);
    }
    if (!rc) rc = choose_strip_height(in.d, r->R, r->kvar, in.H, in.W, 0, &TH, TW);
    if (cur != s->device) (void)hipSetDevice(cur);
    if (rc) return rc;
  }
  fused_geometry(r->a, in.H, in.W, r->R, r->kvar, TH,
                 r->kvar == 3 ? spatial_boxes(in.spatial) : 0, TW);
  if ((rc = check_acc_size(r->a, in.d))) return rc;
  r->a.f = in.f;
  r->a.fpitch = in.pitch;
  r->n_acc = fused_acc_floats(r->a, in.d);
  // term table at most K rows of d+1 floats, K weights (merged draws), 2R+1 taps
  // hi and lo term rows, weights, taps (term_table's layout)
  r->n_tab = (size_t)in.K * (2 * in.d + 3) + (size_t)(2 * r->R + 1);
  // a host image is uploaded on the reduction's stream before the kernels
  r->need_minmax = in.N == 0 || in.center || in.precision == BF_FP16 ||
                   in.precision == BF_FP32_SPLIT || in.f_host;
  r->nparts = minmax_parts((size_t)in.H * in.W);
  r->n_part = r->need_minmax ? (size_t)r->nparts * kMMFloats + kMMResult : 0;
  r->n_img = in.f_host ? (size_t)in.H * in.W * in.d : 0;
  r->n_out = in.out ? 0 : (size_t)in.H * in.W * in.d;
  r->dev_bytes = Arena::round_up((r->n_acc + r->n_tab) * sizeof(float), kAlign) +
                 Arena::round_up(r->n_part * sizeof(float), kAlign) +
                 Arena::round_up(r->n_img * sizeof(float), kAlign) +
                 Arena::round_up(r->n_out * sizeof(float), kAlign);
  r->pin_bytes = (32 + r->n_tab) * sizeof(float);
  r->cost_term = model_term_us(r->a, in.d, r->kvar);
  if (!s->dev_arena.fits_ever(r->dev_bytes))
    return fail(BF_ENOMEM, "request footprint exceeds the server's device arena");
  if (!s->pin_arena.fits_ever(r->pin_bytes))
    return fail(BF_ENOMEM, "request term table exceeds the server's host staging");
  return BF_OK;
}

Req* find(Server* s, uint64_t ticket) {
  auto it = s->reqs.find(ticket);
  return it == s->reqs.end() ? nullptr : it->second.get();
}

}  // namespace
}  // namespace bfvec

struct bf_server : bfvec::Server {};

using namespace bfvec;

extern "C" {

void bf_server_config_init(bf_server_config* cfg) {
  if (cfg) std::memset(cfg, 0, sizeof(*cfg));
}

void bf_request_init(bf_request* req) {
  if (!req) return;
  std::memset(req, 0, sizeof(*req));
  req->precision = BF_FP16;
  req->center = 1;
}

int bf_server_create(const bf_server_config* cfg_in, bf_server** out) {
  clear_error();
  if (!out) return fail(BF_EINVAL, "srv must be non-null");
  *out = nullptr;
  bf_server_config cfg{};
  if (cfg_in) cfg = *cfg_in;
  if (cfg.arena_bytes == 0) cfg.arena_bytes = 8ull << 30;
  if (cfg.max_active == 0) cfg.max_active = 64;
  if (cfg.streams == 0) cfg.streams = 4;
  if (cfg.depth == 0) cfg.depth = 2;
  if (cfg.quantum_us == 0.0) cfg.quantum_us = 2000.0;
  if (cfg.max_active < 1 || cfg.max_queued < 0 || cfg.streams < 1 || cfg.streams > 16 ||
      cfg.depth < 1 || !(cfg.quantum_us > 0.0) || cfg.arena_bytes < (1u << 20) ||
      (cfg.policy != BF_POLICY_SHARE && cfg.policy != BF_POLICY_SHORTEST_FIRST) ||
      (cfg.autotune != 0 && cfg.autotune != 1) || (cfg.graph_rounds != 0 && cfg.graph_rounds != 1))
    return fail(BF_EINVAL, "bad server configuration");
  auto s = std::make_unique<bf_server>();
  s->cfg = cfg;
  s->stats.model_scale = 1.0f;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  // host staging: one term table per admitted request at most K = 65536, d = 8
  const size_t pin_bytes = (size_t)cfg.max_active * 4096 * 10 * sizeof(float) + (64u << 20);
  e = hipMalloc((void**)&s->dev_base, cfg.arena_bytes);
  if (e != hipSuccess) return fail(BF_ENOMEM, "device arena allocation failed");
  e = hipHostMalloc((void**)&s->pin_base, pin_bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(s->dev_base);
    return fail(BF_ENOMEM, "pinned staging allocation failed");
  }
  s->dev_arena.reset(cfg.arena_bytes, kAlign);
  if (const char* fi = std::getenv("BF_FAULT_INJECT")) {
    unsigned long long n = 0;
    if (std::sscanf(fi, "launch:%llu", &n) == 1) s->fault_at = n;
  }
  s->pin_arena.reset(pin_bytes, kAlign);
  for (int i = 0; i <= cfg.streams && e == hipSuccess; ++i) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) (i < cfg.streams ? s->streams.push_back(st) : (void)(s->aux = st));
  }
  if (e == hipSuccess && cfg.autotune) e = hipStreamCreateWithFlags(&s->tune_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    if (s->aux) (void)hipStreamDestroy(s->aux);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->dev_base);
    (void)hipHostFree(s->pin_base);
    return hip_err(e, "hipStreamCreate");
  }
  s->stats.arena_bytes = cfg.arena_bytes;
  s->epoch = Clock::now();
  Server* raw = s.get();
  s->worker = std::thread([raw] { raw->run(); });
  *out = s.release();
  return BF_OK;
}

int bf_server_submit(bf_server* s, const bf_request* q, uint64_t* ticket) {
  clear_error();
  if (!s || !ticket) return fail(BF_EINVAL, "srv and ticket must be non-null");
  auto r = std::make_unique<Req>();
  int rc = plan_request(s, q, r.get());
  if (rc) return rc;
  const double t = s->now();
  r->t_arrival = r->in.arrival > 0.0 ? r->in.arrival : t;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(BF_EINVAL, "server is shutting down");
  if (s->fatal) return fail(s->fatal, s->fatal_msg);
  if (s->cfg.max_queued > 0 && s->queued >= s->cfg.max_queued)
    return fail(BF_EBUSY, "serving queue full");
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  Req* raw = r.get();
  s->reqs.emplace(r->ticket, std::move(r));
  s->incoming.push_back(raw);
  ++s->queued;
  ++s->stats.submitted;
  s->cv_work.notify_one();
  return BF_OK;
}

int bf_server_poll(bf_server* s, uint64_t ticket, bf_request_status* st) {
  clear_error();
  if (!s || !st) return fail(BF_EINVAL, "srv and st must be non-null");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(BF_EINVAL, "unknown ticket");
  s->fill_status(r, st);
  return BF_OK;
}

int bf_server_wait(bf_server* s, uint64_t ticket, double timeout_s, bf_request_status* st) {
  clear_error();
  if (!s) return fail(BF_EINVAL, "srv must be non-null");
  std::unique_lock<std::mutex> lk(s->mu);
  Req* r = find(s, ticket);
  if (!r) return fail(BF_EINVAL, "unknown ticket");
  auto done = [&] { return ended(r->state); };
  bool ok = true;
  if (timeout_s < 0) s->cv_done.wait(lk, done);
  else ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
  if (st) s->fill_status(r, st);
  if (!ok) return fail(BF_ETIMEDOUT, "request still in flight");
  return BF_OK;
}

int bf_server_drain(bf_server* s, double timeout_s) {
  clear_error();
  if (!s) return fail(BF_EINVAL, "srv must be non-null");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    for (auto& kv : s->reqs)
      if (!ended(kv.second->state)) return false;
    return true;
  };
  bool ok = true;
  if (timeout_s < 0) s->cv_done.wait(lk, done);
  else ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
  if (!ok) return fail(BF_ETIMEDOUT, "requests still in flight");
  return BF_OK;
}

int bf_server_forget(bf_server* s, uint64_t ticket) {
  clear_error();
  if (!s) return fail(BF_EINVAL, "srv must be non-null");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BF_EINVAL, "unknown ticket");
  if (!ended(it->second->state)) return fail(BF_EBUSY, "request has not ended");
  s->reqs.erase(it);
  return BF_OK;
}

int bf_server_get_stats(bf_server* s, bf_server_stats* out) {
  clear_error();
  if (!s || !out) return fail(BF_EINVAL, "srv and stats must be non-null");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->arena_peak = s->dev_arena.peak();
  out->admitted = s->admitted;
  out->queued = s->queued;
  return BF_OK;
}

double bf_server_clock(const bf_server* s) { return s ? s->now() : 0.0; }

int bf_server_destroy(bf_server* s) {
  clear_error();
  if (!s) return BF_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  if (s->aux) (void)hipStreamSynchronize(s->aux);
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->tevent_pool) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->aux) (void)hipStreamDestroy(s->aux);
  if (s->tune_stream) {
    (void)hipStreamSynchronize(s->tune_stream);
    (void)hipStreamDestroy(s->tune_stream);
  }
  (void)hipFree(s->dev_base);
  (void)hipHostFree(s->pin_base);
  delete s;
  return BF_OK;
}

}  // extern "C"
