// Host-only parts of the serving scheduler: the device-memory arena that
// admission control draws from, and the round planner of continuous batching.
// No HIP here, so the logic is testable on any host compiler.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <map>
#include <vector>

namespace bfvec {

// First-fit allocator over a range of `bytes` bytes; hands out offsets aligned
// to `align`.  Freed blocks merge with free neighbours.
class Arena {
 public:
  explicit Arena(size_t bytes = 0, size_t align = 256) { reset(bytes, align); }

  void reset(size_t bytes, size_t align = 256) {
    align_ = align;
    size_ = bytes / align * align;
    free_.clear();
    used_.clear();
    in_use_ = peak_ = 0;
    if (size_) free_[0] = size_;
  }

  static size_t round_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

  // true and *off on success; false when no free block is large enough
  bool alloc(size_t n, size_t* off) {
    n = round_up(std::max<size_t>(n, 1), align_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t o = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[o + n] = rest;
      used_[o] = n;
      in_use_ += n;
      peak_ = std::max(peak_, in_use_);
      *off = o;
      return true;
    }
    return false;
  }

  // false if off is not the start of a live block
  bool release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t o = off, n = u->second;
    used_.erase(u);
    in_use_ -= n;
    auto next = free_.lower_bound(o);
    if (next != free_.end() && next->first == o + n) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == o) {
        o = prev->first;
        n += prev->second;
        free_.erase(prev);
      }
    }
    free_[o] = n;
    return true;
  }

  bool fits_ever(size_t n) const { return round_up(std::max<size_t>(n, 1), align_) <= size_; }
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  size_t blocks() const { return used_.size(); }

  // Internal consistency: blocks tile [0, size) without overlap, free blocks
  // never touch each other, byte counts agree.
  bool check() const {
    std::map<size_t, std::pair<size_t, bool>> all;
    for (auto& kv : free_) all[kv.first] = {kv.second, true};
    for (auto& kv : used_) {
      if (all.count(kv.first)) return false;
      all[kv.first] = {kv.second, false};
    }
    size_t pos = 0, used = 0;
    bool prev_free = false;
    for (auto& kv : all) {
      if (kv.first != pos || kv.second.first == 0 || kv.first % align_) return false;
      if (kv.second.second && prev_free) return false;
      prev_free = kv.second.second;
      if (!kv.second.second) used += kv.second.first;
      pos += kv.second.first;
    }
    return pos == size_ && used == in_use_;
  }

 private:
  size_t align_ = 256, size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_, used_;
};

// One admitted request as the planner sees it.
struct PlanJob {
  int job;               // caller's index
  int variant;           // kernel instance (d, R, precision); one launch per variant group
  int next_t, K;         // terms done so far, and in total
  double cost_per_term;  // modelled device time of one term over the whole image
};

struct PlanItem {
  int job;
  int t0, t1;            // terms of this round
};

struct PlanLaunch {
  int variant;
  std::vector<PlanItem> items;
};

// Round policies: processor sharing (every job advances by one quantum of
// modelled time per round), or shortest remaining work first (the round's
// budget, one quantum per job, goes to the jobs with the least modelled work
// left, each taking all it needs, in that order; jobs past the budget wait).
enum { kPolicyShare = 0, kPolicyShortestFirst = 1 };

// One round of continuous batching.  kPolicyShare: every job in `jobs`
// (admission order) gets the next chunk of its terms, as many as fit in
// `quantum` of modelled time (at least one, at most what is left), so a small
// request finishes in its first round while a large one advances a quantum at
// a time (round-robin processor sharing).  kPolicyShortestFirst: jobs in
// order of remaining modelled work (ties: admission order) take all their
// remaining terms while the round's budget of quantum x (number of jobs)
// lasts; the job that crosses the budget takes the terms that fit (at least
// one), the rest get none this round.  Jobs of one variant share launches of
// at most `max_batch` jobs each, launches ordered by first appearance.
inline std::vector<PlanLaunch> plan_round(const std::vector<PlanJob>& jobs, double quantum,
                                          int max_batch, int policy = kPolicyShare) {
  std::vector<PlanLaunch> out;
  std::map<int, size_t> open;  // variant -> index of its last launch in out
  std::vector<size_t> order(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) order[i] = i;
  std::vector<int> take(jobs.size(), 0);
  if (policy == kPolicyShortestFirst) {
    auto work = [&](size_t i) {
      return (double)std::max(0, jobs[i].K - jobs[i].next_t) * jobs[i].cost_per_term;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return work(x) < work(y); });
    double budget = quantum * (double)jobs.size();
    for (size_t i : order) {
      const int left = jobs[i].K - jobs[i].next_t;
      if (left <= 0 || budget <= 0.0) continue;
      int n = left;
      if (jobs[i].cost_per_term > 0.0 && work(i) > budget)
        n = (int)std::max(1.0, std::floor(budget / jobs[i].cost_per_term));
      take[i] = n;
      budget -= n * jobs[i].cost_per_term;
    }
  }
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const PlanJob& j = jobs[order[oi]];
    const int left = j.K - j.next_t;
    if (left <= 0) continue;
    int n = left;
    if (policy == kPolicyShortestFirst) {
      n = take[order[oi]];
      if (n <= 0) continue;
    } else if (j.cost_per_term > 0.0 && quantum > 0.0) {
      const double q = std::ceil(quantum / j.cost_per_term);
      n = (int)std::max(1.0, std::min((double)left, q));
    }
    auto it = open.find(j.variant);
    if (it == open.end() || (int)out[it->second].items.size() >= max_batch) {
      out.push_back(PlanLaunch{j.variant, {}});
      open[j.variant] = out.size() - 1;
      it = open.find(j.variant);
    }
    out[it->second].items.push_back(PlanItem{j.job, j.next_t, j.next_t + n});
  }
  return out;
}

// Nearest-rank percentile of v (q in [0, 100]); 0 for an empty vector.
inline double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double r = std::ceil(q / 100.0 * (double)v.size());
  const size_t i = (size_t)std::min<double>(std::max(r, 1.0), (double)v.size()) - 1;
  return v[i];
}

}  // namespace bfvec
