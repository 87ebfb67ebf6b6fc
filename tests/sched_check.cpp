// Host checks of the serving scheduler's arena and round planner
// (paper_1605_02164_amd/csrc/scheduler.h), built with g++ by
// tests/test_server_host.py.  Prints one "PASS <name>" or "FAIL <name>: why"
// line per check.

#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "scheduler.h"

using namespace bfvec;

static int failures = 0;

static void report(const char* name, const std::string& why) {
  if (why.empty()) {
    std::printf("PASS %s\n", name);
  } else {
    std::printf("FAIL %s: %s\n", name, why.c_str());
    ++failures;
  }
}

// Random alloc/release sequences against a byte map: blocks never overlap,
// stay aligned and inside the arena, the free list stays coalesced, and an
// allocation fails only when no run of free bytes is long enough.
static std::string arena_random(unsigned seed) {
  std::mt19937_64 rng(seed);
  const size_t align = 256, size = 1 << 20;
  Arena A(size, align);
  std::vector<int> owner(size / align, -1);  // per aligned unit
  std::vector<std::pair<size_t, size_t>> live;  // (off, units)
  for (int step = 0; step < 4000; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const size_t n = 1 + rng() % (size / 16);
      size_t off = 0;
      const size_t units = (n + align - 1) / align;
      if (A.alloc(n, &off)) {
        if (off % align) return "unaligned offset";
        if (off + units * align > size) return "block past the end";
        for (size_t u = off / align; u < off / align + units; ++u) {
          if (owner[u] != -1) return "overlapping blocks";
          owner[u] = step;
        }
        live.push_back({off, units});
      } else {
        size_t run = 0, best = 0;
        for (int o : owner) {
          run = o == -1 ? run + 1 : 0;
          best = std::max(best, run);
        }
        if (best >= units) return "allocation failed with a long enough free run";
      }
    } else {
      const size_t i = rng() % live.size();
      if (!A.release(live[i].first)) return "release of a live block failed";
      for (size_t u = live[i].first / align; u < live[i].first / align + live[i].second; ++u)
        owner[u] = -1;
      live.erase(live.begin() + i);
    }
    if (!A.check()) return "inconsistent block lists at step " + std::to_string(step);
    size_t used = 0;
    for (auto& b : live) used += b.second * align;
    if (A.in_use() != used) return "in_use disagrees";
  }
  for (auto& b : live)
    if (!A.release(b.first)) return "final release failed";
  if (A.in_use() != 0 || !A.check()) return "arena not empty at the end";
  size_t off = 0;
  if (!A.alloc(size, &off) || off != 0) return "free list did not coalesce back to one block";
  if (A.release(off + align)) return "release of a non-block offset succeeded";
  if (A.fits_ever(size + 1)) return "fits_ever past the size";
  return "";
}

// Rounds until every job is done: each job's chunks are contiguous from 0 to
// K, one per round it takes part in, at least one term and at most the
// quantum's worth (unless one term alone exceeds it); launches hold one
// variant and at most max_batch jobs; a job whose remaining work fits the
// quantum finishes in that round.
static std::string planner_random(unsigned seed) {
  std::mt19937_64 rng(seed);
  for (int trial = 0; trial < 200; ++trial) {
    const int nj = 1 + rng() % 40, max_batch = 1 + rng() % 16;
    const double quantum = 50.0 + (rng() % 5000);
    std::vector<PlanJob> jobs;
    for (int j = 0; j < nj; ++j)
      jobs.push_back(PlanJob{j, (int)(rng() % 5), 0, 1 + (int)(rng() % 300),
                             0.5 + (rng() % 2000) / 10.0});
    int rounds = 0;
    for (;;) {
      std::vector<PlanJob> act;
      for (auto& j : jobs)
        if (j.next_t < j.K) act.push_back(j);
      if (act.empty()) break;
      if (++rounds > 100000) return "no termination";
      const auto plan = plan_round(act, quantum, max_batch);
      std::vector<int> seen(nj, 0);
      for (const auto& L : plan) {
        if (L.items.empty() || (int)L.items.size() > max_batch) return "bad launch size";
        for (const auto& it : L.items) {
          PlanJob& j = jobs[it.job];
          if (j.variant != L.variant) return "job in another variant's launch";
          if (seen[it.job]++) return "job twice in one round";
          if (it.t0 != j.next_t) return "chunk not contiguous";
          if (it.t1 <= it.t0 || it.t1 > j.K) return "empty or overlong chunk";
          const int n = it.t1 - it.t0;
          if (n > 1 && (n - 1) * j.cost_per_term >= quantum) return "chunk above the quantum";
          if ((j.K - j.next_t) * j.cost_per_term <= quantum && it.t1 != j.K)
            return "small remainder not finished in one round";
          j.next_t = it.t1;
        }
      }
      for (auto& j : act)
        if (!seen[j.job]) return "active job left out of a round";
    }
  }
  std::vector<PlanJob> none;
  if (!plan_round(none, 100.0, 4).empty()) return "plan of no jobs not empty";
  return "";
}

// Shortest-remaining-work-first rounds: chunks stay contiguous and every job
// finishes; each round's modelled work stays within quantum x (active jobs)
// plus one term; the job with the least remaining work is served first and
// runs to completion whenever the budget allows; a served job with less
// remaining work than an unserved one never exists.
static std::string planner_shortest_first(unsigned seed) {
  std::mt19937_64 rng(seed);
  for (int trial = 0; trial < 200; ++trial) {
    const int nj = 1 + rng() % 40, max_batch = 1 + rng() % 16;
    const double quantum = 50.0 + (rng() % 5000);
    std::vector<PlanJob> jobs;
    for (int j = 0; j < nj; ++j)
      jobs.push_back(PlanJob{j, (int)(rng() % 5), 0, 1 + (int)(rng() % 300),
                             0.5 + (rng() % 2000) / 10.0});
    int rounds = 0;
    for (;;) {
      std::vector<PlanJob> act;
      for (auto& j : jobs)
        if (j.next_t < j.K) act.push_back(j);
      if (act.empty()) break;
      if (++rounds > 100000) return "no termination";
      const auto plan = plan_round(act, quantum, max_batch, kPolicyShortestFirst);
      if (plan.empty()) return "round with active jobs but no work";
      std::vector<int> seen(nj, 0);
      double work = 0.0, max_term = 0.0;
      for (auto& j : act) max_term = std::max(max_term, j.cost_per_term);
      double least = 1e300;
      for (auto& j : act) least = std::min(least, (j.K - j.next_t) * j.cost_per_term);
      double served_max = -1.0, unserved_min = 1e300;
      std::vector<double> rem(nj, 0.0);
      for (auto& j : act) rem[j.job] = (j.K - j.next_t) * j.cost_per_term;
      for (const auto& L : plan) {
        if (L.items.empty() || (int)L.items.size() > max_batch) return "bad launch size";
        for (const auto& it : L.items) {
          PlanJob& j = jobs[it.job];
          if (j.variant != L.variant) return "job in another variant's launch";
          if (seen[it.job]++) return "job twice in one round";
          if (it.t0 != j.next_t) return "chunk not contiguous";
          if (it.t1 <= it.t0 || it.t1 > j.K) return "empty or overlong chunk";
          work += (it.t1 - it.t0) * j.cost_per_term;
          if (rem[it.job] == least && least <= quantum * act.size() && it.t1 != j.K)
            return "shortest job not finished within the budget";
          served_max = std::max(served_max, rem[it.job]);
          j.next_t = it.t1;
        }
      }
      for (auto& j : act)
        if (!seen[j.job]) unserved_min = std::min(unserved_min, rem[j.job]);
      if (work > quantum * act.size() + max_term + 1e-6) return "round above its budget";
      if (unserved_min < served_max) return "a shorter job waited while a longer one ran";
    }
  }
  return "";
}

static std::string percentiles() {
  std::vector<double> v;
  for (int i = 100; i >= 1; --i) v.push_back(i);
  if (percentile(v, 50) != 50 || percentile(v, 99) != 99 || percentile(v, 100) != 100 ||
      percentile(v, 0) != 1)
    return "nearest rank of 1..100";
  if (percentile({7.0}, 99) != 7.0 || percentile({}, 50) != 0.0) return "edge cases";
  if (percentile({1, 2, 3}, 50) != 2) return "median of three";
  return "";
}

int main() {
  report("arena_random_seed1", arena_random(1));
  report("arena_random_seed2", arena_random(2));
  report("planner_random", planner_random(3));
  report("planner_shortest_first", planner_shortest_first(4));
  report("percentiles", percentiles());
  return failures ? 1 : 0;
}
