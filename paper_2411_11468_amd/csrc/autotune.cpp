// autotune.cpp -- search over the degree-class thresholds, slice size and
// block shapes of lpa_tuning for one graph (or one packed batch of graphs):
// successive halving over a grid of candidates, each measured as the wall
// time of complete runs with the caller's options.  Built on the public C ABI
// only (lpa_create / lpa_run / lpa_destroy).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "host_common.h"

using namespace lpa;

namespace {

struct Cand {
  lpa_tuning t;
  double ms = 0.0;      // median of the last round
  bool ok = false;
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::vector<lpa_tuning> grid(const lpa_tuning& base) {
  std::vector<lpa_tuning> out;
  out.push_back(base);  // the defaults are always a candidate
  for (int s4 : {2, 4})
    for (int s16 : {8, 16})
      for (int wv : {128, 256, 512})
        for (int bl : {2048, 4096, 8192})
          for (int ch : {4096, 8192}) {
            lpa_tuning t = base;
            t.small4 = s4;
            t.small16 = s16;
            t.wave = wv;
            t.block = bl;
            t.hub_chunk = ch;
            if (std::memcmp(&t, &base, sizeof(t)) != 0) out.push_back(t);
          }
  return out;
}

}  // namespace

extern "C" lpa_status lpa_autotune(const lpa_csr* csr, int32_t num_graphs, const int64_t* v_off,
                                   void* stream, const lpa_options* opt, double budget_ms,
                                   lpa_tuning* best, lpa_tune_report* report) {
  if (!csr || !best) return fail(LPA_ERR_INVALID, "NULL argument");
  if (num_graphs < 0 || (num_graphs > 0 && !v_off))
    return fail(LPA_ERR_INVALID, "num_graphs < 0 or v_off is NULL");
  if (!(budget_ms > 0.0)) return fail(LPA_ERR_INVALID, "budget_ms must be > 0");
  lpa_options o;
  if (opt) o = *opt; else lpa_options_default(&o);
  o.profile = 0;
  o.learned = 0;
  lpa_tuning base;
  lpa_tuning_default(&base);
  std::vector<Cand> cands;
  for (const lpa_tuning& t : grid(base)) cands.push_back(Cand{t, 0.0, false});
  const int64_t n = csr->num_vertices;
  int32_t* labels = nullptr;
  if (hipMalloc(&labels, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LPA_ERR_OOM, "hipMalloc failed for the labels");
  }
  lpa_csr c = *csr;
  const double t_start = now_ms();
  int32_t runs = 0;
  double default_ms = -1.0;
  lpa_status err = LPA_OK;
  // one candidate: build a handle, one warm-up run, reps timed runs (median)
  auto measure = [&](Cand& cd, int reps) -> lpa_status {
    lpa_graph g = nullptr;
    lpa_status e = num_graphs > 0
                       ? lpa_create_batched(num_graphs, v_off, &c, stream, &cd.t, &g)
                       : lpa_create(&c, stream, &cd.t, &g);
    if (e != LPA_OK) return e;
    c.validate = 0;  // the first creation validated the graph
    std::vector<double> ts;
    for (int r = 0; r <= reps && e == LPA_OK; ++r) {
      const double t0 = now_ms();
      e = num_graphs > 0 ? lpa_run_batched(g, &o, labels, nullptr, nullptr, nullptr)
                         : lpa_run(g, &o, labels, nullptr, 0, nullptr);
      if (r > 0) ts.push_back(now_ms() - t0);
      ++runs;
    }
    lpa_destroy(g);
    if (e != LPA_OK) return e;
    std::sort(ts.begin(), ts.end());
    cd.ms = ts[ts.size() / 2];
    cd.ok = true;
    return LPA_OK;
  };
  std::vector<Cand*> alive;
  for (Cand& cd : cands) alive.push_back(&cd);
  int reps = 1;
  int32_t rounds = 0;
  while (true) {
    for (Cand* cd : alive) {
      if (now_ms() - t_start > budget_ms && cd != alive.front()) break;
      if ((err = measure(*cd, reps)) != LPA_OK) break;
      if (cd == &cands[0] && default_ms < 0.0) default_ms = cd->ms;
    }
    ++rounds;
    if (err != LPA_OK) break;
    std::vector<Cand*> done;
    for (Cand* cd : alive)
      if (cd->ok) done.push_back(cd);
    std::sort(done.begin(), done.end(), [](Cand* a, Cand* b) { return a->ms < b->ms; });
    const size_t keep = std::max<size_t>(1, (done.size() + 2) / 3);
    done.resize(std::min(done.size(), keep));
    alive = done;
    if (alive.size() <= 1 || now_ms() - t_start > budget_ms) break;
    for (Cand* cd : alive) cd->ok = false;
    reps *= 2;
  }
  (void)hipFree(labels);
  if (err != LPA_OK) return err;
  if (alive.empty()) return fail(LPA_ERR_STATE, "no candidate could be measured");
  *best = alive.front()->t;
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->candidates = (int32_t)cands.size();
    report->runs = runs;
    report->rounds = rounds;
    report->best_ms = alive.front()->ms;
    report->default_ms = default_ms;
    report->elapsed_ms = now_ms() - t_start;
  }
  return LPA_OK;
}
