// autotune.cpp -- search over lpa_tuning for one graph (or one packed batch of
// graphs) by successive halving, each candidate measured as the wall time of
// complete runs with the caller's options.  Built on the public C ABI only
// (lpa_create / lpa_create_batched / lpa_run / lpa_destroy).
//
// The search goes in stages, each over a grid around the best tuning so far
// (the defaults included in the first):
//   batch     (batched handles) the schedule: the work-queue kernel with
//             chunks of 128..1024 vertices and 16-lane rows up to 16, 32 or
//             64 entries, or the class kernels over the packed CSR;
//   classes   the degree-class thresholds (small4 2/4, small16 8/16, wave
//             128/256/512, block 2048/4096/8192) and the hub slice size
//             (4096/8192);
//   shapes    threads per workgroup of the workgroup classes (the per-class
//             defaults, or 256/512/1024 for all of them), the hashtable
//             capacity rule (load up to 1, 1/2 or 1/4) and the push/pull
//             crossover of the neighbour flags (1/8, 1/16 or 1/32 of the
//             entries).
// A batch that the work queue wins skips the other two stages, which tune
// kernels it does not run.
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
  bool dead = false;    // the handle could not be built with this tuning
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

void add_unique(std::vector<lpa_tuning>& out, const lpa_tuning& t) {
  for (const lpa_tuning& u : out)
    if (std::memcmp(&u, &t, sizeof(t)) == 0) return;
  out.push_back(t);
}

std::vector<lpa_tuning> grid_batch(const lpa_tuning& base) {
  std::vector<lpa_tuning> out;
  out.push_back(base);
  lpa_tuning c = base;
  c.batch_queue = 0;
  add_unique(out, c);
  for (int ch : {128, 256, 512, 1024})
    for (int gr : {16, 32, 64}) {
      lpa_tuning t = base;
      t.batch_queue = 1;
      t.queue_chunk = ch;
      t.queue_group = gr;
      add_unique(out, t);
    }
  return out;
}

std::vector<lpa_tuning> grid_classes(const lpa_tuning& base) {
  std::vector<lpa_tuning> out;
  out.push_back(base);
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
            add_unique(out, t);
          }
  return out;
}

std::vector<lpa_tuning> grid_shapes(const lpa_tuning& base) {
  std::vector<lpa_tuning> out;
  out.push_back(base);
  for (int bt : {0, 256, 512, 1024})
    for (int ld : {1, 2, 4})
      for (int pd : {8, 16, 32}) {
        lpa_tuning t = base;
        t.block_threads = bt;
        t.table_load = ld;
        t.pull_divisor = pd;
        add_unique(out, t);
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
  const int64_t n = csr->num_vertices;
  int32_t* labels = nullptr;
  if (hipMalloc(&labels, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LPA_ERR_OOM, "hipMalloc failed for the labels");
  }
  lpa_csr c = *csr;
  const double t_start = now_ms();
  int32_t runs = 0, rounds = 0, total = 0;
  double default_ms = -1.0;
  lpa_status err = LPA_OK;
  // one candidate: build a handle, one warm-up run, reps timed runs (median);
  // a tuning the handle refuses (LPA_ERR_UNSUPPORTED) drops out
  auto measure = [&](Cand& cd, int reps) -> lpa_status {
    lpa_graph g = nullptr;
    lpa_status e = num_graphs > 0
                       ? lpa_create_batched(num_graphs, v_off, &c, stream, &cd.t, &g)
                       : lpa_create(&c, stream, &cd.t, &g);
    if (e == LPA_ERR_UNSUPPORTED) {
      cd.dead = true;
      return LPA_OK;
    }
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
  // successive halving over one stage's grid until the wall time `until`;
  // the winner and its measured time go to *win, *win_ms
  auto halving = [&](const std::vector<lpa_tuning>& grid, double until,
                     lpa_tuning* win, double* win_ms) -> lpa_status {
    std::vector<Cand> cands;
    for (const lpa_tuning& t : grid) cands.push_back(Cand{t, 0.0, false, false});
    total += (int32_t)cands.size();
    std::vector<Cand*> alive;
    for (Cand& cd : cands) alive.push_back(&cd);
    int reps = 1;
    while (true) {
      for (Cand* cd : alive) {
        // the first candidate (the stage's base) is always measured
        if (now_ms() > until && cd != alive.front()) break;
        if (lpa_status e = measure(*cd, reps)) return e;
        if (default_ms < 0.0 && cd->ok) default_ms = cd->ms;
      }
      ++rounds;
      std::vector<Cand*> done;
      for (Cand* cd : alive)
        if (cd->ok) done.push_back(cd);
      std::sort(done.begin(), done.end(), [](Cand* a, Cand* b) { return a->ms < b->ms; });
      const size_t keep = std::max<size_t>(1, (done.size() + 2) / 3);
      done.resize(std::min(done.size(), keep));
      alive = done;
      if (alive.size() <= 1 || now_ms() > until) break;
      for (Cand* cd : alive) cd->ok = false;
      reps *= 2;
    }
    if (alive.empty()) return fail(LPA_ERR_STATE, "no candidate could be measured");
    *win = alive.front()->t;
    *win_ms = alive.front()->ms;
    return LPA_OK;
  };
  lpa_tuning cur = base;
  double cur_ms = 0.0;
  bool queue_won = false;
  if (num_graphs > 0) {
    err = halving(grid_batch(cur), t_start + budget_ms / 3.0, &cur, &cur_ms);
    if (err == LPA_OK && cur.batch_queue == -1) {
      // the defaults won: they take the queue unless a row is too long for it
      lpa_tuning t = cur;
      t.batch_queue = 1;
      lpa_graph g = nullptr;
      const lpa_status e = lpa_create_batched(num_graphs, v_off, &c, stream, &t, &g);
      if (e == LPA_OK) lpa_destroy(g);
      else if (e != LPA_ERR_UNSUPPORTED) err = e;
      cur.batch_queue = e == LPA_OK ? 1 : 0;
    }
    queue_won = err == LPA_OK && cur.batch_queue == 1;
  }
  if (err == LPA_OK && !queue_won) {
    err = halving(grid_classes(cur), t_start + budget_ms * 2.0 / 3.0, &cur, &cur_ms);
    if (err == LPA_OK) err = halving(grid_shapes(cur), t_start + budget_ms, &cur, &cur_ms);
  }
  (void)hipFree(labels);
  if (err != LPA_OK) return err;
  *best = cur;
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->candidates = total;
    report->runs = runs;
    report->rounds = rounds;
    report->best_ms = cur_ms;
    report->default_ms = default_ms;
    report->elapsed_ms = now_ms() - t_start;
  }
  return LPA_OK;
}
