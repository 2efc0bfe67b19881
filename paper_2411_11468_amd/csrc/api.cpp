// api.cpp -- host runtime of the label-propagation library and its C ABI
// (declared in include/lpa.h).  Owns device memory, builds the degree classes
// at create time and drives the iterations of Algorithm 1 (lpa): per
// iteration it enqueues the hub plan, the frontier, the class sweeps and (in
// deterministic mode) the label apply, reads back the iteration counters and
// applies the stop rule.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lpa.h"
#include "host_common.h"
#include "lpa_internal.h"
#include "lpa_mlp.h"

using namespace lpa;

namespace lpa {

thread_local std::string g_err;

lpa_status fail(lpa_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace lpa

namespace {

// kernel ids of the optional profile
constexpr int kKidPlan = 0, kKidFrontier = 1, kKidHubPart = 2, kKidSweep0 = 2,
              kKidHubFin = 11, kKidApply = 12, kKidPull = 13, kKidPullHubs = 14,
              kKidPush = 15, kKidPushHubs = 16, kKidDecide = 17, kKidHubReduce = 18,
              kKidBatch = 19, kKidHubSpill = 20, kKidDirect0 = 20, kKidHubDirect = 29,
              kKidQueueSweep = 30, kKidQueueStep = 31, kNumKids = 32;
const char* const kKidNames[kNumKids] = {
    "hub_plan", "frontier", "hub_part", "sweep_small4", "sweep_small16", "sweep_wave127",
    "sweep_wave1023", "sweep_block2047", "sweep_block4095", "sweep_block8191",
    "sweep_block16383", "hub_fin", "apply", "pull_flags", "pull_hubs", "push_flags",
    "push_hubs", "flag_decide", "hub_reduce", "batch_step", "hub_spill", "direct_small4",
    "direct_small16", "direct_wave127", "direct_wave1023", "direct_block2047",
    "direct_block4095", "direct_block8191", "direct_block16383", "hub_direct", "queue_sweep",
    "queue_step"};

}  // namespace

struct RunCtx;

struct lpa_graph_s {
  hipStream_t stream = nullptr;
  int64_t n = 0, m = 0;
  bool off64 = false;
  bool strict_rows = false;   // every row's targets strictly increase
  const void* off = nullptr;     // CSR the kernels read: the internal order
  const int32_t* tgt = nullptr;  // when relabeled, else the caller's arrays
  const float* w = nullptr;
  const void* uoff = nullptr;    // the caller's CSR (uploaded or borrowed)
  const int32_t* utgt = nullptr;
  int32_t* ctgt = nullptr;       // internal rows with the caller's ids (or NULL)
  uint32_t* chg_bits = nullptr;  // the change bytes as bits, for the pull kernels
  const float* uw = nullptr;
  int32_t* perm = nullptr;       // caller id -> internal id; NULL: one order
  int32_t* inv = nullptr;        // internal id -> caller id
  uint8_t* stage8 = nullptr;     // n bytes, flags in the caller's order
  unsigned long long* stage64 = nullptr;  // n records in the caller's order
  uint32_t* probe_sink = nullptr;         // lpa_label_read_rate
  bool flags_pending = false;  // the last run left its final flags to chg
  int32_t* cc_prev = nullptr;  // Cross-Check: labels before the iteration
  uint8_t* cc_rev = nullptr;   // Cross-Check: revert decisions (zero between uses)
  lpa_tuning tun{};
  uint8_t* cls = nullptr;
  int32_t* C = nullptr;
  uint8_t* F = nullptr;
  int32_t* lists[kNumClasses] = {};
  int64_t cls_count[kNumClasses] = {};
  // vertices that can be flagged after the first iteration: in the internal
  // order (by degree, largest first) those of degree 0 come last and are
  // left out; in the caller's order all n
  int64_t n_active = 0;
  int grid[kNumClasses] = {};
  int direct_grid[kNumClasses] = {};  // table-free first sweep
  int tv_grid[kNumClasses] = {};      // table_values 32 / 64: sweep_tv.hip
  void* tv_gvals = nullptr;           // hubs' table values of that width
  unsigned long long* tv_vmax = nullptr;
  uint32_t* tv_nl = nullptr;
  int frontier_grid = 1, apply_grid = 1, hub_acc_grid = 1, hub_fin_grid = 1, pull_grid = 1,
      push_grid = 1, hub_direct_grid = 1;
  int32_t* pend_v = nullptr;
  int32_t* pend_c = nullptr;
  int32_t* Cn = nullptr;
  uint8_t* chg = nullptr;
  DevStats* st = nullptr;
  DevStats* st_host = nullptr;
  int32_t H = 0;
  int32_t* hub_vid = nullptr;
  int64_t* hub_tab = nullptr;
  unsigned long long* hub_best = nullptr;
  int32_t* hub_old = nullptr;
  uint32_t* gkeys = nullptr;
  float* gvals = nullptr;
  uint32_t* items = nullptr;
  uint32_t* bitems = nullptr;
  uint32_t* witems = nullptr;     // hub slices grouped by target window (or NULL)
  unsigned int* wctr = nullptr;   // their pop counters
  uint32_t wbase[kXcds + 1] = {};
  uint32_t* part_keys = nullptr;
  float* part_vals = nullptr;
  uint32_t* boff = nullptr;
  uint32_t* bsize = nullptr;   // per queued bucket: pairs over all slices
  int32_t* hub_bq = nullptr;   // per hub: queue index of its bucket 0
  int32_t* hub_nch = nullptr;
  int32_t* hub_ovf = nullptr;
  int32_t* hub_lgb = nullptr;
  int64_t* hub_slice0 = nullptr;
  int64_t* hub_boff0 = nullptr;
  int64_t max_items = 0, max_bitems = 0;
  int hub_reduce_grid = 8;
  double* mod_sig = nullptr;
  double* mod_acc = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<void*> dev_allocs;
  size_t dev_bytes = 0;          // bytes held in dev_allocs
  // optional per-kernel profile: events bracketing each launch, and the
  // accumulated launches, time and algorithmic bytes per kernel
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kid;
  lpa_kernel_profile prof[kNumKids] = {};

  lpa_status ensure_events(int count) {
    while ((int)ev_pool.size() < count) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return fail(LPA_ERR_HIP, "hipEventCreate failed");
      ev_pool.push_back(e);
      ev_kid.push_back(-1);
    }
    return LPA_OK;
  }

  // Algorithmic bytes of one launch: what the method must read and write,
  // independent of caching (per scanned CSR entry: target 4 B, weight 4 B
  // unless unit weights, gathered neighbour label 4 B; per processed vertex:
  // its active-list id 4 B, its two row offsets, its own label 4 B, and in
  // deterministic mode its next label 4 B; per change: the new label 4 B in
  // asynchronous mode (a queued hub pair 8 B in deterministic mode) and one
  // flag byte per neighbour).
  // flag_mode: 0 pushed, 1 pulled, 2 deferred to lpa_get_flags
  void account(int kid, float ms, const DevStats& h, bool async_mode, int flag_mode) {
    const bool pull = flag_mode == 1, push = flag_mode == 0;
    if (kid < 0 || kid >= kNumKids) return;
    lpa_kernel_profile& p = prof[kid];
    // first iteration from labels = ids: the neighbour labels are not
    // gathered; the table-free kernels read the caller's rows, where the
    // targets are the labels, and know each vertex's own label
    const bool id0 = h.iter == 1 && h.ident;
    const bool direct = (kid > kKidDirect0 && kid <= kKidDirect0 + 8) || kid == kKidHubDirect;
    const double eb = ((id0 || direct) ? 4.0 : 8.0) + (w ? 4.0 : 0.0);
    const double ob = off64 ? 16.0 : 8.0;
    const double chb = async_mode ? 4.0 : 8.0;
    double bytes = 0.0;
    int64_t edges = 0, verts = 0;
    if ((kid >= kKidSweep0 + 1 && kid <= kKidSweep0 + 8) || (direct && kid != kKidHubDirect)) {
      const int c = direct ? kid - kKidDirect0 : kid - kKidSweep0;
      edges = (int64_t)h.edges[c];
      verts = (int64_t)h.active[c];
      // own label: read, or (table-free) the caller id through inv when
      // the handle keeps an internal order
      const double own = direct ? (perm ? 4.0 : 0.0) : 4.0;
      // table-free sweep of rows up to 4 entries: internal rows, each
      // target's caller id read from inv
      const double ebc = eb + ((direct && c == 1 && perm) ? 4.0 : 0.0);
      bytes = ebc * edges + (4.0 + ob + own) * verts + (double)h.changed[c] +
              (async_mode ? 4.0 * h.changed[c] : 4.0 * verts);
      if (acct_feat && c >= acct_feat_cmin && c <= acct_feat_cmax)
        bytes += 16.0 * verts;  // state record read and written
    } else if (kid == kKidHubPart || kid == kKidHubDirect) {
      edges = (int64_t)h.edges[kClassHub];
      bytes = eb * edges;
    } else if (kid == kKidHubReduce) {
      // not the method's bytes: the (label, sum) pairs the slices wrote,
      // 8 B each, read back and reduced per bucket (their entries)
      edges = (int64_t)h.hub_pairs;
      bytes = 8.0 * (double)h.hub_pairs;
    } else if (kid == kKidHubFin) {
      bytes = chb * h.changed[kClassHub] + (double)h.changed[kClassHub];
    } else if (kid == kKidFrontier) {
      verts = (int64_t)h.processed;
      // flag, class and change byte per vertex; flag clear + list id per
      // taken vertex
      bytes = 3.0 * n + 5.0 * (double)h.processed;
      // learned frontier: the record of every predicted or traced vertex
      if (acct_feat) bytes += 8.0 * (double)(h.processed + h.skipped);
    } else if (kid == kKidPull || kid == kKidPullHubs) {
      // row offsets and class per vertex, target + change byte per entry
      // read, flag byte per vertex; the two kernels share one counter, so
      // the whole figure is booked on the first
      if (kid == kKidPull && pull) {
        edges = (int64_t)h.pull_scanned;
        bytes = (double)n * ((off64 ? 8.0 : 4.0) + 2.0) + 5.0 * (double)h.pull_scanned;
      }
    } else if (kid == kKidPush || kid == kKidPushHubs) {
      // per changed row: its offsets and, per entry, target read + flag byte
      if (kid == kKidPush && push) {
        unsigned long long fw = 0, ch = 0, listed = 0;
        for (int c = 0; c < kNumClasses; ++c) { fw += h.flagw[c]; ch += h.changed[c]; }
        for (int c = 1; c < kClassHub; ++c) listed += h.active[c];
        edges = (int64_t)fw;
        bytes = 5.0 * (double)listed + (off64 ? 16.0 : 8.0) * (double)ch + 5.0 * (double)fw;
      }
    } else if (kid == kKidQueueSweep) {
      // per scanned entry as the class sweeps; per processed vertex its flag,
      // offsets and own label (and the next label in deterministic mode);
      // per change the new label (asynchronous mode)
      edges = (int64_t)h.edges[0];
      verts = (int64_t)h.processed;
      bytes = eb * edges + (1.0 + ob + 4.0 + (async_mode ? 0.0 : 4.0)) * verts +
              (async_mode ? 4.0 * h.changed[0] : 0.0);
    } else if (kid == kKidBatch) {
      bytes = 2.0 * n;  // change byte read, flag cleared at most once
    } else if (kid == kKidApply) {
      unsigned long long listed = 0;
      for (int c = 1; c < kClassHub; ++c) listed += h.active[c];
      verts = (int64_t)(h.pending + listed);
      bytes = 12.0 * (double)h.pending + 12.0 * (double)listed;
    }
    p.launches += 1;
    p.total_ms += ms;
    p.bytes += bytes;
    p.edges += edges;
    p.vertices += verts;
  }

  template <typename T>
  lpa_status dalloc(T** p, int64_t count) {
    void* q = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    if (tun.memory_limit_kib > 0 &&
        dev_bytes + bytes > (size_t)tun.memory_limit_kib * 1024u) {
      *p = nullptr;
      return fail(LPA_ERR_OOM, "the handle's device memory limit (" +
                                   std::to_string(tun.memory_limit_kib) +
                                   " KiB) would be exceeded by " + std::to_string(bytes) +
                                   " more bytes");
    }
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(LPA_ERR_OOM, "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " +
                                   hipGetErrorString(e));
    }
    dev_allocs.push_back(q);
    dev_bytes += bytes;
    *p = static_cast<T*>(q);
    return LPA_OK;
  }

  // device history of per-iteration statistics
  DevIterStats* hist = nullptr;
  int32_t hist_cap = 0;
  // batched runs
  int32_t G = 0;
  const int64_t* b_voff = nullptr;
  uint8_t* b_done = nullptr;
  int32_t* b_iters = nullptr;
  long long* b_changed = nullptr;
  // batched runs as a work queue (queue.hip)
  bool wq = false;             // queue structures built at create
  int wq_grid = 1;
  int32_t wq_chunk_log2 = 9;
  int32_t wq_group = 64;
  int64_t wq_nchunks = 0;
  int64_t* wq_cbase = nullptr;
  int32_t* wq_cgraph = nullptr;
  uint32_t* wq_items = nullptr;
  uint32_t* wq_items0 = nullptr;     // the initial queue
  int64_t* wq_qbase = nullptr;
  unsigned int* wq_qctr = nullptr;
  unsigned int* wq_qctr0 = nullptr;  // the initial queue's counters
  uint8_t* wq_cmark = nullptr;
  uint8_t* wq_F1 = nullptr;
  unsigned int* wq_gchanged = nullptr;
  QueueArgs queue_args(int async_mode) const {
    QueueArgs q;
    q.off = off; q.tgt = tgt; q.w = w;
    q.C0 = C; q.C1 = async_mode ? C : Cn;
    q.F0 = F; q.F1 = wq_F1;
    q.cmark = wq_cmark; q.cbase = wq_cbase; q.cgraph = wq_cgraph;
    q.items = wq_items; q.qbase = wq_qbase; q.qctr = wq_qctr; q.gchanged = wq_gchanged;
    q.b = batch_args(); q.st = st;
    q.nchunks = wq_nchunks; q.chunk_log2 = wq_chunk_log2; q.group_max = wq_group;
    q.async_mode = async_mode;
    q.strict_rows = strict_rows ? 1 : 0;
    q.probe = ProbeCfg{tun.max_retries, tun.probe};
    return q;
  }
  // captured iterations, one executable graph per launch configuration
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec[24] = {};
  const MlpTiles* graph_tiles[24] = {};
  // learned skipping: attached predictor and options, per-vertex records
  lpa_predictor pred = nullptr;
  lpa_learned_options lopt{};
  unsigned long long* lrec = nullptr;
  bool lrec_valid = false;
  int learn_grid = 1;
  int32_t learned_iters = 0;   // iterations of the last learned run
  bool acct_feat = false;      // profile: the run keeps records ...
  int acct_feat_cmin = 1;      // ... for the classes acct_feat_cmin ..
  int acct_feat_cmax = 8;      // acct_feat_cmax

  BatchArgs batch_args() const {
    BatchArgs b;
    b.G = G; b.v_off = b_voff; b.done = b_done; b.iters = b_iters; b.changed_last = b_changed;
    return b;
  }

  lpa_status ensure_history(int32_t cap) {
    if (cap <= hist_cap && hist) return LPA_OK;
    DevIterStats* h = nullptr;
    if (lpa_status e = dalloc(&h, std::max(cap, 32))) return e;
    hist = h;  // the old buffer stays in dev_allocs until destroy
    hist_cap = std::max(cap, 32);
    return LPA_OK;
  }

  lpa_status iteration_graph(const lpa_options& o, const RunCtx& rc, hipGraphExec_t* out);

  HubArgs hub_args(int async_mode) const {
    HubArgs a;
    a.off = off; a.tgt = tgt; a.w = w; a.C = C; a.F = F; a.chg = chg;
    a.uoff = uoff; a.utgt = utgt; a.uw = uw; a.inv = inv; a.ctgt = ctgt;
    a.pend_v = pend_v; a.pend_c = pend_c; a.st = st;
    a.hub_vid = hub_vid; a.hub_tab = hub_tab; a.hub_best = hub_best; a.hub_old = hub_old;
    a.hub_nch = hub_nch; a.hub_ovf = hub_ovf; a.hub_lgb = hub_lgb;
    a.hub_slice0 = hub_slice0; a.hub_boff0 = hub_boff0;
    a.gkeys = gkeys; a.gvals = gvals; a.items = items; a.bitems = bitems;
    a.part_keys = part_keys; a.part_vals = part_vals; a.boff = boff;
    a.bsize = bsize; a.hub_bq = hub_bq;
    a.H = H; a.chunk = tun.hub_chunk; a.async_mode = async_mode;
    a.probe = ProbeCfg{tun.max_retries, tun.probe};
    a.xcd_map = tun.xcd_local & 1;
    a.witems = witems;
    a.wctr = wctr;
    for (int x = 0; x <= kXcds; ++x) a.wbase[x] = wbase[x];
    uint32_t cap = 16383u;
    if (tun.hub_table_cap > 0) {
      cap = 1u;
      while (2u * cap + 1u <= (uint32_t)std::min(tun.hub_table_cap, 16383)) cap = 2u * cap + 1u;
    }
    a.table_cap = cap;
    return a;
  }

  ~lpa_graph_s() {
    for (hipGraphExec_t x : graph_exec)
      if (x) (void)hipGraphExecDestroy(x);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : dev_allocs) (void)hipFree(p);
    if (st_host) (void)hipHostFree(st_host);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

extern "C" {

void lpa_options_default(lpa_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->mode = LPA_MODE_ASYNC;
  opt->max_iterations = 20;
  opt->tolerance = 0.05;
  opt->pl_period = 4;
  opt->prune = 1;
  opt->initial_labels = nullptr;
  opt->profile = 0;
  opt->flag_mode = LPA_FLAGS_AUTO;
  opt->launch = LPA_LAUNCH_EAGER;
}

void lpa_tuning_default(lpa_tuning* t) {
  if (!t) return;
  std::memset(t, 0, sizeof(*t));
  t->small4 = 4;
  t->small16 = 16;
  t->wave = 512;
  t->block = 8192;
  t->hub_chunk = 8192;
  t->max_retries = 32;
  t->xcd_local = 3;
  t->relabel = -1;
  t->batch_queue = -1;
  t->queue_chunk = 512;
  t->queue_group = 64;
  t->sort_rows = -1;
  t->block_threads = 0;
  t->table_load = 2;
  t->pull_divisor = 16;
}

void lpa_learned_options_default(lpa_learned_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->threshold = 0.1f;
  o->fn_bound = 0.02f;
  o->guard_period = 4;
  o->first_predicted = 2;
}

const char* lpa_status_string(lpa_status s) {
  switch (s) {
    case LPA_OK: return "ok";
    case LPA_ERR_INVALID: return "invalid argument";
    case LPA_ERR_OOM: return "out of memory";
    case LPA_ERR_HIP: return "HIP runtime error";
    case LPA_ERR_STATE: return "invalid state";
    case LPA_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* lpa_last_error(void) { return g_err.c_str(); }

// Hub slices grouped by target window, one group per XCD: a slice of a
// row sorted by target covers a contiguous range of ids, placed here by its
// middle entry's position in the id order weighted by entries (rows are
// read as often as their vertex's degree, so equal-weight windows spread
// the label reads evenly).  The slices are sorted by that position and cut
// into kXcds runs of equal entry counts; k_hub_part takes run x on XCD x
// first, so that each XCD's L2 holds the labels of its own window.
static lpa_status group_hub_slices(lpa_graph G, const std::vector<int64_t>& hd, int64_t items,
                                   hipStream_t s) {
  const int chunk = G->tun.hub_chunk;
  std::vector<uint32_t> sl(2 * (size_t)items);
  std::vector<int64_t> len((size_t)items);
  int64_t k = 0;
  for (int32_t h = 0; h < G->H; ++h)
    for (int64_t c = 0, nch = (hd[h] + chunk - 1) / chunk; c < nch; ++c, ++k) {
      sl[2 * k] = (uint32_t)h;
      sl[2 * k + 1] = (uint32_t)c;
      len[k] = std::min<int64_t>(chunk, hd[h] - c * chunk);
    }
  uint32_t* dsl = nullptr;
  int64_t* dkey = nullptr;
  if (lpa_status e = G->dalloc(&dsl, 2 * items)) return e;
  if (lpa_status e = G->dalloc(&dkey, items)) return e;
  LPA_HIP(hipMemcpyAsync(dsl, sl.data(), sizeof(uint32_t) * sl.size(), hipMemcpyHostToDevice, s));
  LPA_HIP(launch_slice_keys(G->off64, G->off, G->tgt, G->hub_vid, dsl, items, chunk, dkey, s));
  std::vector<int64_t> key((size_t)items);
  LPA_HIP(hipMemcpyAsync(key.data(), dkey, sizeof(int64_t) * items, hipMemcpyDeviceToHost, s));
  LPA_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> order((size_t)items);
  for (int64_t i = 0; i < items; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  int64_t total = 0;
  for (int64_t i = 0; i < items; ++i) total += len[i];
  std::vector<uint32_t> out(2 * (size_t)items);
  int64_t acc = 0;
  int x = 0;
  G->wbase[0] = 0;
  for (int64_t i = 0; i < items; ++i) {
    // group x holds the slices whose entries start below (x + 1) / kXcds
    // of the total
    while (x + 1 < kXcds && acc >= total * (x + 1) / kXcds) G->wbase[++x] = (uint32_t)i;
    out[2 * i] = sl[2 * order[i]];
    out[2 * i + 1] = sl[2 * order[i] + 1];
    acc += len[order[i]];
  }
  while (x + 1 <= kXcds) G->wbase[++x] = (uint32_t)items;
  // the slice list is reused for the grouped order
  LPA_HIP(hipMemcpyAsync(dsl, out.data(), sizeof(uint32_t) * out.size(), hipMemcpyHostToDevice, s));
  if (lpa_status e = G->dalloc(&G->wctr, kXcds * kQueueCtrStride)) return e;
  LPA_HIP(launch_fill_u32(G->wctr, 0u, kXcds * kQueueCtrStride, s));
  LPA_HIP(hipStreamSynchronize(s));
  G->witems = dsl;
  return LPA_OK;
}

static lpa_status create_impl(const lpa_csr* g, void* stream, const lpa_tuning* tuning,
                              lpa_graph_s* G) {
  G->stream = (hipStream_t)stream;
  G->n = g->num_vertices;
  G->m = g->num_edges;
  G->off64 = g->offset_type == LPA_INDEX_I64;
  if (tuning) G->tun = *tuning; else lpa_tuning_default(&G->tun);
  const lpa_tuning& t = G->tun;
  if (!(0 <= t.small4 && t.small4 <= 4 && t.small4 <= t.small16 && t.small16 <= 16 &&
        t.small16 <= t.wave && t.wave <= 512 && t.wave <= t.block && t.block <= 8192 &&
        t.hub_chunk >= 64 && t.hub_chunk <= 8192 && t.max_retries >= 0 &&
        t.hub_table_cap >= 0 && t.relabel >= -1 && t.relabel <= 1 && t.probe >= 0 &&
        t.probe <= 3 &&
        (t.table_values == 0 || t.table_values == 32 || t.table_values == 64) &&
        t.batch_queue >= -1 && t.batch_queue <= 1 &&
        (t.queue_chunk == 0 ||
         (t.queue_chunk >= 64 && t.queue_chunk <= (1 << kQueueMaxChunkLog2) &&
          (t.queue_chunk & (t.queue_chunk - 1)) == 0)) &&
        (t.queue_group == 0 || (t.queue_group >= 16 && t.queue_group <= 64)) &&
        t.sort_rows >= -1 && t.sort_rows <= 1 &&
        (t.block_threads == 0 || t.block_threads == 256 || t.block_threads == 512 ||
         t.block_threads == 1024) &&
        (t.table_load == 1 || t.table_load == 2 || t.table_load == 4) &&
        t.memory_limit_kib >= 0 && t.xcd_local >= 0 && t.xcd_local <= 3 &&
        t.pull_divisor >= 1 && t.pull_divisor <= 4096))
    return fail(LPA_ERR_INVALID, "tuning thresholds out of range");
  // the ablation kernels' largest LDS table has 8191 slots (rows of <= 4096)
  if (t.table_values != 0) G->tun.block = std::min(G->tun.block, 4096);
  hipStream_t s = G->stream;
  const int64_t n = G->n, m = G->m;

  // graph arrays: borrow device pointers or copy host arrays in
  const size_t osz = G->off64 ? sizeof(int64_t) : sizeof(int32_t);
  if (g->on_device) {
    if ((n >= 0 && !is_device_ptr(g->offsets)) || (m > 0 && !is_device_ptr(g->targets)) ||
        (g->weights && !is_device_ptr(g->weights)))
      return fail(LPA_ERR_INVALID, "on_device = 1 but an array is not device memory");
    G->off = g->offsets;
    G->tgt = g->targets;
    G->w = g->weights;
  } else {
    void* doff = nullptr;
    int32_t* dtgt = nullptr;
    float* dw = nullptr;
    if (G->off64) {
      int64_t* p; if (lpa_status e = G->dalloc(&p, n + 1)) return e; doff = p;
    } else {
      int32_t* p; if (lpa_status e = G->dalloc(&p, n + 1)) return e; doff = p;
    }
    if (lpa_status e = G->dalloc(&dtgt, m)) return e;
    LPA_HIP(hipMemcpyAsync(doff, g->offsets, osz * (size_t)(n + 1), hipMemcpyHostToDevice, s));
    if (m > 0)
      LPA_HIP(hipMemcpyAsync(dtgt, g->targets, sizeof(int32_t) * (size_t)m,
                             hipMemcpyHostToDevice, s));
    if (g->weights) {
      if (lpa_status e = G->dalloc(&dw, m)) return e;
      if (m > 0)
        LPA_HIP(hipMemcpyAsync(dw, g->weights, sizeof(float) * (size_t)m,
                               hipMemcpyHostToDevice, s));
    }
    G->off = doff;
    G->tgt = dtgt;
    G->w = dw;
  }
  G->uoff = G->off;
  G->utgt = G->tgt;
  G->uw = G->w;

  // counters
  if (lpa_status e = G->dalloc(&G->st, 1)) return e;
  {
    void* h = nullptr;
    LPA_HIP(hipHostMalloc(&h, sizeof(DevStats), hipHostMallocDefault));
    G->st_host = static_cast<DevStats*>(h);
  }
  LPA_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(G->st), 0u,
                          sizeof(DevStats) / sizeof(uint32_t), s));
  if (g->validate) {
    LPA_HIP(launch_validate(G->off64, G->off, G->tgt, G->w, n, m, G->st, s));
    LPA_HIP(hipMemcpyAsync(G->st_host, G->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
    LPA_HIP(hipStreamSynchronize(s));
    const unsigned err = G->st_host->error;
    if (err) {
      std::string why;
      if (err & 1u) why += " offsets are not 0..M non-decreasing;";
      if (err & 2u) why += " a target is outside [0, N);";
      if (err & 8u) why += " a weight is negative, -0, infinite or NaN;";
      return fail(LPA_ERR_INVALID, "malformed CSR:" + why);
    }
  }
  // weights that are all 1.0f are the unit weights of a NULL array: the
  // kernels then read none (the sums, hence every result, are the same)
  if (G->w && m > 0) {
    unsigned int* other = nullptr;
    if (hipMalloc(&other, sizeof(unsigned)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LPA_ERR_OOM, "hipMalloc failed for the weight check");
    }
    unsigned int h = 1u;
    hipError_t e = launch_unit_weights(G->w, m, other, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, other, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(other);
    if (e != hipSuccess)
      return fail(LPA_ERR_HIP, std::string("weight check: ") + hipGetErrorString(e));
    if (h == 0u) {
      G->w = nullptr;
      G->uw = nullptr;
    }
  }

  // rows with strictly increasing targets: in the first sweep from identity
  // labels every neighbour then carries its own label once, so the row's
  // Eq. 3 maximum is the largest (weight, smallest id) entry -- no table
  if (m > 1) {
    uint8_t* mark = nullptr;
    unsigned int* bad = nullptr;
    if (hipMalloc(&mark, (size_t)m) != hipSuccess || hipMalloc(&bad, sizeof(unsigned)) != hipSuccess) {
      (void)hipGetLastError();
      if (mark) (void)hipFree(mark);
      return fail(LPA_ERR_OOM, "hipMalloc failed for the row check");
    }
    unsigned int hb = 1u;
    hipError_t e = launch_rows_strict(G->off64, G->off, G->tgt, n, m, mark, bad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(mark);
    (void)hipFree(bad);
    if (e != hipSuccess) return fail(LPA_ERR_HIP, std::string("row check: ") + hipGetErrorString(e));
    G->strict_rows = hb == 0u;
  } else {
    G->strict_rows = true;
  }

  // internal vertex order by degree (relabel.hip).  Automatic: when the
  // labels outgrow one XCD's L2 (N > 2^20) and fewer than half of the
  // sampled entries point within 2^16 ids of their row, i.e. the caller's
  // order gives the label reads no locality of its own.
  bool relabel = t.relabel == 1;
  if (t.relabel < 0 && n > (int64_t)1 << 20) {
    unsigned long long* acc = nullptr;
    if (hipMalloc(&acc, 4 * sizeof(unsigned long long)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LPA_ERR_OOM, "hipMalloc failed for the locality sample");
    }
    unsigned long long h[4] = {0, 0, 0, 0};
    hipError_t e = relabel_locality(G->off64, G->off, G->tgt, n, acc, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(acc);
    if (e != hipSuccess)
      return fail(LPA_ERR_HIP, std::string("locality sample: ") + hipGetErrorString(e));
    relabel = 2 * h[0] < h[1];
  }
  if (relabel && n > 0) {
    if (lpa_status e = G->dalloc(&G->perm, n)) return e;
    if (lpa_status e = G->dalloc(&G->inv, n)) return e;
    void* noff = nullptr;
    if (G->off64) {
      int64_t* p; if (lpa_status e = G->dalloc(&p, n + 1)) return e; noff = p;
    } else {
      int32_t* p; if (lpa_status e = G->dalloc(&p, n + 1)) return e; noff = p;
    }
    int32_t* ntgt = nullptr;
    float* nw = nullptr;
    if (lpa_status e = G->dalloc(&ntgt, m)) return e;
    if (G->uw) {
      if (lpa_status e = G->dalloc(&nw, m)) return e;
    }
    const hipError_t e = relabel_build(G->off64, G->uoff, G->utgt, G->uw, n, G->perm, G->inv,
                                       noff, ntgt, nw, s);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return fail(LPA_ERR_OOM, "hipMalloc failed while building the internal order");
    }
    if (e != hipSuccess)
      return fail(LPA_ERR_HIP, std::string("internal order: ") + hipGetErrorString(e));
    if (t.sort_rows != 0 && m <= (int64_t)INT32_MAX) {
      const hipError_t se = sort_rows(G->off64, noff, ntgt, nw, n, m, s);
      if (se == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return fail(LPA_ERR_OOM, "hipMalloc failed while sorting the internal rows");
      }
      if (se != hipSuccess)
        return fail(LPA_ERR_HIP, std::string("row sort: ") + hipGetErrorString(se));
    }
    G->off = noff;
    G->tgt = ntgt;
    G->w = nw;
    // the internal rows once more with the caller's ids as targets: the
    // first sweep of a run, whose labels are the caller's ids, streams them
    // instead of reading the caller's rows in a scattered order
    if (lpa_status e = G->dalloc(&G->ctgt, m)) return e;
    if (m > 0) LPA_HIP(launch_unpermute_i32(G->inv, ntgt, m, G->ctgt, s));
  }

  // labels, flags, deterministic-mode queue
  if (lpa_status e = G->dalloc(&G->C, n)) return e;
  if (lpa_status e = G->dalloc(&G->F, n)) return e;
  if (lpa_status e = G->dalloc(&G->pend_v, n)) return e;
  if (lpa_status e = G->dalloc(&G->pend_c, n)) return e;
  if (lpa_status e = G->dalloc(&G->Cn, n)) return e;
  if (lpa_status e = G->dalloc(&G->chg, n)) return e;
  if (lpa_status e = G->dalloc(&G->chg_bits, (n + 31) / 32)) return e;
  if (lpa_status e = G->dalloc(&G->cls, n)) return e;

  // degree classes
  int32_t bounds[kNumClasses] = {0};
  // a table of 2^s - 1 slots holds rows of up to 2^(s-1) entries at load <= 1/2
  bounds[1] = t.small4;
  bounds[2] = t.small16;
  bounds[3] = std::min(64, t.wave);     // 127 slots
  bounds[4] = t.wave;                   // 1023 slots
  bounds[5] = std::min(1024, t.block);  // 2047 slots
  bounds[6] = std::min(2048, t.block);  // 4095 slots
  bounds[7] = std::min(4096, t.block);  // 8191 slots
  bounds[8] = t.block;                  // 16383 slots
  bounds[9] = INT32_MAX;
  unsigned long long* counts = nullptr;
  unsigned int* hub_count = nullptr;
  int32_t* hub_tmp = nullptr;
  const int64_t hub_cap = m / ((int64_t)t.block + 1) + 1;
  if (lpa_status e = G->dalloc(&counts, kNumClasses + 2)) return e;
  hub_count = reinterpret_cast<unsigned int*>(counts + kNumClasses);
  if (lpa_status e = G->dalloc(&hub_tmp, hub_cap)) return e;
  LPA_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(counts), 0u, 2 * (kNumClasses + 2), s));
  if (n > 0)
    LPA_HIP(launch_classify(G->off64, G->off, n, bounds, G->cls, counts, hub_tmp, hub_count, s));
  unsigned long long hcounts[kNumClasses + 2];
  LPA_HIP(hipMemcpyAsync(hcounts, counts, sizeof(hcounts), hipMemcpyDeviceToHost, s));
  LPA_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < kNumClasses; ++c) G->cls_count[c] = (int64_t)hcounts[c];
  G->n_active = G->perm ? n - G->cls_count[0] : n;
  G->H = (int32_t)(uint32_t)hcounts[kNumClasses];
  for (int c = 1; c < kNumClasses; ++c) {
    if (c == kClassHub) continue;
    if (lpa_status e = G->dalloc(&G->lists[c], G->cls_count[c])) return e;
    const int64_t per = sweep_items_per_block(c);
    const int64_t need = (G->cls_count[c] + per - 1) / per;
    G->grid[c] = (int)std::max<int64_t>(1, std::min<int64_t>(need, sweep_max_resident(c)));
    const int64_t dper = sweep_direct_items_per_block(c);
    G->direct_grid[c] =
        (int)std::max<int64_t>(1, std::min<int64_t>((G->cls_count[c] + dper - 1) / dper, 256 * 8));
    if (t.table_values != 0 && c <= 7) {
      const int64_t tper = tv_items_per_block(c);
      G->tv_grid[c] = (int)std::max<int64_t>(
          1, std::min<int64_t>((G->cls_count[c] + tper - 1) / tper,
                               tv_max_resident(c, t.table_values)));
    }
  }
  G->frontier_grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 8191) / 8192, 256 * 8));
  G->learn_grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, 2048));
  G->apply_grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 256 * 8));
  G->pull_grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 31) / 32, 256 * 8));
  G->push_grid = 256 * 8;

  // hubs: sorted ids, global table offsets (p1 = nextPow2(D) - 1 slots each),
  // slice scratch
  if (G->H > 0) {
    std::vector<int32_t> hv(G->H);
    std::vector<int64_t> hd(G->H);
    LPA_HIP(hipMemcpyAsync(hv.data(), hub_tmp, sizeof(int32_t) * G->H, hipMemcpyDeviceToHost, s));
    LPA_HIP(hipStreamSynchronize(s));
    std::sort(hv.begin(), hv.end());
    if (lpa_status e = G->dalloc(&G->hub_vid, G->H)) return e;
    LPA_HIP(hipMemcpyAsync(G->hub_vid, hv.data(), sizeof(int32_t) * G->H, hipMemcpyHostToDevice, s));
    int64_t* ddeg = nullptr;
    if (lpa_status e = G->dalloc(&ddeg, G->H)) return e;
    LPA_HIP(launch_gather_degrees(G->off64, G->off, G->hub_vid, G->H, ddeg, s));
    LPA_HIP(hipMemcpyAsync(hd.data(), ddeg, sizeof(int64_t) * G->H, hipMemcpyDeviceToHost, s));
    LPA_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> tab(G->H), slice0(G->H), boff0(G->H);
    std::vector<int32_t> lgb(G->H);
    int64_t slots = 0, items = 0, bitems = 0, boffs = 0;
    for (int32_t h = 0; h < G->H; ++h) {
      if (hd[h] > (int64_t)INT32_MAX / 2)
        return fail(LPA_ERR_INVALID, "a vertex degree exceeds 2^30");
      int64_t p = 1;
      while (p < 2 * hd[h]) p <<= 1;  // spill table: smallest 2^m >= 2D, minus one
      tab[h] = slots;
      slots += p - 1;
      const int64_t nch = (hd[h] + t.hub_chunk - 1) / t.hub_chunk;
      lgb[h] = hub_bucket_log2(hd[h], t.hub_chunk);
      slice0[h] = items;
      boff0[h] = boffs;
      items += nch;
      bitems += (int64_t)1 << lgb[h];
      boffs += nch * (((int64_t)1 << lgb[h]) + 1);
    }
    G->max_items = items;
    G->max_bitems = bitems;
    auto up64 = [&](int64_t** dst, const std::vector<int64_t>& v) -> lpa_status {
      if (lpa_status e = G->dalloc(dst, G->H)) return e;
      LPA_HIP(hipMemcpyAsync(*dst, v.data(), sizeof(int64_t) * G->H, hipMemcpyHostToDevice, s));
      return LPA_OK;
    };
    if (lpa_status e = up64(&G->hub_tab, tab)) return e;
    if (lpa_status e = up64(&G->hub_slice0, slice0)) return e;
    if (lpa_status e = up64(&G->hub_boff0, boff0)) return e;
    if (lpa_status e = G->dalloc(&G->hub_lgb, G->H)) return e;
    LPA_HIP(hipMemcpyAsync(G->hub_lgb, lgb.data(), sizeof(int32_t) * G->H, hipMemcpyHostToDevice, s));
    if (lpa_status e = G->dalloc(&G->hub_nch, G->H)) return e;
    if (lpa_status e = G->dalloc(&G->hub_ovf, G->H)) return e;
    if (lpa_status e = G->dalloc(&G->hub_best, G->H)) return e;
    if (lpa_status e = G->dalloc(&G->hub_old, G->H)) return e;
    if (lpa_status e = G->dalloc(&G->gkeys, slots)) return e;
    if (lpa_status e = G->dalloc(&G->gvals, slots)) return e;
    LPA_HIP(launch_fill_u32(G->gkeys, kEmpty, slots, s));
    LPA_HIP(launch_fill_f32(G->gvals, 0.0f, slots, s));
    if (t.table_values == 64) {
      double* gv = nullptr;
      if (lpa_status e = G->dalloc(&gv, slots)) return e;
      LPA_HIP(launch_fill_f64(gv, 0.0, slots, s));
      G->tv_gvals = gv;
    } else if (t.table_values == 32) {
      G->tv_gvals = G->gvals;
    }
    if (t.table_values != 0) {
      if (lpa_status e = G->dalloc(&G->tv_vmax, G->H)) return e;
      if (lpa_status e = G->dalloc(&G->tv_nl, G->H)) return e;
      LPA_HIP(launch_fill_u64(G->tv_vmax, 0ull, G->H, s));
      LPA_HIP(launch_fill_u32(G->tv_nl, 0u, G->H, s));
    }
    if (lpa_status e = G->dalloc(&G->items, 2 * items)) return e;
    if (lpa_status e = G->dalloc(&G->bitems, 2 * bitems)) return e;
    if (lpa_status e = G->dalloc(&G->part_keys, items * (int64_t)t.hub_chunk)) return e;
    if (lpa_status e = G->dalloc(&G->part_vals, items * (int64_t)t.hub_chunk)) return e;
    if (lpa_status e = G->dalloc(&G->boff, boffs)) return e;
    if (lpa_status e = G->dalloc(&G->bsize, bitems)) return e;
    if (lpa_status e = G->dalloc(&G->hub_bq, G->H)) return e;
    // one resident workgroup per CU for the two LDS-table kernels (a
    // multiple of the 8 XCDs for the bucket mapping)
    G->hub_acc_grid = (int)std::max<int64_t>(1, std::min<int64_t>(items, hub_max_resident()));
    G->hub_reduce_grid = hub_max_resident();
    G->hub_fin_grid = (int)std::max<int64_t>(1, std::min<int64_t>(items, 256 * 8));
    G->hub_direct_grid = G->hub_fin_grid;
    LPA_HIP(hipStreamSynchronize(s));
    if ((t.xcd_local & 2) && G->strict_rows && items > 0)
      if (lpa_status e = group_hub_slices(G, hd, items, s)) return e;
  }
  LPA_HIP(hipEventCreate(&G->ev0));
  LPA_HIP(hipEventCreate(&G->ev1));
  LPA_HIP(hipStreamSynchronize(s));
  return LPA_OK;
}

lpa_status lpa_create(const lpa_csr* g, void* stream, const lpa_tuning* tuning,
                      lpa_graph* out) {
  if (!out) return fail(LPA_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!g) return fail(LPA_ERR_INVALID, "graph is NULL");
  if (g->num_vertices < 0 || g->num_vertices > (int64_t)INT32_MAX)
    return fail(LPA_ERR_INVALID, "num_vertices must lie in [0, 2^31 - 1]");
  if (g->num_edges < 0) return fail(LPA_ERR_INVALID, "num_edges < 0");
  if (g->offset_type != LPA_INDEX_I32 && g->offset_type != LPA_INDEX_I64)
    return fail(LPA_ERR_INVALID, "offset_type must be LPA_INDEX_I32 or LPA_INDEX_I64");
  if (g->offset_type == LPA_INDEX_I32 && g->num_edges > (int64_t)INT32_MAX)
    return fail(LPA_ERR_INVALID, "int32 offsets cannot address more than 2^31 - 1 edges");
  if (!g->offsets || (g->num_edges > 0 && !g->targets))
    return fail(LPA_ERR_INVALID, "offsets or targets is NULL");
  lpa_graph_s* G = new (std::nothrow) lpa_graph_s();
  if (!G) return fail(LPA_ERR_OOM, "host allocation failed");
  const lpa_status st = create_impl(g, stream, tuning, G);
  if (st != LPA_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    delete G;
    return st;
  }
  *out = G;
  g_err.clear();
  return LPA_OK;
}

void lpa_destroy(lpa_graph g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  delete g;
}

lpa_status lpa_graph_classes(lpa_graph g, int64_t* counts) {
  if (!g || !counts) return fail(LPA_ERR_INVALID, "NULL argument");
  counts[0] = g->cls_count[0];
  counts[1] = g->cls_count[1];
  counts[2] = g->cls_count[2];
  counts[3] = g->cls_count[3] + g->cls_count[4];
  counts[4] = g->cls_count[5] + g->cls_count[6] + g->cls_count[7] + g->cls_count[8];
  counts[5] = g->cls_count[kClassHub];
  return LPA_OK;
}

// Copy n int32 labels from host or device memory into dst (device).
static lpa_status stage_labels(lpa_graph g, const int32_t* src, int32_t* dst) {
  const hipMemcpyKind kind = is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  LPA_HIP(hipMemcpyAsync(dst, src, sizeof(int32_t) * (size_t)g->n, kind, g->stream));
  return LPA_OK;
}

}  // extern "C"

// Enqueue one iteration of Algorithm 1 on stream s.  Every kernel reads the
// iteration's Pick-Less flag and the stop flag from device memory, so the
// sequence can be replayed without the host (eagerly or as a captured graph).
// mark(kid) brackets launches for the optional per-kernel profile.
// Learned-variant context of a run: records kept (feat), predictor tiles
// (NULL: no predictions) and trace buffers (X NULL: no trace).
struct RunCtx {
  bool feat = false;
  bool infer = true;  // feat: the frontier may run the network (else the
                      // plain frontier, which lists the same vertices)
  int feat_cmin = 1;  // classes outside feat_cmin .. feat_cmax run the plain
  int feat_cmax = 8;  // kernels (no records)
  const MlpTiles* tiles = nullptr;
  TraceArgs tr{};
};

// direct: the first sweep of a run from identity labels over rows with
// strictly increasing targets, which takes the table-free kernels.  cc: a
// Cross-Check iteration (eager launches only: its revert rounds are repeated
// from the host until they settle).
template <typename Mark>
static lpa_status enqueue_iteration(lpa_graph g, const lpa_options& o, const RunCtx& rc,
                                    hipStream_t s, Mark&& mark, bool direct = false,
                                    bool cc = false) {
  const int64_t n = g->n;
  const int async_mode = o.mode == LPA_MODE_ASYNC;
  if (g->wq && o.prune) {
    // batched run as a work queue: counters, sweep, per-graph step
    const QueueArgs q = g->queue_args(async_mode);
    if (lpa_status e = mark(-1)) return e;
    LPA_HIP(launch_queue_iter_begin(q, s));
    if (lpa_status e = mark(kKidQueueSweep)) return e;
    LPA_HIP(launch_queue_sweep(g->off64, q, g->wq_grid, s));
    if (lpa_status e = mark(kKidQueueStep)) return e;
    LPA_HIP(launch_queue_step(q, s));
    if (lpa_status e = mark(-1)) return e;
    LPA_HIP(launch_iter_end(g->st, g->hist, n, s));
    return LPA_OK;
  }
  const int tv = g->tun.table_values;  // 0, or the ablation kernels' value bits
  if (cc) LPA_HIP(launch_cc_save(g->C, g->cc_prev, n, s));
  // without pruning every vertex is processed in every iteration
  if (!o.prune) LPA_HIP(launch_arm_flags(g->F, n, g->st, s));
  const HubArgs ha = g->hub_args(async_mode);
  if (lpa_status e = mark(kKidPlan)) return e;
  LPA_HIP(launch_hub_plan(g->off64, ha, g->C, g->F, s));
  if (lpa_status e = mark(kKidFrontier)) return e;
  // after the first iteration only the vertices of positive degree can be
  // flagged (without pruning every vertex is, every iteration)
  const int64_t n_later = o.prune ? g->n_active : n;
  if (rc.feat && rc.infer)
    LPA_HIP(launch_frontier_learned(n, n_later, g->F, g->cls, g->lists, g->chg, g->st, g->lrec, rc.tiles,
                                    rc.tr, g->learn_grid, s));
  else
    LPA_HIP(launch_frontier(n, n_later, g->F, g->cls, g->lists, g->chg, g->st, g->frontier_grid, s));
  if (g->H > 0 && direct) {
    if (lpa_status e = mark(kKidHubDirect)) return e;
    LPA_HIP(launch_hub_direct(g->off64, ha, g->hub_direct_grid, s));
  } else if (g->H > 0 && tv) {
    if (lpa_status e = mark(kKidHubPart)) return e;
    LPA_HIP(launch_tv_hub_acc(g->off64, tv, ha, g->tv_gvals, g->hub_fin_grid, s));
    if (lpa_status e = mark(kKidHubReduce)) return e;
    LPA_HIP(launch_tv_hub_select(g->off64, tv, ha, g->tv_gvals, g->tv_vmax, g->tv_nl,
                                 g->hub_fin_grid, s));
  } else if (g->H > 0) {
    if (lpa_status e = mark(kKidHubPart)) return e;
    LPA_HIP(launch_hub_part(g->off64, ha, g->hub_acc_grid, s));
    if (lpa_status e = mark(kKidHubReduce)) return e;
    LPA_HIP(launch_hub_reduce(g->off64, ha, g->hub_reduce_grid, s));
    if (lpa_status e = mark(kKidHubSpill)) return e;
    LPA_HIP(launch_hub_spill(g->off64, ha, g->hub_fin_grid, s));
  }
  SweepArgs a;
  a.off = g->off; a.tgt = g->tgt; a.w = g->w; a.C = g->C; a.Cn = g->Cn; a.F = g->F;
  a.chg = g->chg; a.st = g->st;
  a.uoff = g->uoff; a.utgt = g->utgt; a.uw = g->uw; a.inv = g->inv; a.ctgt = g->ctgt;
  a.async_mode = async_mode;
  a.probe = ProbeCfg{g->tun.max_retries, g->tun.probe};
  a.rec = g->lrec;
  a.tload = g->tun.table_load;
  a.block_threads = g->tun.block_threads;
  for (int c = kClassHub - 1; c >= 1; --c) {
    if (g->cls_count[c] == 0) continue;
    a.cls = c;
    a.active = g->lists[c];
    if (lpa_status e = mark((direct ? kKidDirect0 : kKidSweep0) + c)) return e;
    if (direct)
      LPA_HIP(launch_sweep_direct(g->off64, c, a, g->direct_grid[c],
                                  rc.feat && c >= rc.feat_cmin && c <= rc.feat_cmax, s));
    else if (tv)
      LPA_HIP(launch_sweep_tv(g->off64, c, tv, a, g->tv_grid[c], s));
    else
      LPA_HIP(launch_sweep(g->off64, c, a, g->grid[c],
                           rc.feat && c >= rc.feat_cmin && c <= rc.feat_cmax, s));
  }
  if (g->H > 0) {
    if (lpa_status e = mark(kKidHubFin)) return e;
    LPA_HIP(launch_hub_fin(g->off64, ha, g->hub_fin_grid, s));
  }
  if (!async_mode) {
    if (lpa_status e = mark(kKidApply)) return e;
    LPA_HIP(launch_apply(g->st, g->lists, g->Cn, g->pend_v, g->pend_c, g->C, g->apply_grid, s));
  }
  if (cc) {
    // Cross-Check: rounds until no revert decision changes (the decisions
    // depend only on smaller ids, so at most one round per chain step)
    if (lpa_status e = mark(-1)) return e;
    for (int64_t round = 0;; ++round) {
      if (round > n + 1) return fail(LPA_ERR_HIP, "Cross-Check rounds did not settle");
      LPA_HIP(launch_cc_round(g->C, g->cc_prev, g->chg, g->cc_rev, g->perm, g->inv, n, g->st,
                              s));
      LPA_HIP(hipMemcpyAsync(&g->st_host->cc_moved, &g->st->cc_moved, sizeof(unsigned int),
                             hipMemcpyDeviceToHost, s));
      LPA_HIP(hipStreamSynchronize(s));
      if (!g->st_host->cc_moved) break;
    }
    LPA_HIP(launch_cc_apply(g->C, g->cc_prev, g->chg, g->cc_rev, n, g->st, s));
  }
  // flag the neighbours of the changed vertices: the decide kernel picks
  // push or pull from this iteration's counters, the other kernels return
  if (lpa_status e = mark(kKidDecide)) return e;
  LPA_HIP(launch_flag_decide(g->st, g->m, g->n, o.flag_mode, g->tun.pull_divisor, s));
  if (lpa_status e = mark(kKidPush)) return e;
  LPA_HIP(launch_push_lists(g->off64, g->off, g->tgt, g->lists, g->chg, g->F, g->st,
                            g->push_grid, s));
  if (g->H > 0) {
    if (lpa_status e = mark(kKidPushHubs)) return e;
    LPA_HIP(launch_push_hubs(g->off64, ha, g->hub_fin_grid, s));
  }
  if (lpa_status e = mark(kKidPull)) return e;
  LPA_HIP(launch_pull_flags(g->off64, g->off, g->tgt, g->n_active, g->cls, g->chg, g->chg_bits, g->F, g->st,
                            g->pull_grid, s));
  if (g->H > 0) {
    if (lpa_status e = mark(kKidPullHubs)) return e;
    LPA_HIP(launch_pull_hubs(g->off64, g->off, g->tgt, g->hub_vid, g->H, g->chg_bits, g->F,
                             g->st, s));
  }
  if (g->G > 0) {
    if (lpa_status e = mark(kKidBatch)) return e;
    LPA_HIP(launch_batch_step(g->batch_args(), g->chg, g->F, g->st, s));
  }
  if (rc.tr.X) {
    if (lpa_status e = mark(-1)) return e;
    LPA_HIP(launch_trace_label(g->st, g->chg, rc.tr, s));
  }
  if (lpa_status e = mark(-1)) return e;
  LPA_HIP(launch_iter_end(g->st, g->hist, n, s));
  return LPA_OK;
}

lpa_status lpa_graph_s::iteration_graph(const lpa_options& o, const RunCtx& rc,
                                        hipGraphExec_t* out) {
  // a captured learned iteration holds the predictor's tile address: rebuild
  // it when another predictor is attached
  const int key = (o.mode == LPA_MODE_ASYNC ? 6 : 0) + (o.prune ? 3 : 0) + o.flag_mode +
                  (rc.feat ? 12 : 0);
  if (graph_exec[key] && graph_tiles[key] != rc.tiles) {
    (void)hipGraphExecDestroy(graph_exec[key]);
    graph_exec[key] = nullptr;
  }
  graph_tiles[key] = rc.tiles;
  if (graph_exec[key]) {
    *out = graph_exec[key];
    return LPA_OK;
  }
  if (!cap_stream) LPA_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  LPA_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
  auto nomark = [](int) -> lpa_status { return LPA_OK; };
  const lpa_status st = enqueue_iteration(this, o, rc, cap_stream, nomark);
  hipGraph_t graph = nullptr;
  const hipError_t end = hipStreamEndCapture(cap_stream, &graph);
  if (st != LPA_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (end != hipSuccess) return fail(LPA_ERR_HIP, "hipStreamEndCapture failed");
  hipGraphExec_t exec = nullptr;
  const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (inst != hipSuccess) return fail(LPA_ERR_HIP, "hipGraphInstantiate failed");
  graph_exec[key] = exec;
  *out = exec;
  return LPA_OK;
}

// Trace request of lpa_trace (device buffers).
struct TraceReq {
  TraceArgs tr;
  double rate;
  uint64_t seed;
  int64_t cap;
};

static lpa_status run_impl(lpa_graph g, const lpa_options* opt, int32_t* labels,
                           lpa_iter_stats* stats, int32_t stats_cap, int32_t* iters_done,
                           const TraceReq* trace = nullptr) {
  if (!g) return fail(LPA_ERR_INVALID, "graph is NULL");
  lpa_options o;
  if (opt) o = *opt; else lpa_options_default(&o);
  if (o.mode != LPA_MODE_DETERMINISTIC && o.mode != LPA_MODE_ASYNC)
    return fail(LPA_ERR_INVALID, "mode must be LPA_MODE_DETERMINISTIC or LPA_MODE_ASYNC");
  if (o.max_iterations < 0) return fail(LPA_ERR_INVALID, "max_iterations < 0");
  if (o.pl_period < 0) return fail(LPA_ERR_INVALID, "pl_period < 0");
  if (o.flag_mode < LPA_FLAGS_AUTO || o.flag_mode > LPA_FLAGS_PULL)
    return fail(LPA_ERR_INVALID, "flag_mode must be LPA_FLAGS_AUTO, _PUSH or _PULL");
  if (o.launch != LPA_LAUNCH_EAGER && o.launch != LPA_LAUNCH_GRAPH)
    return fail(LPA_ERR_INVALID, "launch must be LPA_LAUNCH_EAGER or LPA_LAUNCH_GRAPH");
  if (stats_cap < 0 || (stats_cap > 0 && !stats))
    return fail(LPA_ERR_INVALID, "stats_cap < 0 or stats is NULL");
  if (g->n > 0 && !labels) return fail(LPA_ERR_INVALID, "labels is NULL");
  if (o.learned != 0 && o.learned != 1) return fail(LPA_ERR_INVALID, "learned must be 0 or 1");
  if (o.learned && !g->pred)
    return fail(LPA_ERR_STATE, "learned run without a predictor (lpa_set_predictor)");
  if (o.cc_period < 0) return fail(LPA_ERR_INVALID, "cc_period < 0");
  if (o.cc_period > 0 && (o.launch != LPA_LAUNCH_EAGER || o.learned || trace || g->G > 0))
    return fail(LPA_ERR_UNSUPPORTED,
                "Cross-Check needs a single-graph, eager, plain run (cc_period > 0)");
  if ((o.learned || trace) && g->G > 0)
    return fail(LPA_ERR_UNSUPPORTED, "learned skipping and traces need a single graph");
  if ((o.learned || trace) && g->tun.table_values != 0)
    return fail(LPA_ERR_UNSUPPORTED,
                "learned skipping and traces use the fp32 class kernels (table_values 0)");
  if (iters_done) *iters_done = 0;
  const int64_t n = g->n;
  if (n == 0) return LPA_OK;
  g->flags_pending = false;
  if (o.cc_period > 0 && !g->cc_prev) {
    if (lpa_status e = g->dalloc(&g->cc_prev, n)) return e;
    if (lpa_status e = g->dalloc(&g->cc_rev, n)) return e;
    LPA_HIP(launch_fill_u8(g->cc_rev, 0, n, g->stream));
  }
  hipStream_t s = g->stream;
  if (lpa_status e = g->ensure_history(o.max_iterations)) return e;

  RunCtx rc;
  LearnParams lp{};
  rc.feat = o.learned || trace;
  if (rc.feat) {
    if (!g->lrec) {
      if (lpa_status e = g->dalloc(&g->lrec, n)) return e;
    }
    LPA_HIP(launch_fill_u64(g->lrec, kRecordInit, n, s));
    g->lrec_valid = true;
  }
  if (o.learned) {
    rc.tiles = predictor_tiles(g->pred);
    if (!rc.tiles) return fail(LPA_ERR_HIP, "packing the predictor's parameters failed");
    const double th = g->lopt.threshold;
    lp.learn = 1;
    lp.guard = g->lopt.guard_period;
    lp.z_theta = (float)std::log(th / (1.0 - th));
    lp.fn_bound = g->lopt.fn_bound;
  }
  rc.tr.inv = g->inv;
  rc.tr.perm = g->perm;
  if (trace) {
    rc.tr = trace->tr;
    rc.tr.inv = g->inv;
    rc.tr.perm = g->perm;
    lp.trace = 1;
    lp.trace_rate = trace->rate;
    lp.trace_seed = trace->seed;
    lp.trace_cap = (unsigned long long)trace->cap;
  }
  // rows of the register classes (at most small16 entries) are predicted,
  // recorded and traced only with predict_small, those of the workgroup
  // classes (wave+1 .. block entries) only with predict_large
  rc.feat_cmin = g->lopt.predict_small ? 1 : 3;
  rc.feat_cmax = g->lopt.predict_large ? kClassHub - 1 : 4;
  lp.cmin = rc.feat_cmin;
  lp.cmax = rc.feat_cmax;
  // the iterations before the one ahead of the first prediction keep no
  // records: plain kernels (a handle without a predictor: the defaults)
  lp.pstart = g->lopt.first_predicted >= 1 ? g->lopt.first_predicted : 2;
  const int32_t feat_from = rc.feat ? lp.pstart - 1 : 0;
  RunCtx rc_plain = rc;
  rc_plain.feat = false;
  rc_plain.tiles = nullptr;
  rc_plain.tr.X = nullptr;
  // the iteration ahead of the first prediction writes records but neither
  // predicts nor traces (both start at pstart): the plain frontier
  RunCtx rc_rec = rc;
  rc_rec.infer = false;
  const int32_t infer_from = rc.feat ? lp.pstart : 0;
  auto ctx_of = [&](int32_t l) -> const RunCtx& {
    return l < feat_from ? rc_plain : (l < infer_from ? rc_rec : rc);
  };
  g->acct_feat = rc.feat;
  g->acct_feat_cmin = rc.feat_cmin;
  g->acct_feat_cmax = rc.feat_cmax;
  LPA_HIP(launch_run_begin(g->st, o.tolerance, o.max_iterations, o.pl_period, g->G > 0,
                           g->G, lp, s));
  if (g->G > 0) LPA_HIP(launch_batch_reset(g->batch_args(), s));
  const int32_t* init = nullptr;
  if (o.initial_labels) {
    if (lpa_status e = stage_labels(g, o.initial_labels, g->pend_v)) return e;
    init = g->pend_v;
  }
  LPA_HIP(launch_init(n, init, g->inv, g->C, g->F, g->st, s));
  if (init) {
    LPA_HIP(hipMemcpyAsync(g->st_host, g->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
    LPA_HIP(hipStreamSynchronize(s));
    if (g->st_host->error & 4u)
      return fail(LPA_ERR_INVALID, "initial_labels must lie in [0, N)");
  }

  const bool use_queue = g->wq && o.prune;
  if (use_queue) {
    const QueueArgs q = g->queue_args(o.mode == LPA_MODE_ASYNC);
    LPA_HIP(launch_queue_begin(q, n, s));
    if (g->wq_nchunks > 0)
      LPA_HIP(hipMemcpyAsync(g->wq_items, g->wq_items0, sizeof(uint32_t) * g->wq_nchunks,
                             hipMemcpyDeviceToDevice, s));
    LPA_HIP(hipMemcpyAsync(g->wq_qctr, g->wq_qctr0,
                           sizeof(unsigned int) * 2 * kXcds * 2 * kQueueCtrStride,
                           hipMemcpyDeviceToDevice, s));
  }
  // a run from identity labels over strict rows: table-free first sweep
  const bool first_direct =
      !use_queue && !init && g->strict_rows && g->tun.table_values == 0;
  int32_t done = 0;
  const bool graph_mode = o.launch == LPA_LAUNCH_GRAPH && !o.profile && !trace;
  if (graph_mode) {
    // capture one iteration on the private stream, replay it max_iterations
    // times on the handle's stream; the kernels of iterations after the stop
    // return at once
    hipGraphExec_t exec = nullptr;
    if (lpa_status e = g->iteration_graph(o, rc, &exec)) return e;
    // iterations enqueued one by one: the table-free first sweep, and the
    // iterations before the first prediction (no records, or records
    // without the network)
    int32_t l0 = std::min(o.max_iterations, std::max<int32_t>(first_direct ? 1 : 0, infer_from));
    for (int32_t l = 0; l < l0; ++l) {
      auto nomark = [](int) -> lpa_status { return LPA_OK; };
      if (lpa_status e = enqueue_iteration(g, o, ctx_of(l), s, nomark,
                                           first_direct && l == 0))
        return e;
    }
    for (int32_t l = l0; l < o.max_iterations; ++l) LPA_HIP(hipGraphLaunch(exec, s));
    LPA_HIP(hipMemcpyAsync(g->st_host, g->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
    LPA_HIP(hipStreamSynchronize(s));
    done = g->st_host->iter;
    const int32_t k = std::min(done, stats_cap);
    if (k > 0) {
      std::vector<DevIterStats> h(k);
      LPA_HIP(hipMemcpyAsync(h.data(), g->hist, sizeof(DevIterStats) * k,
                             hipMemcpyDeviceToHost, s));
      LPA_HIP(hipStreamSynchronize(s));
      for (int32_t l = 0; l < k; ++l) {
        std::memset(&stats[l], 0, sizeof(stats[l]));
        stats[l].iteration = h[l].iteration;
        stats[l].pick_less = h[l].pick_less;
        stats[l].changed = h[l].changed;
        stats[l].processed = h[l].processed;
        stats[l].edges_scanned = h[l].edges;
        stats[l].skipped = (int32_t)h[l].skipped;
      }
    }
  } else {
    const bool prof = o.profile != 0;
    for (int32_t l = 0; l < o.max_iterations; ++l) {
      int nev = 0;
      auto mark = [&](int kid) -> lpa_status {
        if (!prof) return LPA_OK;
        if (lpa_status e = g->ensure_events(nev + 1)) return e;
        g->ev_kid[nev] = kid;
        LPA_HIP(hipEventRecord(g->ev_pool[nev], s));
        ++nev;
        return LPA_OK;
      };
      LPA_HIP(hipEventRecord(g->ev0, s));
      const bool cc_it = o.cc_period > 0 && l % o.cc_period == 0;
      if (lpa_status e = enqueue_iteration(g, o, ctx_of(l), s, mark,
                                           first_direct && l == 0, cc_it))
        return e;
      LPA_HIP(hipEventRecord(g->ev1, s));
      LPA_HIP(hipMemcpyAsync(g->st_host, g->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
      LPA_HIP(hipStreamSynchronize(s));
      float ms = 0.0f;
      LPA_HIP(hipEventElapsedTime(&ms, g->ev0, g->ev1));
      const DevStats& h = *g->st_host;
      unsigned long long changed = 0, edges = 0;
      for (int c = 0; c < kNumClasses; ++c) {
        changed += h.changed[c];
        edges += h.edges[c];
      }
      changed -= h.reverted;  // Cross-Check reverts
      if (prof) {
        for (int q = 0; q + 1 < nev; ++q) {
          float kms = 0.0f;
          LPA_HIP(hipEventElapsedTime(&kms, g->ev_pool[q], g->ev_pool[q + 1]));
          g->account(g->ev_kid[q], kms, h, o.mode == LPA_MODE_ASYNC, (int)h.pull_mode);
        }
      }
      if (l < stats_cap) {
        lpa_iter_stats& r = stats[l];
        std::memset(&r, 0, sizeof(r));
        r.iteration = l;
        r.pick_less = h.pl;
        r.changed = (int64_t)changed;
        r.processed = (int64_t)h.processed;
        r.edges_scanned = (int64_t)edges;
        r.ms = ms;
        r.skipped = (int32_t)h.skipped;
      }
      done = l + 1;
      if (h.stop) break;
    }
  }
  if (use_queue) {
    LPA_HIP(launch_queue_finish(g->queue_args(o.mode == LPA_MODE_ASYNC), s));
    if (g->st_host->error & 32u)
      return fail(LPA_ERR_INVALID,
                  "a row is longer than the work queue takes (the CSR changed after create)");
  }
  if (iters_done) *iters_done = done;
  g->flags_pending = g->st_host->flags_deferred != 0;
  g->learned_iters = o.learned ? done : 0;
  const bool dev_out = is_device_ptr(labels);
  if (g->perm) {
    // labels in the caller's order (Cn is free once the run has ended)
    int32_t* dst = dev_out ? labels : g->Cn;
    LPA_HIP(launch_unpermute_i32(g->C, g->perm, n, dst, s));
    if (!dev_out)
      LPA_HIP(hipMemcpyAsync(labels, dst, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  } else {
    const hipMemcpyKind kind = dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    LPA_HIP(hipMemcpyAsync(labels, g->C, sizeof(int32_t) * (size_t)n, kind, s));
  }
  LPA_HIP(hipStreamSynchronize(s));
  return LPA_OK;
}

extern "C" {

lpa_status lpa_run(lpa_graph g, const lpa_options* opt, int32_t* labels,
                   lpa_iter_stats* stats, int32_t stats_cap, int32_t* iters_done) {
  return run_impl(g, opt, labels, stats, stats_cap, iters_done);
}

lpa_status lpa_run_batched(lpa_graph g, const lpa_options* opt, int32_t* labels,
                           int32_t* iters_per_graph, int64_t* changed_last_per_graph,
                           int32_t* iters_done) {
  if (!g) return fail(LPA_ERR_INVALID, "graph is NULL");
  if (g->G <= 0) return fail(LPA_ERR_STATE, "handle was not made by lpa_create_batched");
  if (lpa_status e = run_impl(g, opt, labels, nullptr, 0, iters_done)) return e;
  if (g->n == 0) return LPA_OK;
  if (iters_per_graph)
    LPA_HIP(hipMemcpyAsync(iters_per_graph, g->b_iters, sizeof(int32_t) * g->G,
                           hipMemcpyDeviceToHost, g->stream));
  if (changed_last_per_graph)
    LPA_HIP(hipMemcpyAsync(changed_last_per_graph, g->b_changed, sizeof(int64_t) * g->G,
                           hipMemcpyDeviceToHost, g->stream));
  LPA_HIP(hipStreamSynchronize(g->stream));
  return LPA_OK;
}

// Work-queue structures of a batched handle (queue.hip): chunks of
// 2^chunk_log2 vertices per graph, the graphs' first chunks, each chunk's
// graph, and the initial queue -- every chunk of every non-empty graph in
// one part per XCD (graph g in part g mod 8) -- with its counters.  With
// batch_queue = -1 a row longer than the queue kernel takes leaves the
// handle on the class kernels.
static lpa_status build_queue(lpa_graph g, const int64_t* v_off, const lpa_tuning& t) {
  hipStream_t s = g->stream;
  unsigned long long* dmax = nullptr;
  if (lpa_status e = g->dalloc(&dmax, 1)) return e;
  unsigned long long hmax = 0;
  LPA_HIP(launch_fill_u64(dmax, 0ull, 1, s));
  LPA_HIP(launch_max_degree(g->off64, g->off, g->n, dmax, s));
  LPA_HIP(hipMemcpyAsync(&hmax, dmax, sizeof(hmax), hipMemcpyDeviceToHost, s));
  LPA_HIP(hipStreamSynchronize(s));
  if (hmax > (unsigned long long)kQueueMaxDegree) {
    if (t.batch_queue == 1)
      return fail(LPA_ERR_UNSUPPORTED, "batch_queue = 1 takes rows of at most 512 entries; "
                                       "the longest has " + std::to_string(hmax));
    return LPA_OK;
  }
  const int chunk = t.queue_chunk ? t.queue_chunk : 512;
  int lg = 0;
  while ((1 << lg) < chunk) ++lg;
  g->wq_chunk_log2 = lg;
  g->wq_group = t.queue_group ? t.queue_group : 64;
  const int32_t G = g->G;
  std::vector<int64_t> cbase(G + 1, 0);
  for (int32_t q = 0; q < G; ++q)
    cbase[q + 1] = cbase[q] + (((v_off[q + 1] - v_off[q]) + (1 << lg) - 1) >> lg);
  const int64_t nch = cbase[G];
  if (nch >= (int64_t)UINT32_MAX) return fail(LPA_ERR_INVALID, "too many queue items");
  std::vector<int32_t> cgraph((size_t)std::max<int64_t>(nch, 1));
  std::vector<int64_t> qbase(kXcds + 1, 0);
  for (int32_t q = 0; q < G; ++q) {
    for (int64_t c = cbase[q]; c < cbase[q + 1]; ++c) cgraph[(size_t)c] = q;
    qbase[(q & (kXcds - 1)) + 1] += cbase[q + 1] - cbase[q];
  }
  for (int x = 0; x < kXcds; ++x) qbase[x + 1] += qbase[x];
  std::vector<uint32_t> items0((size_t)std::max<int64_t>(nch, 1));
  std::vector<int64_t> fill(qbase.begin(), qbase.end() - 1);
  for (int32_t q = 0; q < G; ++q)
    for (int64_t c = cbase[q]; c < cbase[q + 1]; ++c)
      items0[(size_t)fill[q & (kXcds - 1)]++] = (uint32_t)c;
  const int nctr = 2 * kXcds * 2 * kQueueCtrStride;
  std::vector<unsigned int> ctr0(nctr, 0u);
  for (int x = 0; x < kXcds; ++x)  // iteration 0: head 0, tail = the part's size
    ctr0[(size_t)(x * 2 + 1) * kQueueCtrStride] = (unsigned int)(qbase[x + 1] - qbase[x]);
  g->wq_nchunks = nch;
  if (lpa_status e = g->dalloc(&g->wq_cbase, G + 1)) return e;
  if (lpa_status e = g->dalloc(&g->wq_cgraph, nch)) return e;
  if (lpa_status e = g->dalloc(&g->wq_items, 2 * nch)) return e;
  if (lpa_status e = g->dalloc(&g->wq_items0, nch)) return e;
  if (lpa_status e = g->dalloc(&g->wq_qbase, kXcds + 1)) return e;
  if (lpa_status e = g->dalloc(&g->wq_qctr, nctr)) return e;
  if (lpa_status e = g->dalloc(&g->wq_qctr0, nctr)) return e;
  if (lpa_status e = g->dalloc(&g->wq_cmark, nch)) return e;
  if (lpa_status e = g->dalloc(&g->wq_F1, g->n)) return e;
  if (lpa_status e = g->dalloc(&g->wq_gchanged, G)) return e;
  LPA_HIP(hipMemcpyAsync(g->wq_cbase, cbase.data(), sizeof(int64_t) * (G + 1),
                         hipMemcpyHostToDevice, s));
  if (nch > 0) {
    LPA_HIP(hipMemcpyAsync(g->wq_cgraph, cgraph.data(), sizeof(int32_t) * nch,
                           hipMemcpyHostToDevice, s));
    LPA_HIP(hipMemcpyAsync(g->wq_items0, items0.data(), sizeof(uint32_t) * nch,
                           hipMemcpyHostToDevice, s));
  }
  LPA_HIP(hipMemcpyAsync(g->wq_qbase, qbase.data(), sizeof(int64_t) * (kXcds + 1),
                         hipMemcpyHostToDevice, s));
  LPA_HIP(hipMemcpyAsync(g->wq_qctr0, ctr0.data(), sizeof(unsigned int) * nctr,
                         hipMemcpyHostToDevice, s));
  LPA_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  g->wq_grid = queue_sweep_resident();
  g->wq = true;
  return LPA_OK;
}

lpa_status lpa_create_batched(int32_t num_graphs, const int64_t* v_off, const lpa_csr* csr,
                              void* stream, const lpa_tuning* tuning, lpa_graph* out) {
  if (!out) return fail(LPA_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (num_graphs <= 0 || !v_off || !csr)
    return fail(LPA_ERR_INVALID, "num_graphs must be positive; v_off and csr non-NULL");
  if (v_off[0] != 0 || v_off[num_graphs] != csr->num_vertices)
    return fail(LPA_ERR_INVALID, "v_off must run from 0 to num_vertices");
  for (int32_t q = 0; q < num_graphs; ++q)
    if (v_off[q + 1] < v_off[q]) return fail(LPA_ERR_INVALID, "v_off must be non-decreasing");
  // the packed graphs keep the caller's order (their stop test works on
  // ranges of vertex ids)
  lpa_tuning tb;
  if (tuning) tb = *tuning; else lpa_tuning_default(&tb);
  if (tb.relabel == 1)
    return fail(LPA_ERR_UNSUPPORTED, "relabel = 1 needs a single graph (lpa_create)");
  if (tb.table_values != 0)
    return fail(LPA_ERR_UNSUPPORTED, "table_values 32 / 64 need a single graph (lpa_create)");
  tb.relabel = 0;
  lpa_graph g = nullptr;
  if (lpa_status e = lpa_create(csr, stream, &tb, &g)) return e;
  hipStream_t s = g->stream;
  auto cleanup = [&](lpa_status e) { lpa_destroy(g); return e; };
  g->G = num_graphs;
  int64_t* dv = nullptr;
  if (lpa_status e = g->dalloc(&dv, num_graphs + 1)) return cleanup(e);
  g->b_voff = dv;
  if (lpa_status e = g->dalloc(&g->b_done, num_graphs)) return cleanup(e);
  if (lpa_status e = g->dalloc(&g->b_iters, num_graphs)) return cleanup(e);
  if (lpa_status e = g->dalloc(&g->b_changed, num_graphs)) return cleanup(e);
  if (hipMemcpyAsync(dv, v_off, sizeof(int64_t) * (num_graphs + 1), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return cleanup(fail(LPA_ERR_HIP, "copying v_off failed"));
  if (csr->validate) {
    if (launch_fill_u32(reinterpret_cast<uint32_t*>(g->st), 0u,
                        sizeof(DevStats) / sizeof(uint32_t), s) != hipSuccess ||
        launch_batch_validate(g->off64, g->off, g->tgt, g->batch_args(), g->n, g->st, s) !=
            hipSuccess ||
        hipMemcpyAsync(g->st_host, g->st, sizeof(DevStats), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return cleanup(fail(LPA_ERR_HIP, "batched validation failed to run"));
    if (g->st_host->error & 16u)
      return cleanup(fail(LPA_ERR_INVALID, "a CSR entry points outside its own graph"));
  }
  if (tb.batch_queue != 0) {
    if (lpa_status e = build_queue(g, v_off, tb)) return cleanup(e);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return cleanup(fail(LPA_ERR_HIP, "sync failed"));
  *out = g;
  return LPA_OK;
}

lpa_status lpa_profile(lpa_graph g, lpa_kernel_profile* out, int32_t cap, int32_t* count) {
  if (!g || (cap > 0 && !out) || cap < 0) return fail(LPA_ERR_INVALID, "bad argument");
  int32_t k = 0;
  for (int q = 0; q < kNumKids; ++q) {
    if (g->prof[q].launches == 0) continue;
    if (k < cap) {
      out[k] = g->prof[q];
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", kKidNames[q]);
    }
    ++k;
  }
  if (count) *count = k;
  return LPA_OK;
}

lpa_status lpa_profile_reset(lpa_graph g) {
  if (!g) return fail(LPA_ERR_INVALID, "graph is NULL");
  for (int q = 0; q < kNumKids; ++q) g->prof[q] = lpa_kernel_profile{};
  return LPA_OK;
}

lpa_status lpa_set_predictor(lpa_graph g, lpa_predictor p, const lpa_learned_options* lo) {
  if (!g) return fail(LPA_ERR_INVALID, "graph is NULL");
  if (g->G > 0) return fail(LPA_ERR_UNSUPPORTED, "learned skipping needs a single graph");
  lpa_learned_options o;
  if (lo) o = *lo; else lpa_learned_options_default(&o);
  if (!(o.threshold > 0.0f && o.threshold < 1.0f))
    return fail(LPA_ERR_INVALID, "threshold must lie in (0, 1)");
  if (!(o.fn_bound >= 0.0f)) return fail(LPA_ERR_INVALID, "fn_bound must be >= 0");
  if (o.guard_period < 0) return fail(LPA_ERR_INVALID, "guard_period must be >= 0");
  if ((o.predict_small != 0 && o.predict_small != 1) ||
      (o.predict_large != 0 && o.predict_large != 1))
    return fail(LPA_ERR_INVALID, "predict_small and predict_large must be 0 or 1");
  if (o.first_predicted < 1) return fail(LPA_ERR_INVALID, "first_predicted must be >= 1");
  g->pred = p;
  g->lopt = o;
  return LPA_OK;
}

lpa_status lpa_learned_history(lpa_graph g, lpa_learned_iter* out, int32_t cap,
                               int32_t* count) {
  if (!g || !count || cap < 0 || (cap > 0 && !out))
    return fail(LPA_ERR_INVALID, "bad argument");
  *count = 0;
  const int32_t k = std::min(g->learned_iters, cap);
  if (k <= 0) return LPA_OK;
  std::vector<DevIterStats> h(k);
  LPA_HIP(hipMemcpyAsync(h.data(), g->hist, sizeof(DevIterStats) * k, hipMemcpyDeviceToHost,
                         g->stream));
  LPA_HIP(hipStreamSynchronize(g->stream));
  for (int32_t l = 0; l < k; ++l) {
    std::memset(&out[l], 0, sizeof(out[l]));
    out[l].iteration = h[l].iteration;
    out[l].skipping = h[l].skipping;
    out[l].fallback = h[l].fallback;
    out[l].skipped = h[l].skipped;
    out[l].predicted = h[l].npred;
    out[l].false_negatives = h[l].fneg;
  }
  *count = k;
  return LPA_OK;
}

lpa_status lpa_get_records(lpa_graph g, uint64_t* out) {
  if (!g || (g->n > 0 && !out)) return fail(LPA_ERR_INVALID, "NULL argument");
  if (g->n == 0) return LPA_OK;
  if (!g->lrec_valid) return fail(LPA_ERR_STATE, "no learned or traced run yet");
  const bool dev_out = is_device_ptr(out);
  const unsigned long long* src = g->lrec;
  if (g->perm) {
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(out);
    if (!dev_out) {
      if (!g->stage64) {
        if (lpa_status e = g->dalloc(&g->stage64, g->n)) return e;
      }
      dst = g->stage64;
    }
    LPA_HIP(launch_unpermute_u64(g->lrec, g->perm, g->n, dst, g->stream));
    src = dst;
  }
  if (src != reinterpret_cast<const unsigned long long*>(out)) {
    const hipMemcpyKind kind = dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    LPA_HIP(hipMemcpyAsync(out, src, sizeof(uint64_t) * (size_t)g->n, kind, g->stream));
  }
  LPA_HIP(hipStreamSynchronize(g->stream));
  return LPA_OK;
}

lpa_status lpa_trace(lpa_graph g, const lpa_options* opt, double sample_rate, uint64_t seed,
                     float* X, float* y, int32_t* vertex, int32_t* iteration, int64_t cap,
                     int64_t* count) {
  if (!g || !count) return fail(LPA_ERR_INVALID, "NULL argument");
  if (cap < 0 || (cap > 0 && (!X || !y))) return fail(LPA_ERR_INVALID, "bad trace buffers");
  if (!(sample_rate >= 0.0 && sample_rate <= 1.0))
    return fail(LPA_ERR_INVALID, "sample_rate must lie in [0, 1]");
  *count = 0;
  if (g->n == 0) return LPA_OK;
  hipStream_t s = g->stream;
  // device buffers: the caller's when they are device memory, else staging
  std::vector<void*> staged;
  struct Free {
    std::vector<void*>* v;
    ~Free() { for (void* q : *v) (void)hipFree(q); }
  } guard{&staged};
  auto dev = [&](void* user, size_t bytes, void** out) -> lpa_status {
    if (user && is_device_ptr(user)) { *out = user; return LPA_OK; }
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(bytes, 4)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LPA_ERR_OOM, "hipMalloc failed for trace staging");
    }
    staged.push_back(q);
    *out = q;
    return LPA_OK;
  };
  const size_t c = (size_t)cap;
  void *dX, *dy, *dv, *dl;
  if (lpa_status e = dev(X, sizeof(float) * 12 * c, &dX)) return e;
  if (lpa_status e = dev(y, sizeof(float) * c, &dy)) return e;
  if (lpa_status e = dev(vertex, sizeof(int32_t) * c, &dv)) return e;
  if (lpa_status e = dev(iteration, sizeof(int32_t) * c, &dl)) return e;
  TraceReq req;
  req.tr.X = static_cast<float*>(dX);
  req.tr.y = static_cast<float*>(dy);
  req.tr.v = static_cast<int32_t*>(dv);
  req.tr.l = static_cast<int32_t*>(dl);
  req.rate = sample_rate;
  req.seed = seed;
  req.cap = cap;
  std::vector<int32_t> labels((size_t)g->n);
  if (lpa_status e = run_impl(g, opt, labels.data(), nullptr, 0, nullptr, &req)) return e;
  const int64_t drawn = (int64_t)g->st_host->trace_n;
  *count = drawn;
  const size_t kept = (size_t)std::min<int64_t>(drawn, cap);
  auto back = [&](void* user, void* d, size_t bytes) -> lpa_status {
    if (!user || user == d || bytes == 0) return LPA_OK;
    LPA_HIP(hipMemcpyAsync(user, d, bytes, hipMemcpyDeviceToHost, s));
    return LPA_OK;
  };
  if (lpa_status e = back(X, dX, sizeof(float) * 12 * kept)) return e;
  if (lpa_status e = back(y, dy, sizeof(float) * kept)) return e;
  if (lpa_status e = back(vertex, dv, sizeof(int32_t) * kept)) return e;
  if (lpa_status e = back(iteration, dl, sizeof(int32_t) * kept)) return e;
  LPA_HIP(hipStreamSynchronize(s));
  return LPA_OK;
}

lpa_status lpa_get_flags(lpa_graph g, uint8_t* flags) {
  if (!g || (g->n > 0 && !flags)) return fail(LPA_ERR_INVALID, "NULL argument");
  if (g->n == 0) return LPA_OK;
  if (g->flags_pending) {
    // the run skipped flagging after its final iteration: pull those flags
    // from the change bytes it left (the frontier of a next run clears them)
    hipStream_t s = g->stream;
    LPA_HIP(launch_flags_resume(g->st, s));
    LPA_HIP(launch_pull_flags(g->off64, g->off, g->tgt, g->n_active, g->cls, g->chg, g->chg_bits, g->F, g->st,
                              g->pull_grid, s));
    if (g->H > 0)
      LPA_HIP(launch_pull_hubs(g->off64, g->off, g->tgt, g->hub_vid, g->H, g->chg_bits, g->F,
                               g->st, s));
    LPA_HIP(launch_flags_done(g->st, s));
    g->flags_pending = false;
  }
  const bool dev_out = is_device_ptr(flags);
  const uint8_t* src = g->F;
  if (g->perm) {
    uint8_t* dst = flags;
    if (!dev_out) {
      if (!g->stage8) {
        if (lpa_status e = g->dalloc(&g->stage8, g->n)) return e;
      }
      dst = g->stage8;
    }
    LPA_HIP(launch_unpermute_u8(g->F, g->perm, g->n, dst, g->stream));
    src = dst;
  }
  if (src != flags) {
    const hipMemcpyKind kind = dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    LPA_HIP(hipMemcpyAsync(flags, src, (size_t)g->n, kind, g->stream));
  }
  LPA_HIP(hipStreamSynchronize(g->stream));
  return LPA_OK;
}

lpa_status lpa_label_read_rate(lpa_graph g, int32_t reps, double* reads_per_s) {
  if (!g || !reads_per_s) return fail(LPA_ERR_INVALID, "NULL argument");
  if (reps < 1) return fail(LPA_ERR_INVALID, "reps must be at least 1");
  *reads_per_s = 0.0;
  if (g->m == 0 || g->n == 0) return LPA_OK;
  hipStream_t s = g->stream;
  constexpr int kGrid = 256 * 16;
  if (!g->probe_sink) {
    if (lpa_status e = g->dalloc(&g->probe_sink, (int64_t)kGrid * 256)) return e;
  }
  // labels of a plain start, so that the reads see valid ids
  LPA_HIP(launch_init(g->n, nullptr, g->inv, g->C, g->F, g->st, s));
  g->flags_pending = false;
  LPA_HIP(launch_label_read_probe(g->tgt, g->m, g->C, g->probe_sink, kGrid, s));  // warm-up
  LPA_HIP(hipEventRecord(g->ev0, s));
  for (int32_t r = 0; r < reps; ++r)
    LPA_HIP(launch_label_read_probe(g->tgt, g->m, g->C, g->probe_sink, kGrid, s));
  LPA_HIP(hipEventRecord(g->ev1, s));
  LPA_HIP(hipEventSynchronize(g->ev1));
  float ms = 0.0f;
  LPA_HIP(hipEventElapsedTime(&ms, g->ev0, g->ev1));
  *reads_per_s = ms > 0.0f ? (double)g->m * reps / (1e-3 * ms) : 0.0;
  return LPA_OK;
}

// The CSR and labels Eq. 1's edge pass reads.  With an internal order the
// pass goes through the internal CSR (degree order, rows sorted by target,
// where a neighbour-label read costs half as much as in an unordered
// caller's order), with the labels first moved to the internal positions
// (into the deterministic next-label array, free between runs).  The sums
// are the same up to fp64 rounding order.  lab NULL in the result: the move
// failed to launch.
struct ModCsr {
  const void* off;
  const int32_t* tgt;
  const float* w;
  const int32_t* lab;
};
static ModCsr modularity_csr(lpa_graph g, const int32_t* lab) {
  if (!g->perm) return ModCsr{g->uoff, g->utgt, g->uw, lab};
  if (launch_unpermute_i32(lab, g->inv, g->n, g->Cn, g->stream) != hipSuccess)
    return ModCsr{nullptr, nullptr, nullptr, nullptr};
  return ModCsr{g->off, g->tgt, g->w, g->Cn};
}

lpa_status lpa_modularity(lpa_graph g, const int32_t* labels, double* q) {
  if (!g || !q) return fail(LPA_ERR_INVALID, "NULL argument");
  *q = 0.0;
  if (g->n == 0) return LPA_OK;
  if (!labels) return fail(LPA_ERR_INVALID, "labels is NULL");
  hipStream_t s = g->stream;
  if (!g->mod_sig) {
    if (lpa_status e = g->dalloc(&g->mod_sig, g->n)) return e;
    if (lpa_status e = g->dalloc(&g->mod_acc, 4)) return e;
  }
  const int32_t* lab = labels;
  if (!is_device_ptr(labels)) {
    if (lpa_status e = stage_labels(g, labels, g->pend_v)) return e;
    lab = g->pend_v;
  }
  LPA_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(g->st), 0u,
                          sizeof(DevStats) / sizeof(uint32_t), s));
  LPA_HIP(launch_check_labels(g->n, lab, g->st, s));
  LPA_HIP(hipMemcpyAsync(g->st_host, g->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
  LPA_HIP(hipStreamSynchronize(s));
  if (g->st_host->error & 4u) return fail(LPA_ERR_INVALID, "labels must lie in [0, N)");
  const ModCsr mc = modularity_csr(g, lab);
  if (!mc.lab) return fail(LPA_ERR_HIP, "moving the labels to the internal order failed");
  LPA_HIP(launch_modularity(g->off64, mc.off, mc.tgt, mc.w, g->n, g->m, mc.lab, g->mod_sig,
                            g->mod_acc, s));
  double acc[4];
  LPA_HIP(hipMemcpyAsync(acc, g->mod_acc, sizeof(acc), hipMemcpyDeviceToHost, s));
  LPA_HIP(hipStreamSynchronize(s));
  const double two_m = acc[1];
  *q = two_m > 0.0 ? acc[0] / two_m - acc[2] / (two_m * two_m) : 0.0;
  return LPA_OK;
}

// The same result as lpa_modularity with no device allocation: Sigma_c and
// the accumulators in the GPU's file-scope scratch (graph.hip), host labels
// staged through the handle's own buffer, the accumulators read back with
// the handle's pinned counters.
lpa_status lpa_modularity_noalloc(lpa_graph g, const int32_t* labels, double* q) {
  if (!g || !q) return fail(LPA_ERR_INVALID, "NULL argument");
  *q = 0.0;
  if (g->n > kModScratchVertices)
    return fail(LPA_ERR_INVALID, "lpa_modularity_noalloc takes at most " +
                                     std::to_string(kModScratchVertices) +
                                     " vertices (its fixed scratch); use lpa_modularity");
  if (g->n == 0) return LPA_OK;
  if (!labels) return fail(LPA_ERR_INVALID, "labels is NULL");
  hipStream_t s = g->stream;
  double* sig = nullptr;
  double* acc = nullptr;
  LPA_HIP(modularity_scratch(&sig, &acc));
  const int32_t* lab = labels;
  if (!is_device_ptr(labels)) {
    if (lpa_status e = stage_labels(g, labels, g->pend_v)) return e;
    lab = g->pend_v;
  }
  LPA_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(g->st), 0u,
                          sizeof(DevStats) / sizeof(uint32_t), s));
  LPA_HIP(launch_check_labels(g->n, lab, g->st, s));
  const ModCsr mc = modularity_csr(g, lab);
  if (!mc.lab) return fail(LPA_ERR_HIP, "moving the labels to the internal order failed");
  LPA_HIP(launch_modularity(g->off64, mc.off, mc.tgt, mc.w, g->n, g->m, mc.lab, sig, acc, s));
  LPA_HIP(hipMemcpyAsync(g->st->mod_acc, acc, sizeof(double) * 4, hipMemcpyDeviceToDevice, s));
  LPA_HIP(hipMemcpyAsync(g->st_host, g->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
  LPA_HIP(hipStreamSynchronize(s));
  if (g->st_host->error & 4u) return fail(LPA_ERR_INVALID, "labels must lie in [0, N)");
  const double two_m = g->st_host->mod_acc[1];
  *q = two_m > 0.0 ? g->st_host->mod_acc[0] / two_m -
                         g->st_host->mod_acc[2] / (two_m * two_m)
                   : 0.0;
  return LPA_OK;
}

}  // extern "C"
