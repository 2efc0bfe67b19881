// lpa_internal.h -- declarations shared by the host runtime and the kernel
// translation units of the label-propagation library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpa {

// Vertex classes by degree (bounds come from lpa_tuning):
//   0 degree 0 (never processed: no neighbour to adopt a label from)
//   1 4-lane register groups          2 16-lane register groups
//   3 wave, LDS table <= 127 slots    4 wave, LDS table <= 1023 slots
//   5..8 workgroup, LDS table <= 2047 / 4095 / 8191 / 16383 slots
//   9 hub: several workgroups per vertex + global-memory table
constexpr int kNumClasses = 10;
constexpr int kClassHub = 9;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // empty hashtable key
constexpr int kXcds = 8;                  // accelerator complex dies of an MI355X

// Per-iteration device counters.  Reset at the start of every iteration by
// the hub-plan kernel, read back by the host after the iteration.
struct DevStats {
  unsigned long long processed;                 // vertices taken this iteration
  unsigned long long pending;                   // deterministic mode: queued hub label writes
  unsigned long long edges[kNumClasses];        // CSR entries scanned, per class
  unsigned long long changed[kNumClasses];      // label changes, per class
  unsigned long long flagw[kNumClasses];        // sum of degrees of changed vertices
  unsigned long long pull_scanned;              // entries read by the pull-flag kernels
  unsigned int pull_mode;                       // 0: flags of this iteration pushed,
                                                // 1: pulled, 2: deferred (the run
                                                // stops after this iteration)
  unsigned int flags_deferred;                  // the last iteration's flags are
                                                // still to be set from chg
  unsigned int cc_moved;                        // Cross-Check: a round changed a
                                                // revert decision
  unsigned long long reverted;                  // Cross-Check: changes reverted
                                                // in this iteration
  unsigned int active[kNumClasses];             // vertices appended per class
  unsigned long long hub_pairs;                 // (label, sum) pairs the hub slices
                                                // wrote this iteration
  unsigned int hub_items;                       // hub slices queued this iteration
  unsigned int hub_all;                         // every hub is flagged this iteration
  unsigned int hub_bitems;                      // hub label buckets queued this iteration
  // run control, resident on the device so that iterations can be launched
  // back to back (or replayed from a captured graph) without the host
  double tol;                                   // stop tolerance
  int cap;                                      // iteration cap
  int rho;                                      // Pick-Less period (0: off)
  int iter;                                     // index of the iteration being run
  int ident;                                    // the run started from labels = vertex ids
  int stop;                                     // 1: run ended, kernels return at once
  int pl;                                       // Pick-Less in this iteration
  int batched;                                  // per-graph stop rule
  unsigned int graphs_left;                     // batched: graphs still running
  unsigned int error;                           // sticky error bits (validation, labels)
  // learned skipping (a project addition): run parameters ...
  int learn;                                    // 1: predictions are made
  int pred_cmin;                                // predicted classes: pred_cmin ..
  int pred_cmax;                                // pred_cmax
  int pred_start;                               // first predicted iteration
  int guard;                                    // guard period (0: none)
  int trace;                                    // 1: record trace samples
  float z_theta;                                // predicted unchanged: logit < z_theta
  double fn_bound;                              // fallback bound on false negatives
  double trace_rate;                            // sampling rate of the trace
  unsigned long long trace_seed;
  unsigned long long trace_cap;
  // ... and state
  int predict;                                  // this iteration evaluates the predictor
  int skipping;                                 // this iteration skips predicted vertices
  int fallback;                                 // skipping off for the rest of the run
  int cand;                                     // last iteration changed < tol * N
  unsigned long long skipped;                   // flagged vertices left unprocessed
  unsigned long long npred;                     // vertices predicted unchanged
  unsigned long long fneg;                      // of those, processed and changed
  unsigned long long trace_n;                   // samples drawn so far
  unsigned long long trace_first;               // trace_n when the iteration began
  double mod_acc[4];                            // lpa_modularity_noalloc: the
                                                // accumulators, read back with
                                                // the counters
};

// Learned-skipping parameters of a run (zero: plain run).
struct LearnParams {
  int learn;
  int guard;
  int trace;
  int cmin;               // classes cmin .. cmax are predicted, recorded, traced
  int cmax;
  int pstart;             // first iteration with predictions and traces
  float z_theta;
  double fn_bound;
  double trace_rate;
  unsigned long long trace_seed;
  unsigned long long trace_cap;
};

// Per-vertex state record of the learned variant, 8 bytes (byte i = bits
// 8i..8i+7): 0 own-label share, 1 best-second margin, 2 best-own gain (each
// floor(255 x / K)), 3 distinct labels per entry, 4 log-quantised degree,
// 5 log-quantised weighted degree, 6 change history (bit 7: predicted
// unchanged in this plain iteration), 7 iteration of the evaluation (255:
// never).
constexpr unsigned long long kRecordInit = 0xFFull << 56;

// Trace output of a run (device pointers; X may be NULL: no trace).
struct TraceArgs {
  float* X;               // [cap][12] features
  float* y;               // [cap] 1 if the vertex changed label
  int32_t* v;             // [cap] vertex (the caller's id)
  int32_t* l;             // [cap] iteration
  const int32_t* inv;     // internal id -> caller id (NULL: one order)
  const int32_t* perm;    // caller id -> internal id
};

// Hashtable probe sequence (probe_next in lpa_device.h): mode 0..3 and the
// probes made before the linear continuation.
struct ProbeCfg {
  int max_retries;
  int mode;
};

// Everything a sweep kernel needs, passed by value.
struct SweepArgs {
  const void* off;        // int32_t* or int64_t* (kernel template picks)
  const int32_t* tgt;
  const float* w;         // NULL: unit weights
  int32_t* C;             // labels (read; written in place in async mode)
  int32_t* Cn;            // deterministic mode: label after this iteration,
                          // written for every processed vertex
  uint8_t* F;             // flags for the next iteration (set on change)
  uint8_t* chg;           // changed-in-this-iteration byte per vertex
  const int32_t* active;  // active vertex list of this class
  DevStats* st;
  int cls;                // class index (selects st->active[cls])
  int async_mode;         // 1: write labels in place, 0: queue them
  ProbeCfg probe;         // probe sequence and probes before the linear continuation
  unsigned long long* rec;  // learned variant: per-vertex state records
  int tload;              // table capacity rule (lpa_tuning.table_load: 1, 2, 4)
  int block_threads;      // workgroup classes: threads (0: per-class defaults)
  // the caller's CSR and inv (internal id -> caller id; NULL when the two
  // orders agree), read by the table-free first sweep
  const void* uoff;
  const int32_t* utgt;
  // internal rows with the caller's ids as targets (NULL: none); the first
  // sweep streams these instead of the caller's rows
  const int32_t* ctgt = nullptr;
  const float* uw;
  const int32_t* inv;
};

// Hubs (rows longer than the largest LDS table).  Each slice of chunk CSR
// entries is reduced in an LDS table; its distinct (label, partial sum) pairs
// are written out grouped by label bucket (a hash of the label, 2^lgb
// buckets per hub, about chunk entries each).  Each bucket is then reduced in
// LDS by one workgroup, which folds its maximum into the hub's packed best.
// A bucket whose distinct labels overflow the LDS table spills the rest into
// the hub's global-memory table, scanned afterwards.
struct HubArgs {
  const void* off;
  const int32_t* tgt;
  const float* w;
  const void* uoff;                // the caller's CSR and inv, as in SweepArgs
  const int32_t* utgt;
  const int32_t* ctgt = nullptr;   // as in SweepArgs
  const float* uw;
  const int32_t* inv;
  int32_t* C;
  uint8_t* F;
  uint8_t* chg;
  int32_t* pend_v;                 // deterministic mode: queued (hub, label)
  int32_t* pend_c;
  DevStats* st;
  const int32_t* hub_vid;          // H hub vertex ids
  const int64_t* hub_tab;          // H offsets into the overflow table
  unsigned long long* hub_best;    // H packed (weight, ~label) maxima
  int32_t* hub_old;                // H labels at iteration start
  int32_t* hub_nch;                // per hub: slices queued this iteration
  int32_t* hub_ovf;                // per hub: some bucket spilled this iteration
  const int32_t* hub_lgb;          // per hub: log2 of its bucket count
  const int64_t* hub_slice0;       // per hub: index of its first slice
  const int64_t* hub_boff0;        // per hub: start of its bucket offsets
  uint32_t* gkeys;                 // overflow table keys
  float* gvals;                    // overflow table values
  uint32_t* items;                 // queued slices: (hub, slice) word pairs
  uint32_t* bitems;                // queued buckets: (hub, bucket) word pairs
  uint32_t* part_keys;             // per slice: chunk entries, grouped by bucket
  float* part_vals;
  uint32_t* boff;                  // per slice: 2^lgb + 1 bucket offsets
  uint32_t* bsize;                 // per queued bucket: its pairs over all slices
  int32_t* hub_bq;                 // per hub: queue index of its bucket 0
  int32_t H;
  int32_t chunk;                   // edges per slice
  int async_mode;
  ProbeCfg probe;
  int xcd_map;                     // 1: consecutive buckets on one XCD
  uint32_t table_cap;              // largest bucket table (2^m - 1 slots)
  // slices grouped by target window: when every hub is flagged, k_hub_part
  // takes the slices of group x (witems[wbase[x] .. wbase[x+1]), (hub,
  // slice) word pairs) on XCD x first, popped with the counters wctr (one
  // per group, kQueueCtrStride words apart), then the other groups'
  const uint32_t* witems;          // NULL: no grouping
  unsigned int* wctr;
  uint32_t wbase[kXcds + 1];
};

// Statistics of one iteration as recorded on the device (same layout as the
// leading fields of lpa_iter_stats).
struct DevIterStats {
  int32_t iteration;
  int32_t pick_less;
  long long changed;
  long long processed;
  long long edges;
  long long skipped;
  long long npred;
  long long fneg;
  int32_t skipping;
  int32_t fallback;
};

// Per-graph state of a batched run.
struct BatchArgs {
  int32_t G;
  const int64_t* v_off;            // G + 1 vertex offsets
  uint8_t* done;                   // 1 once the graph has stopped
  int32_t* iters;                  // iterations the graph performed
  long long* changed_last;         // changed vertices in its last iteration
};

// Batched runs as a persistent work queue (queue.hip).  Each graph's vertex
// range is cut into chunks of 2^chunk_log2 vertices (the last one shorter);
// an item is a chunk's global index.  Two queues alternate by iteration
// parity; each is split into 8 parts, one per XCD, and all chunks of graph g
// go to part g mod 8 (its labels then stay in one XCD's L2).  The sweep
// kernel's resident workgroups pop items from their own XCD's part, then
// from the others; the step kernel applies each graph's stop test and queues
// the chunks marked for the next iteration.
constexpr int kQueueMaxChunkLog2 = 10;   // chunks of at most 1024 vertices
constexpr int kQueueMaxDegree = 512;     // longest row the queue kernel takes
constexpr int kQueueCtrStride = 16;      // words between two queue counters
struct QueueArgs {
  const void* off;
  const int32_t* tgt;
  const float* w;                  // NULL: unit weights
  int32_t* C0;                     // labels read in even iterations ...
  int32_t* C1;                     // ... and odd ones (the same array in
                                   // asynchronous mode)
  uint8_t* F0;                     // flags of even / odd iterations
  uint8_t* F1;
  uint8_t* cmark;                  // per chunk: visit in the next iteration
  const int64_t* cbase;            // G + 1: each graph's first chunk
  const int32_t* cgraph;           // per chunk: its graph
  uint32_t* items;                 // two queues of nchunks items each
  const int64_t* qbase;            // 9: start of each XCD's part of a queue
  unsigned int* qctr;              // [parity][xcd] head, tail (kQueueCtrStride apart)
  unsigned int* gchanged;          // per graph: labels changed in this iteration
  BatchArgs b;
  DevStats* st;
  int64_t nchunks;
  int32_t chunk_log2;
  int32_t group_max;               // rows of up to this many entries: 16 lanes
  int async_mode;
  int strict_rows;                 // every row's targets strictly increase
  ProbeCfg probe;
};

// ---- launch wrappers (defined in the .hip files) ----------------------------
// C[v'] = initial label of the caller's vertex inv[v'] (its id when init is
// NULL; inv NULL: one order).
hipError_t launch_init(int64_t n, const int32_t* init, const int32_t* inv, int32_t* C,
                       uint8_t* F, DevStats* st, hipStream_t s);
hipError_t launch_run_begin(DevStats* st, double tol, int cap, int rho, int batched,
                            int graphs, const LearnParams& lp, hipStream_t s);
hipError_t launch_arm_flags(uint8_t* F, int64_t n, const DevStats* st, hipStream_t s);
hipError_t launch_iter_end(DevStats* st, DevIterStats* hist, int64_t n, hipStream_t s);
hipError_t launch_batch_step(const BatchArgs& b, const uint8_t* chg, uint8_t* F, DevStats* st,
                             hipStream_t s);
hipError_t launch_batch_reset(const BatchArgs& b, hipStream_t s);
hipError_t launch_batch_validate(bool off64, const void* off, const int32_t* tgt,
                                 const BatchArgs& b, int64_t n, DevStats* st, hipStream_t s);
hipError_t launch_validate(bool off64, const void* off, const int32_t* tgt,
                           const float* w, int64_t n, int64_t m, DevStats* st,
                           hipStream_t s);
hipError_t launch_check_labels(int64_t n, const int32_t* lab, DevStats* st,
                               hipStream_t s);
hipError_t launch_rows_strict(bool off64, const void* off, const int32_t* tgt, int64_t n,
                              int64_t m, uint8_t* mark, unsigned int* bad, hipStream_t s);
hipError_t launch_classify(bool off64, const void* off, int64_t n,
                           const int32_t* bounds, uint8_t* cls,
                           unsigned long long* counts, int32_t* hub_out,
                           unsigned int* hub_count, hipStream_t s);
hipError_t launch_slice_keys(bool off64, const void* off, const int32_t* tgt,
                             const int32_t* hub_vid, const uint32_t* sl, int64_t ns, int chunk,
                             int64_t* key, hipStream_t s);
hipError_t launch_gather_degrees(bool off64, const void* off, const int32_t* vids,
                                 int32_t h, int64_t* deg, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int64_t count, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t count,
                           hipStream_t s);
hipError_t launch_hub_plan(bool off64, const HubArgs& a, int32_t* C, uint8_t* F,
                           hipStream_t s);
// n: vertices scanned in iteration 0; n_later: in the iterations after it
hipError_t launch_frontier(int64_t n, int64_t n_later, uint8_t* F, const uint8_t* cls,
                           int32_t* const* lists_dev, uint8_t* chg_clear, DevStats* st,
                           int grid, hipStream_t s);
struct MlpTiles;
hipError_t launch_frontier_learned(int64_t n, int64_t n_later, uint8_t* F, const uint8_t* cls,
                                   int32_t* const* lists, uint8_t* chg_clear, DevStats* st,
                                   unsigned long long* rec, const MlpTiles* tiles,
                                   const TraceArgs& tr, int grid, hipStream_t s);
hipError_t launch_trace_label(const DevStats* st, const uint8_t* chg, const TraceArgs& tr,
                              hipStream_t s);
hipError_t launch_flag_decide(DevStats* st, int64_t m, int64_t n, int force, int pdiv,
                              hipStream_t s);
// Cross-Check (Sec. 4.1): save the labels before an iteration; one round of
// the id-order revert decisions (st->cc_moved set when one changes; the host
// repeats rounds until none does); apply the reverts.  perm/inv map caller
// ids to internal ids (NULL: one order); R: one byte per vertex, zero
// between iterations.
hipError_t launch_cc_save(const int32_t* C, int32_t* Cp, int64_t n, hipStream_t s);
hipError_t launch_cc_round(const int32_t* C, const int32_t* Cp, const uint8_t* chg, uint8_t* R,
                           const int32_t* perm, const int32_t* inv, int64_t n, DevStats* st,
                           hipStream_t s);
hipError_t launch_cc_apply(int32_t* C, const int32_t* Cp, uint8_t* chg, uint8_t* R, int64_t n,
                           DevStats* st, hipStream_t s);

// Deferred flags of a finished run: re-open the run control for one pull
// pass (resume), close it again (done).
hipError_t launch_flags_resume(DevStats* st, hipStream_t s);
hipError_t launch_flags_done(DevStats* st, hipStream_t s);
// packs chg into chg_bits ((n + 31) / 32 words), then pulls the flags
hipError_t launch_pull_flags(bool off64, const void* off, const int32_t* tgt, int64_t n,
                             const uint8_t* cls, const uint8_t* chg, uint32_t* chg_bits,
                             uint8_t* F, DevStats* st, int grid, hipStream_t s);
hipError_t launch_push_lists(bool off64, const void* off, const int32_t* tgt,
                             int32_t* const* lists, const uint8_t* chg, uint8_t* F,
                             DevStats* st, int grid, hipStream_t s);
hipError_t launch_push_hubs(bool off64, const HubArgs& a, int grid, hipStream_t s);
hipError_t launch_pull_hubs(bool off64, const void* off, const int32_t* tgt,
                            const int32_t* hub_vid, int32_t H, const uint32_t* chg_bits,
                            uint8_t* F, DevStats* st, hipStream_t s);
hipError_t launch_apply(const DevStats* st, int32_t* const* lists, const int32_t* Cn,
                        const int32_t* pv, const int32_t* pc, int32_t* C, int grid,
                        hipStream_t s);
hipError_t launch_sweep(bool off64, int cls, const SweepArgs& a, int grid, bool feat,
                        hipStream_t s);
// The first sweep from identity labels over rows with strictly increasing
// targets: table-free kernels (every neighbour label occurs once per row).
hipError_t launch_sweep_direct(bool off64, int cls, const SweepArgs& a, int grid, bool feat,
                               hipStream_t s);
hipError_t launch_hub_direct(bool off64, const HubArgs& a, int grid, hipStream_t s);
hipError_t launch_hub_part(bool off64, const HubArgs& a, int grid, hipStream_t s);
hipError_t launch_hub_reduce(bool off64, const HubArgs& a, int grid, hipStream_t s);
hipError_t launch_hub_spill(bool off64, const HubArgs& a, int grid, hipStream_t s);
hipError_t launch_hub_fin(bool off64, const HubArgs& a, int grid, hipStream_t s);
// Table-value precision ablation (sweep_tv.hip; lpa_tuning.table_values):
// the class sweeps and the hub tables with bits = 32 or 64 bit values.
// gvals holds the hubs' table values (float or double, at a.hub_tab[h]);
// vmax (u64) and hub_nl (u32) hold H zeros between iterations.
hipError_t launch_sweep_tv(bool off64, int cls, int bits, const SweepArgs& a, int grid,
                           hipStream_t s);
hipError_t launch_tv_hub_acc(bool off64, int bits, const HubArgs& a, void* gvals, int grid,
                             hipStream_t s);
hipError_t launch_tv_hub_select(bool off64, int bits, const HubArgs& a, void* gvals,
                                unsigned long long* vmax, uint32_t* hub_nl, int grid,
                                hipStream_t s);
int tv_items_per_block(int cls);
int tv_max_resident(int cls, int bits);
// Bucket count of a hub of degree d: 2^lgb buckets of about chunk entries.
int hub_bucket_log2(int64_t d, int chunk);
constexpr int kHubMaxBucketLog2 = 12;   // 4096 buckets (LDS histogram of k_hub_part)
// lpa_modularity_noalloc: the device addresses of the current GPU's
// file-scope scratch (kModScratchVertices doubles for Sigma_c, then 4
// accumulators), looked up once per device.
constexpr int64_t kModScratchVertices = (int64_t)1 << 22;
hipError_t modularity_scratch(double** sig, double** acc);
hipError_t launch_modularity(bool off64, const void* off, const int32_t* tgt,
                             const float* w, int64_t n, int64_t m,
                             const int32_t* C, double* sig, double* acc,
                             hipStream_t s);

// Work-queue form of a batched run (queue.hip): queue every chunk of every
// non-empty graph for iteration 0 (counters, marks and the odd flags
// cleared, the odd labels copied in deterministic mode); per iteration the
// counters reset, the sweep, the per-graph stop test and next queue; at the
// end the flags (and deterministic labels) of graphs that stopped after an
// odd number of iterations moved to F0 (C0).
hipError_t launch_queue_begin(const QueueArgs& q, int64_t n, hipStream_t s);
hipError_t launch_queue_iter_begin(const QueueArgs& q, hipStream_t s);
hipError_t launch_queue_sweep(bool off64, const QueueArgs& q, int grid, hipStream_t s);
hipError_t launch_queue_step(const QueueArgs& q, hipStream_t s);
hipError_t launch_queue_finish(const QueueArgs& q, hipStream_t s);
int queue_sweep_resident();
// *dmax = the largest row length (atomic max; *dmax zeroed by the caller).
hipError_t launch_max_degree(bool off64, const void* off, int64_t n, unsigned long long* dmax,
                             hipStream_t s);

// Threads per workgroup of each sweep class and resident-workgroup estimate.
int sweep_block_threads(int cls);
int sweep_items_per_block(int cls);
int sweep_direct_items_per_block(int cls);
int sweep_max_resident(int cls);
int hub_block_threads();
int hub_max_resident();

// *other = 1 if any of the m weights differs from 1.0f, else 0.
hipError_t launch_unit_weights(const float* w, int64_t m, unsigned int* other, hipStream_t s);

// One pass reading every entry's target and neighbour label (sink: grid*256).
hipError_t launch_label_read_probe(const int32_t* tgt, int64_t m, const int32_t* C,
                                   uint32_t* sink, int grid, hipStream_t s);

// Internal vertex order (relabel.hip).
hipError_t relabel_build(bool off64, const void* uoff, const int32_t* utgt, const float* uw,
                         int64_t n, int32_t* perm, int32_t* inv, void* noff, int32_t* ntgt,
                         float* nw, hipStream_t s);
// Sort every row of a CSR by target id, weights (may be NULL) alongside
// (rowsort.hip; n, m < 2^31).
hipError_t sort_rows(bool off64, const void* off, int32_t* tgt, float* w, int64_t n, int64_t m,
                     hipStream_t s);
hipError_t relabel_locality(bool off64, const void* off, const int32_t* tgt, int64_t n,
                            unsigned long long* acc, hipStream_t s);
hipError_t launch_unpermute_i32(const int32_t* in, const int32_t* perm, int64_t n, int32_t* out,
                                hipStream_t s);
hipError_t launch_unpermute_u8(const uint8_t* in, const int32_t* perm, int64_t n, uint8_t* out,
                               hipStream_t s);
hipError_t launch_unpermute_u64(const unsigned long long* in, const int32_t* perm, int64_t n,
                                unsigned long long* out, hipStream_t s);

}  // namespace lpa
