/*
 * lpa.h -- C ABI of the MI355X (gfx950) label-propagation library.
 *
 * The library runs the per-vertex label sweep of nu-LPA (S. Sahu, "nu-LPA:
 * Fast GPU-based Label Propagation Algorithm (LPA) for Community
 * Detection", arXiv 2411.11468) on one AMD Instinct GPU with hand-written HIP
 * kernels.  The method:
 *   - every vertex starts in its own community and unprocessed (Algorithm 1);
 *   - in each iteration every unprocessed vertex is marked processed, sums the
 *     weights of its neighbours per neighbour label in a per-vertex hashtable
 *     with hybrid quadratic-double probing (Algorithm 2, Sec. 4.2), and takes
 *     the label of largest sum (Eq. 3); ties go to the smallest label;
 *   - Pick-Less (Sec. 4.1): in iterations l with l mod pl_period == 0 a vertex
 *     may only move to a strictly smaller label;
 *   - a vertex that changes label marks all its neighbours unprocessed
 *     (vertex pruning, Sec. 4 item 4);
 *   - the run stops after an iteration that is not Pick-Less and in which the
 *     fraction of changed vertices is below the tolerance, or at the
 *     iteration cap (Algorithm 1; defaults 0.05 and 20, Sec. 4).
 *
 * Conventions for every call:
 *   - Return value is an lpa_status; LPA_OK (0) on success.  Nothing aborts
 *     and no C++ exception crosses this boundary.  On error a description is
 *     kept per thread and returned by lpa_last_error().
 *   - Pointers named "device" must be HIP device (or managed) memory of the
 *     current device; pointers named "host" ordinary host memory.  Where a
 *     call accepts either, the kind is detected with hipPointerGetAttributes.
 *   - One lpa_graph handle must not be used from two threads at once.
 *   - All GPU work is enqueued on the stream given to lpa_create (NULL = the
 *     null stream); every call returns after that work has completed.
 */
#ifndef LPA_H_
#define LPA_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lpa_status {
  LPA_OK = 0,
  LPA_ERR_INVALID = 1,     /* bad argument or malformed graph */
  LPA_ERR_OOM = 2,         /* device or host allocation failed */
  LPA_ERR_HIP = 3,         /* a HIP runtime call failed */
  LPA_ERR_STATE = 4,       /* call not valid for this handle */
  LPA_ERR_UNSUPPORTED = 5  /* feature not available in this build */
} lpa_status;

typedef enum lpa_index_t { LPA_INDEX_I32 = 0, LPA_INDEX_I64 = 1 } lpa_index_t;

typedef enum lpa_mode {
  /* Synchronous (Jacobi) sweep: every vertex of an iteration reads the labels
   * as they stood when the iteration began.  Deterministic; with integer
   * weights and every weighted degree below 2^24 its labels and statistics
   * equal the sequential reference exactly. */
  LPA_MODE_DETERMINISTIC = 0,
  /* Asynchronous sweep of the paper (Sec. 4 item 1): one label array updated
   * in place while the sweep runs.  Results depend on scheduling. */
  LPA_MODE_ASYNC = 1
} lpa_mode;

/*
 * Symmetric CSR input (Sec. 3: undirected graph, w_ij = w_ji; every
 * undirected edge is stored in both directions).
 *   num_vertices  N, 0 <= N <= 2^31 - 1
 *   num_edges     M = offsets[N] (directed CSR entries)
 *   offset_type   LPA_INDEX_I32 (requires M <= 2^31 - 1) or LPA_INDEX_I64
 *   offsets       N+1 entries, offsets[0] = 0, non-decreasing, offsets[N] = M
 *   targets       M entries in [0, N); a target equal to its row is a
 *                 self-loop, skipped by the label scan
 *   weights       M finite fp32 values >= 0 (no -0.0), or NULL for all 1.0f;
 *                 an array whose values are all exactly 1.0f is recognised
 *                 by lpa_create and treated as NULL (not read again; the
 *                 same results)
 *   on_device     0: host arrays, copied into library-owned device memory;
 *                 1: device arrays, borrowed: the caller keeps them alive and
 *                 unchanged until lpa_destroy
 *   validate      1: check the conditions above (on the GPU) and fail with
 *                 LPA_ERR_INVALID; 0: trust the caller
 */
typedef struct lpa_csr {
  int64_t num_vertices;
  int64_t num_edges;
  int32_t offset_type;
  int32_t on_device;
  const void* offsets;
  const int32_t* targets;
  const float* weights;
  int32_t validate;
  int32_t reserved;
} lpa_csr;

typedef struct lpa_graph_s* lpa_graph;

/*
 * Degree thresholds that split vertices into kernel classes (all inclusive
 * upper bounds; a vertex of degree D goes to the first class whose bound is
 * >= D; degree 0 is never processed):
 *   small4   rows processed by 4-lane groups in registers     (default 4,
 *                                                              at most 4)
 *   small16  rows processed by 16-lane groups in registers    (default 16,
 *                                                              at most 16)
 *   wave     one wavefront per vertex, LDS hashtable          (default 512,
 *                                                              at most 512)
 *   block    one workgroup per vertex, LDS hashtable up to 16383 slots
 *                                                 (default 8192, at most 8192)
 *   larger degrees ("hubs"): the row is cut into slices, each reduced in an
 *   LDS table by one workgroup; the slices' distinct (label, sum) pairs are
 *   regrouped by a hash bucket of the label and each bucket is summed in an
 *   LDS table by one workgroup; a bucket whose labels overflow its table
 *   spills them into a global-memory hashtable of the hub.
 * Every hashtable holding D keys has 2^m - 1 >= 2D - 1 slots (load <= 1/2).
 * hub_chunk: edges per workgroup slice for the largest rows (default 8192).
 * max_retries: hybrid probes before the linear continuation (default 32).
 * xcd_local: bit 0 (1): the hub buckets of consecutive indices run on one
 *   XCD (their pair runs share cache lines); bit 1 (2): when every hub is
 *   flagged and the rows hold strictly increasing targets, the hub slices
 *   are taken in eight groups by target window, group x first by the
 *   workgroups on XCD x (each XCD's L2 then holds the labels of one window
 *   of ids); 0 = plain round-robin (default 3; every value gives the same
 *   results).
 * hub_table_cap: 0 (default) = bucket tables of up to 16383 slots; else at
 *   most this many slots (rounded down to 2^m - 1), to exercise the spill
 *   path in tests.
 * relabel: where the handle keeps each vertex's label and row.  1 = in an
 *   internal order by degree, largest first (8 steps per octave, ties by
 *   id), built once by lpa_create as a second copy of the CSR (plus its
 *   targets once more as the caller's ids, 4 bytes per entry, which the
 *   first sweep of a run streams): the label reads of every sweep then
 *   concentrate on few cache lines.  0 = in the
 *   caller's order.  -1 (default) = automatic: internal order when N > 2^20
 *   and fewer than half of the CSR entries of a row sample point within
 *   2^16 ids of their row.  Label values, results and every array passed in
 *   or out stay in the caller's numbering either way; a deterministic run
 *   returns the same labels.  lpa_create_batched keeps the caller's order
 *   (relabel = 1 there is LPA_ERR_UNSUPPORTED).
 * probe: the hashtables' probe sequence (Sec. 4.2): 0 = quadratic-double
 *   (default: step 1, then 2*step + (key mod p2)), 1 = linear, 2 = quadratic
 *   (step doubled on each collision), 3 = double hashing (step key mod p2);
 *   every mode continues linearly after max_retries probes.  The same
 *   results; for measuring the probe sequences against each other.
 * table_values: the precision of the hashtable values (Sec. 4.4 compares
 *   32- and 64-bit).  0 (default) = 32-bit, in every class kernel above.
 *   32 or 64 = 32- or 64-bit values in one simpler kernel set used for
 *   both widths, so that only the width differs between the two: a wave per
 *   row of up to `wave` entries, a workgroup per row of up to 4096 entries
 *   (LDS tables of up to 8191 slots; `block` is capped at 4096), and for
 *   longer rows every slice adding into the row's global-memory table; no
 *   register-only classes and no table-free first sweep.  Not with learned
 *   runs, traces or lpa_create_batched (LPA_ERR_UNSUPPORTED).
 * batch_queue (lpa_create_batched only): how a batched run is scheduled.
 *   1 = a persistent work queue: per iteration one resident grid pops
 *   (graph, vertex chunk) items from atomic queues, one part per XCD holding
 *   all chunks of the graphs assigned to it, and processes each chunk's
 *   flagged vertices; a per-graph kernel then applies the stop test and
 *   queues the chunks that hold flagged vertices or changed labels.  Rows
 *   of up to 512 entries only (a longer row makes it LPA_ERR_UNSUPPORTED).
 *   0 = the degree-class kernels of a single graph over the packed CSR.
 *   -1 (default) = the work queue when every row has at most 512 entries.
 *   Both give the same results.  Runs without pruning (prune = 0) always
 *   take the class kernels.
 * queue_chunk: vertices per queue item, a power of two in 64 .. 1024
 *   (0 = default 512).
 * queue_group: rows of up to this many entries (16 .. 64, 0 = default 64)
 *   are processed by 16 lanes each with a 127-slot LDS table; longer rows
 *   by a wavefront each with a 1023-slot table.
 * sort_rows: with the internal order (relabel), sort each row of the
 *   internal CSR by target id at create, so that the label reads of a row
 *   walk upwards through the label array and the entries in its dense
 *   low-id part share cache lines.  1 = sort, 0 = keep the caller's entry
 *   order, -1 (default) = sort.  The same results.
 * block_threads: threads per workgroup of the four workgroup classes (rows
 *   of wave+1 .. block entries): 0 (default) = 256, 256, 512 and 1024 for
 *   the 2047-, 4095-, 8191- and 16383-slot tables; 256, 512 or 1024 = that
 *   many for all four.  Learned runs keep the defaults.
 * table_load: the hashtable capacity of a row of D entries, as a bound on
 *   its load: 1 = nextPow2(D) - 1 (the smallest 2^m > D, minus one: the
 *   paper's, up to full load), 2 (default) = the smallest 2^m >= 2D, minus
 *   one (load <= 1/2), 4 = the smallest 2^m >= 4D, minus one (load <= 1/4),
 *   capped by the class's LDS table.  Same results.
 * pull_divisor: the neighbour flags of an iteration are pulled (every vertex
 *   checks its row) when the changed rows hold at least 1/pull_divisor of
 *   the CSR entries, else pushed (each changed row flags its neighbours);
 *   default 16.  Same flags.
 * memory_limit_kib: a cap on the device memory the handle keeps (its copies
 *   of the graph, labels, flags, lists, tables and run buffers, allocated by
 *   lpa_create and on first use by lpa_run / lpa_modularity), in KiB; 0
 *   (default) = none.  An allocation that would pass it fails with
 *   LPA_ERR_OOM like a failed hipMalloc; a failed lpa_create frees
 *   everything it allocated.  Buffers used only during lpa_create (checks,
 *   sort scratch) are freed before it returns and are not counted.
 */
typedef struct lpa_tuning {
  int32_t small4;
  int32_t small16;
  int32_t wave;
  int32_t block;
  int32_t hub_chunk;
  int32_t max_retries;
  int32_t xcd_local;
  int32_t hub_table_cap;
  int32_t relabel;
  int32_t probe;
  int32_t table_values;
  int32_t batch_queue;
  int32_t queue_chunk;
  int32_t queue_group;
  int32_t sort_rows;
  int32_t block_threads;
  int32_t table_load;
  int32_t pull_divisor;
  int32_t memory_limit_kib;
} lpa_tuning;

/*
 * Per-run options (Algorithm 1 and Sec. 4).
 *   mode            lpa_mode
 *   tolerance       stop when not Pick-Less and changed < tolerance * N,
 *                   compared in double precision (default 0.05)
 *   max_iterations  iteration cap (default 20)
 *   pl_period       Pick-Less in iterations l with l % pl_period == 0,
 *                   counting from 0; 0 disables Pick-Less (default 4)
 *   prune           1: only flagged vertices are processed (default 1)
 *   initial_labels  NULL: label = vertex id; else N labels in [0, N), host or
 *                   device memory
 *   profile         1: bracket every kernel launch with HIP events and add its
 *                   duration and algorithmic bytes to the per-kernel profile
 *                   read by lpa_profile (default 0)
 *   launch          lpa_launch (default LPA_LAUNCH_EAGER)
 *   flag_mode       how the neighbours of the vertices changed in an
 *                   iteration are flagged after its sweep (the flags are
 *                   identical on a symmetric graph):
 *                   LPA_FLAGS_PUSH  each changed vertex writes its neighbours'
 *                                   flags;
 *                   LPA_FLAGS_PULL  every vertex reads its neighbours' change
 *                                   marks up to the first changed one;
 *                   LPA_FLAGS_AUTO  pull when the changed vertices' rows hold
 *                                   at least 1/16 of the CSR entries, push
 *                                   otherwise, decided on the GPU per
 *                                   iteration (default)
 *   learned         1: skip the vertices that the predictor attached with
 *                   lpa_set_predictor marks unchanged (see there; a project
 *                   addition, not in the paper); 0: plain run (default)
 *   cc_period       Cross-Check (Sec. 4.1) in iterations l with
 *                   l % cc_period == 0, counting from 0; 0 = off (default).
 *                   After such an iteration's moves, the changed vertices are
 *                   checked in increasing id order: a change to label c is
 *                   kept when vertex c holds label c at that point (earlier
 *                   reverts included), else the vertex returns to its previous
 *                   label and counts as unchanged.  May be combined with
 *                   pl_period (the paper's hybrid).  Single-graph runs with
 *                   launch = LPA_LAUNCH_EAGER and learned = 0 only (else
 *                   LPA_ERR_UNSUPPORTED): the id-order check is resolved by
 *                   rounds the host repeats until nothing changes.
 */
typedef enum lpa_flag_mode {
  LPA_FLAGS_AUTO = 0,
  LPA_FLAGS_PUSH = 1,
  LPA_FLAGS_PULL = 2
} lpa_flag_mode;

typedef enum lpa_launch {
  /* one host round trip per iteration: per-iteration GPU time in the stats,
   * per-kernel profile available */
  LPA_LAUNCH_EAGER = 0,
  /* one iteration captured once as a HIP graph and replayed max_iterations
   * times without host round trips; the kernels of iterations after the stop
   * return at once; stats carry no per-iteration time; profile ignored */
  LPA_LAUNCH_GRAPH = 1
} lpa_launch;

typedef struct lpa_options {
  int32_t mode;
  int32_t max_iterations;
  double tolerance;
  int32_t pl_period;
  int32_t prune;
  const int32_t* initial_labels;
  int32_t profile;
  int32_t flag_mode;
  int32_t launch;
  int32_t learned;
  int32_t cc_period;
} lpa_options;

/* Statistics of one iteration. */
typedef struct lpa_iter_stats {
  int32_t iteration;      /* 0-based */
  int32_t pick_less;      /* 1 if Pick-Less applied */
  int64_t changed;        /* vertices whose label changed */
  int64_t processed;      /* vertices processed (flagged at the start) */
  int64_t edges_scanned;  /* CSR entries read by the label scan */
  float ms;               /* GPU time of the iteration (eager launch) */
  int32_t skipped;        /* learned runs: flagged vertices left unprocessed */
} lpa_iter_stats;

/*
 * Accumulated per-kernel profile of the runs made with profile = 1.
 * name: kernel ("sweep_block16383", "hub_acc", "frontier", ...);
 * launches, total_ms: launches and summed GPU durations (HIP events on the
 * handle's stream); bytes: algorithmic bytes moved -- per scanned CSR entry
 * the target (4 B), the weight (4 B, none for unit weights) and the gathered
 * neighbour label (4 B); per processed vertex its active-list id (4 B), two
 * row offsets and its own label (4 B); per change the new label (4 B, 8 B for
 * a queued pair in deterministic mode) and one flag byte per neighbour;
 * edges, vertices: CSR entries scanned and vertices processed.
 */
typedef struct lpa_kernel_profile {
  char name[24];
  int64_t launches;
  double total_ms;
  double bytes;
  int64_t edges;
  int64_t vertices;
} lpa_kernel_profile;

/* Fill *opt with the defaults above. */
void lpa_options_default(lpa_options* opt);

/* Fill *t with the default thresholds above. */
void lpa_tuning_default(lpa_tuning* t);

/*
 * Upload (or borrow) a graph and build its degree classes on the GPU.
 * stream: a hipStream_t or NULL.  tuning: NULL for the defaults.
 * On success *out holds a new handle; on error *out is NULL.
 * Errors: LPA_ERR_INVALID (bad sizes, malformed CSR when validate = 1),
 * LPA_ERR_OOM, LPA_ERR_HIP.
 */
lpa_status lpa_create(const lpa_csr* g, void* stream, const lpa_tuning* tuning,
                      lpa_graph* out);

/*
 * Run label propagation to termination.
 *   labels      caller-owned output, N int32, host or device memory
 *   stats       caller-owned host array of stats_cap records (may be NULL
 *               when stats_cap = 0); record l describes iteration l
 *   iters_done  host int32: number of iterations performed (may be NULL)
 * Errors: LPA_ERR_INVALID (bad options, stats_cap < 0, bad initial labels),
 * LPA_ERR_HIP.
 */
lpa_status lpa_run(lpa_graph g, const lpa_options* opt, int32_t* labels,
                   lpa_iter_stats* stats, int32_t stats_cap,
                   int32_t* iters_done);

/*
 * Batched label propagation over many independent graphs packed into one CSR.
 * Graph q owns vertices v_off[q] .. v_off[q+1]-1 (v_off: num_graphs + 1 host
 * int64, from 0 to csr->num_vertices); every CSR entry of a row of graph q
 * must point into graph q (checked when csr->validate = 1).  Vertex ids and
 * labels are global: a graph's initial labels are its global vertex ids, so
 * ties among them order as in a solo run of the graph.
 * lpa_run_batched runs Algorithm 1 on every graph at once with one iteration
 * counter: each graph stops after its own first iteration that is not
 * Pick-Less and in which fewer than tolerance * (its vertex count) of its
 * vertices changed, or at the cap; a stopped graph's vertices are no longer
 * processed.  The result for each graph equals a solo lpa_run of that graph
 * (exactly in deterministic mode), labels offset by v_off[q].
 *   labels                  N int32, host or device
 *   iters_per_graph         num_graphs host int32 (may be NULL): iterations
 *                           graph q performed
 *   changed_last_per_graph  num_graphs host int64 (may be NULL): vertices of
 *                           graph q changed in its last iteration
 *   iters_done              host int32 (may be NULL): iterations of the batch
 * lpa_run, lpa_modularity and the other calls accept a batched handle too
 * (lpa_run then reports statistics summed over the graphs).
 */
lpa_status lpa_create_batched(int32_t num_graphs, const int64_t* v_off, const lpa_csr* csr,
                              void* stream, const lpa_tuning* tuning, lpa_graph* out);
lpa_status lpa_run_batched(lpa_graph g, const lpa_options* opt, int32_t* labels,
                           int32_t* iters_per_graph, int64_t* changed_last_per_graph,
                           int32_t* iters_done);

/*
 * Change predictor (a project addition, not in the paper): a perceptron
 * 12 -> 64 -> 64 -> 1 (ReLU, sigmoid output) that estimates, from a flagged
 * vertex's features, the probability that processing it changes its label.
 * Parameters: LPA_PREDICTOR_PARAMS fp32 values in the order W1[12][64],
 * b1[64], W2[64][64], b2[64], W3[64], b3 (W[k][j] maps input k to unit j);
 * the network computes with bf16 weights and inputs and fp32 accumulation.
 * Samples X are n rows of 12 fp32 features, labels y are 0/1 fp32; both host
 * or device memory.  The loss is the mean binary cross-entropy with the
 * positive class weighted by pos_weight; the optimiser is Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected).
 */
#define LPA_PREDICTOR_PARAMS 5057
typedef struct lpa_predictor_s* lpa_predictor;

typedef struct lpa_train_options {
  int32_t epochs;
  int32_t batch;       /* samples per Adam step */
  float lr;
  float pos_weight;
  uint64_t seed;       /* sample order */
} lpa_train_options;

/* New predictor with He-uniform weights drawn from seed, zero biases. */
lpa_status lpa_predictor_create(uint64_t seed, void* stream, lpa_predictor* out);
void lpa_predictor_destroy(lpa_predictor p);
/* Replace / read the fp32 parameters (host arrays); set also resets Adam. */
lpa_status lpa_predictor_set_params(lpa_predictor p, const float* params);
lpa_status lpa_predictor_get_params(lpa_predictor p, float* params);
/* Checkpoint and resume (host memory): lpa_predictor_save writes the
 * network's shape, its fp32 parameters and Adam's state (moments and step
 * count) into blob (cap bytes) and the blob's size into *size; blob NULL
 * only reports the size (LPA_PREDICTOR_BLOB_BYTES).  lpa_predictor_load
 * restores them into p: it then holds exactly the saved state (the same
 * predictions; training continues from the same parameters and moments,
 * and follows the saved predictor up to the order of the gradient's float
 * atomic sums).  Layout: a 32-byte header
 * (magic "LPAPRED1", uint32 version 1, uint16 layer sizes 12, 64, 64, 1,
 * uint32 parameter count 5057, int32 Adam steps, uint32 0), then 3 x 5057
 * fp32 (parameters, first moments, second moments), little-endian.
 * Errors: LPA_ERR_INVALID (cap too small; load: wrong magic, version or
 * shape, truncated, non-finite parameters; p unchanged then), LPA_ERR_HIP. */
#define LPA_PREDICTOR_BLOB_BYTES (32 + 3 * 4 * LPA_PREDICTOR_PARAMS)
lpa_status lpa_predictor_save(lpa_predictor p, void* blob, int64_t cap, int64_t* size);
lpa_status lpa_predictor_load(lpa_predictor p, const void* blob, int64_t size);
/* Gradient of the loss over the n samples (grad: host, may be NULL; loss:
 * host mean loss, may be NULL). */
lpa_status lpa_predictor_gradient(lpa_predictor p, const float* X, const float* y, int64_t n,
                                  float pos_weight, float* grad, double* loss);
/* One Adam step with the given host gradient (NULL: the last computed one). */
lpa_status lpa_predictor_adam(lpa_predictor p, const float* grad, float lr);
/* Minibatch training; final_loss (host, may be NULL): mean loss of the last
 * epoch. */
lpa_status lpa_predictor_train(lpa_predictor p, const float* X, const float* y, int64_t n,
                               const lpa_train_options* opt, float* final_loss);
/* Probabilities for n samples (prob: host or device). */
lpa_status lpa_predictor_predict(lpa_predictor p, const float* X, int64_t n, float* prob);

/*
 * Learned skipping (a project addition, not in the paper).  A graph with a
 * predictor attached runs, when lpa_options.learned = 1, Algorithm 1 with
 * these changes:
 *  - every evaluated vertex of degree 1 .. lpa_tuning.block (the vertices of
 *    the non-hub classes) keeps an 8-byte state record (label shares of its
 *    last evaluation, log-quantised degrees, change history, iteration);
 *  - from iteration 1 on, the frontier computes 12 features from the record
 *    of each flagged such vertex and runs the predictor on them (bf16 MFMA);
 *    in a skipping iteration a vertex whose probability of change is below
 *    threshold is not processed and keeps its flag;
 *  - iteration l skips unless l % guard_period == 0 or the previous
 *    iteration changed fewer than 2 * tolerance * N labels (guard_period 0:
 *    no periodic guard); the other iterations are plain sweeps that still
 *    predict, and if more than fn_bound of the vertices predicted unchanged
 *    in such a sweep change, skipping is off for the rest of the run;
 *  - the stop test of Algorithm 1 is applied to changed + skipped (an upper
 *    bound on what the plain sweep of the iteration would have changed).
 * Features, in order: log-quantised degree and weighted degree (/ 64), own
 * label share, best-second margin, best-own gain (/ 255 of the total
 * weight), changed in l-1, l-2, l-3, l / cap, Pick-Less in l, iterations
 * since the last evaluation / cap, distinct labels per entry.
 */
typedef struct lpa_learned_options {
  float threshold;        /* skip when P(change) < threshold (default 0.1) */
  float fn_bound;         /* fallback bound on false negatives (default 0.02) */
  int32_t guard_period;   /* plain guard sweep every guard_period (default 4) */
  int32_t predict_small;  /* 1: rows of at most small16 entries are predicted
                             (and keep records, and are traced) too; 0
                             (default): they are always processed, by the
                             plain register kernels */
  int32_t predict_large;  /* 1: rows of wave+1 .. block entries (the
                             workgroup classes) are predicted too; 0
                             (default): they are always processed, by the
                             plain pipelined kernels.  Longer rows are never
                             predicted */
  int32_t first_predicted;  /* first iteration with predictions (>= 1,
                               default 2); the records are kept from the
                               iteration before, and traces sample from this
                               iteration on */
} lpa_learned_options;

typedef struct lpa_learned_iter {
  int32_t iteration;
  int32_t skipping;         /* 1 if the iteration skipped predicted vertices */
  int32_t fallback;         /* skipping switched off after this iteration */
  int32_t reserved;
  int64_t skipped;          /* flagged vertices left unprocessed */
  int64_t predicted;        /* vertices predicted unchanged */
  int64_t false_negatives;  /* plain iterations: of those, changed */
} lpa_learned_iter;

void lpa_learned_options_default(lpa_learned_options* o);
/* Attach p (NULL detaches) with options lo (NULL: defaults).  The graph
 * reads p's parameters at every run; p must outlive its use by g.
 * Errors: LPA_ERR_INVALID (threshold outside (0, 1), fn_bound < 0,
 * guard_period < 0); LPA_ERR_UNSUPPORTED (batched handle). */
lpa_status lpa_set_predictor(lpa_graph g, lpa_predictor p, const lpa_learned_options* lo);
/* Per-iteration skipping statistics of the last learned run (count: host,
 * iterations written, at most cap). */
lpa_status lpa_learned_history(lpa_graph g, lpa_learned_iter* out, int32_t cap,
                               int32_t* count);
/* The N state records after the last learned or traced run (8 N bytes, host
 * or device).  Errors: LPA_ERR_STATE before any such run. */
lpa_status lpa_get_records(lpa_graph g, uint64_t* out);
/*
 * Training traces: run Algorithm 1 as lpa_run with opt (learned skipping if
 * opt->learned, eager launch) and, in every iteration l >= 1, sample each
 * processed vertex of a non-hub class with probability sample_rate: the
 * draw is u = (SplitMix64 output of state seed + 0x9E3779B97F4A7C15 *
 * (1 + (l << 32 | v))) >> 11, taken when u * 2^-53 < sample_rate.  A sample
 * is its 12 features at the start of the iteration (X, row-major), 1 if the
 * vertex then changed label else 0 (y), the vertex and the iteration.  X, y,
 * vertex, iteration: cap entries each (12 cap for X), host or device; vertex
 * and iteration may be NULL.  Samples beyond cap are drawn but dropped;
 * *count (host) receives the number drawn; their order is unspecified.
 */
lpa_status lpa_trace(lpa_graph g, const lpa_options* opt, double sample_rate, uint64_t seed,
                     float* X, float* y, int32_t* vertex, int32_t* iteration, int64_t cap,
                     int64_t* count);

/*
 * Autotuner: pick lpa_tuning for a graph (num_graphs = 0) or a packed batch
 * (num_graphs, v_off as for lpa_create_batched) by successive halving in
 * stages, each over a grid around the best tuning so far (the defaults
 * first): for a batch, the schedule (batch_queue 0, or 1 with queue_chunk
 * 128/256/512/1024 and queue_group 16/32/64); unless the work queue won,
 * the class thresholds (small4 2/4, small16 8/16, wave 128/256/512, block
 * 2048/4096/8192) with slice sizes (4096/8192), then the workgroup sizes
 * (block_threads 0/256/512/1024), table capacities (table_load 1/2/4) and
 * flag policy (pull_divisor 8/16/32).  Each candidate is a fresh handle
 * timed on complete runs with opt (NULL: defaults; profile and learned are
 * turned off); each round keeps the fastest third and doubles the timed
 * runs; a tuning the handle refuses (LPA_ERR_UNSUPPORTED) drops out.  The
 * stages share budget_ms of wall time (the best measured so far is
 * returned when it runs out).
 * The graph is validated once, on the first handle.  Device-resident arrays
 * avoid a copy per candidate.
 * Errors: as lpa_create / lpa_run; LPA_ERR_INVALID for budget_ms <= 0.
 */
typedef struct lpa_tune_report {
  int32_t candidates;   /* grid sizes, summed over the stages */
  int32_t runs;         /* lpa_run calls made */
  int32_t rounds;
  int32_t reserved;
  double best_ms;       /* median run time of the chosen tuning, last round */
  double default_ms;    /* median run time of the defaults, first round */
  double elapsed_ms;    /* wall time of the search */
} lpa_tune_report;

lpa_status lpa_autotune(const lpa_csr* csr, int32_t num_graphs, const int64_t* v_off,
                        void* stream, const lpa_options* opt, double budget_ms,
                        lpa_tuning* best, lpa_tune_report* report);

/*
 * Modularity of a labelling, Eq. 1, in fp64:
 *   Q = sum_c [ sigma_c / 2m - (Sigma_c / 2m)^2 ]
 * with 2m the total CSR weight, Sigma_c the summed weighted degree of the
 * vertices of c and sigma_c the CSR weight between vertices of c.
 *   labels  N int32 in [0, N), host or device memory
 *   q       host double; 0 when the graph has no weight
 * Errors: LPA_ERR_INVALID (label out of range), LPA_ERR_HIP.
 */
lpa_status lpa_modularity(lpa_graph g, const int32_t* labels, double* q);

/*
 * lpa_modularity that allocates no device memory, for callers that cannot
 * allocate: code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result and errors as lpa_modularity,
 * for graphs of at most LPA_MODULARITY_NOALLOC_MAX_VERTICES vertices
 * (larger: LPA_ERR_INVALID, nothing launched).  Its scratch (per-community
 * sums and accumulators, 32 MiB) is a fixed array in the library's device
 * code: each GPU the library runs on holds one copy until the process ends,
 * and every call on that GPU uses it, so calls that overlap on one GPU (from
 * several threads or streams) race and must not be made; each call clears
 * what it uses.  Host labels are staged through the handle's own buffer
 * (allocated by lpa_create).
 */
#define LPA_MODULARITY_NOALLOC_MAX_VERTICES 4194304
lpa_status lpa_modularity_noalloc(lpa_graph g, const int32_t* labels, double* q);

/*
 * Ceiling of the sweep kernels' memory side: the rate (CSR entries per
 * second, into *reads_per_s) of a pass that does nothing but read every
 * entry's target and then its neighbour's label, in the order and vertex
 * numbering the sweeps use (the internal order when the handle has one),
 * averaged over reps passes after one warm-up.  Resets the handle's labels
 * and flags to the plain start (labels = ids, all flagged); a later lpa_run
 * starts afresh anyway.
 * Errors: LPA_ERR_INVALID (NULL, reps < 1), LPA_ERR_OOM, LPA_ERR_HIP.
 */
lpa_status lpa_label_read_rate(lpa_graph g, int32_t reps, double* reads_per_s);

/*
 * Number of vertices in each degree class, in the order: degree 0, small4,
 * small16, wave, block (all LDS sizes), hub.  counts must hold 6 entries.
 */
lpa_status lpa_graph_classes(lpa_graph g, int64_t* counts);

/*
 * Copy the per-vertex flags left by the last lpa_run into flags (N bytes, host
 * or device memory): 1 = the vertex was marked unprocessed by a neighbour's
 * change and would be processed in a further iteration, 0 = not flagged.
 * Used to check an asynchronous run: every vertex that is not flagged holds a
 * label of maximum weight (Eq. 3), unless Pick-Less refused its move.  A
 * single-graph run does not flag after the iteration it stops on; the first
 * lpa_get_flags after it sets those flags from the run's change marks (one
 * pull pass), so the result is the same.
 */
lpa_status lpa_get_flags(lpa_graph g, uint8_t* flags);

/*
 * Copy up to cap kernel records (kernels launched at least once since the
 * last reset) into out; *count receives the number of such kernels.
 */
lpa_status lpa_profile(lpa_graph g, lpa_kernel_profile* out, int32_t cap,
                       int32_t* count);

/* Clear the accumulated per-kernel profile. */
lpa_status lpa_profile_reset(lpa_graph g);

/* Release the handle and all library-owned memory.  NULL is allowed. */
void lpa_destroy(lpa_graph g);

/* Static description of a status code. */
const char* lpa_status_string(lpa_status s);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* lpa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LPA_H_ */
