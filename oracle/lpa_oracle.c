/*
 * lpa_oracle.c -- CPU oracle for the label-propagation sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (paper: "nu-LPA: Fast GPU-based Label Propagation
 * Algorithm (LPA) for Community Detection", arXiv 2411.11468):
 *
 *   oracle_lpa_sync      the lpa()/lpaMove() procedure of Algorithm 1, run in
 *                        a deterministic synchronous (Jacobi) order: every
 *                        vertex of an iteration reads the labels as they stood
 *                        when the iteration began.  Label rule = Eq. 3 (the
 *                        label of maximum summed edge weight), ties resolved to
 *                        the smallest label (the "strict" rule of Sec. 4, item
 *                        5, read as smallest id).  Pick-Less every rho-th
 *                        iteration (Sec. 4.1, Algorithm 1), vertex pruning
 *                        (Sec. 4 item 4), tolerance and iteration cap
 *                        (Sec. 4 items 2-3, Algorithm 1).
 *   oracle_modularity    Eq. 1, community form, in fp64.
 *   oracle_modularity_pairs
 *                        Eq. 1, pair form, summed over all ordered vertex
 *                        pairs (O(N^2); tiny graphs only).
 *   oracle_local_optimal per-vertex check that the current label attains the
 *                        maximum of Eq. 3 (used to judge asynchronous runs).
 *   oracle_lpa_sync_cc   oracle_lpa_sync with the Cross-Check swap mitigation
 *                        of Sec. 4.1 in every cc-th iteration (counting from
 *                        0): after the sweep, the vertices that changed are
 *                        visited in increasing id order; a change of vertex i
 *                        to label c is kept when vertex c holds label c at
 *                        that moment (the reverts made so far included), else
 *                        i returns to its previous label.  A reverted vertex
 *                        does not count as changed and flags no neighbour.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *   - ties go to the smallest label;
 *   - Pick-Less is on in iterations l with l mod rho == 0, counting from 0,
 *     and rho == 0 turns it off;
 *   - under Pick-Less a move is made only when the best label is strictly
 *     smaller than the current one; otherwise the vertex keeps its label (the
 *     best label is not re-chosen among smaller ones);
 *   - the stop test is "not Pick-Less and changed/N < tolerance", evaluated
 *     in double precision, N counting every vertex;
 *   - a vertex with no neighbour other than itself keeps its label;
 *   - a processed vertex is un-flagged; a vertex that changes label flags
 *     every CSR neighbour (a self-loop flags the vertex itself);
 *   - self-loops are skipped in the label scan but counted in modularity.
 *
 * The accumulator is a dense fp64 array indexed by label with a list of the
 * labels touched, which is the plain definition of the per-label sum; no
 * hashtable is implemented here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t iteration;
  int32_t pick_less;
  int64_t changed;
  int64_t processed;
  int64_t edges_scanned;
} oracle_iter_stats;

/* Edge weight of CSR entry e; a NULL weight array means every weight is 1. */
static double edge_w(const float* w, int64_t e) { return w ? (double)w[e] : 1.0; }

/*
 * Deterministic synchronous LPA (Algorithm 1 with Jacobi reads).
 *
 * n, off[n+1], tgt[off[n]], w[off[n]] (or NULL): symmetric CSR.
 * tol: per-iteration tolerance (double).  cap: iteration cap.  rho: Pick-Less
 * period (0 = off).  prune: 1 = vertex pruning, 0 = every vertex every time.
 * init: initial labels or NULL (vertex ids).  labels: output, n entries.
 * stats: one record per performed iteration (up to stats_cap).
 * Returns 0 on success, -1 on an allocation failure or bad argument.
 */
int oracle_lpa_sync_cc(int64_t n, const int64_t* off, const int32_t* tgt,
                       const float* w, double tol, int32_t cap, int32_t rho,
                       int32_t cc, int32_t prune, const int32_t* init, int32_t* labels,
                       oracle_iter_stats* stats, int32_t stats_cap,
                       int32_t* iters_done) {
  if (n < 0 || cap < 0 || rho < 0 || cc < 0) return -1;
  *iters_done = 0;
  if (n == 0) return 0;
  int32_t* C = labels;
  int32_t* Cn = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  unsigned char* F = (unsigned char*)malloc((size_t)n);
  unsigned char* Fn = (unsigned char*)malloc((size_t)n);
  double* acc = (double*)calloc((size_t)n, sizeof(double));
  unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!Cn || !F || !Fn || !acc || !seen || !touched) {
    free(Cn); free(F); free(Fn); free(acc); free(seen); free(touched);
    return -1;
  }
  /* Algorithm 1: every vertex starts in its own community and unprocessed. */
  for (int64_t i = 0; i < n; ++i) {
    C[i] = init ? init[i] : (int32_t)i;
    F[i] = 1;
    if (C[i] < 0 || (int64_t)C[i] >= n) {
      free(Cn); free(F); free(Fn); free(acc); free(seen); free(touched);
      return -1;
    }
  }
  for (int32_t l = 0; l < cap; ++l) {
    const int pl = (rho > 0) && (l % rho == 0);
    int64_t changed = 0, processed = 0, scanned = 0;
    memcpy(Cn, C, sizeof(int32_t) * (size_t)n);
    memset(Fn, 0, (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      if (prune && !F[i]) continue;
      ++processed;
      /* Eq. 3: K_{i->c} for every label c seen among the neighbours. */
      int64_t nt = 0;
      for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        ++scanned;
        const int32_t j = tgt[e];
        if ((int64_t)j == i) continue; /* self-loops are not neighbours */
        const int32_t c = C[j];
        if (!seen[c]) { seen[c] = 1; touched[nt++] = c; acc[c] = 0.0; }
        acc[c] += edge_w(w, e);
      }
      if (nt == 0) continue; /* no neighbour: label kept */
      int32_t best = touched[0];
      for (int64_t t = 1; t < nt; ++t) {
        const int32_t c = touched[t];
        if (acc[c] > acc[best] || (acc[c] == acc[best] && c < best)) best = c;
      }
      for (int64_t t = 0; t < nt; ++t) seen[touched[t]] = 0;
      /* Move rule of Algorithm 1 with Pick-Less taken as strictly smaller. */
      if (best != C[i] && (!pl || best < C[i])) {
        Cn[i] = best;
        ++changed;
      }
    }
    /* Cross-Check (Sec. 4.1): visit the changes in id order; Cn holds the
     * labels with the reverts made so far. */
    if (cc > 0 && l % cc == 0) {
      for (int64_t i = 0; i < n; ++i) {
        if (Cn[i] == C[i]) continue;
        const int32_t c = Cn[i];
        if (Cn[c] != c) {
          Cn[i] = C[i];
          --changed;
        }
      }
    }
    /* a vertex whose label changed flags every CSR neighbour */
    for (int64_t i = 0; i < n; ++i)
      if (Cn[i] != C[i])
        for (int64_t e = off[i]; e < off[i + 1]; ++e) Fn[tgt[e]] = 1;
    memcpy(C, Cn, sizeof(int32_t) * (size_t)n);
    if (prune) memcpy(F, Fn, (size_t)n);
    else memset(F, 1, (size_t)n);
    if (l < stats_cap) {
      stats[l].iteration = l;
      stats[l].pick_less = pl;
      stats[l].changed = changed;
      stats[l].processed = processed;
      stats[l].edges_scanned = scanned;
    }
    *iters_done = l + 1;
    if (!pl && (double)changed < tol * (double)n) break;
  }
  free(Cn); free(F); free(Fn); free(acc); free(seen); free(touched);
  return 0;
}

int oracle_lpa_sync(int64_t n, const int64_t* off, const int32_t* tgt,
                    const float* w, double tol, int32_t cap, int32_t rho,
                    int32_t prune, const int32_t* init, int32_t* labels,
                    oracle_iter_stats* stats, int32_t stats_cap,
                    int32_t* iters_done) {
  return oracle_lpa_sync_cc(n, off, tgt, w, tol, cap, rho, 0, prune, init, labels, stats,
                            stats_cap, iters_done);
}

/*
 * Modularity, Eq. 1, community form:
 *   Q = sum_c [ sigma_c / 2m - (Sigma_c / 2m)^2 ]
 * with 2m = sum of all CSR entry weights (every undirected edge appears in
 * both directions), Sigma_c = sum of K_i over vertices of c, sigma_c = sum of
 * w over CSR entries (i,j) with C_i = C_j = c.  Q = 0 when 2m = 0.
 * labels must lie in [0, n).  Returns NAN on a bad label or allocation error.
 */
double oracle_modularity(int64_t n, const int64_t* off, const int32_t* tgt,
                         const float* w, const int32_t* labels) {
  if (n <= 0) return 0.0;
  double* Sig = (double*)calloc((size_t)n, sizeof(double));
  if (!Sig) return NAN;
  double two_m = 0.0, sigma = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t ci = labels[i];
    if (ci < 0 || (int64_t)ci >= n) { free(Sig); return NAN; }
    double Ki = 0.0;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      const double we = edge_w(w, e);
      Ki += we;
      if (labels[tgt[e]] == ci) sigma += we;
    }
    Sig[ci] += Ki;
    two_m += Ki;
  }
  double q = 0.0;
  if (two_m > 0.0) {
    double s2 = 0.0;
    for (int64_t c = 0; c < n; ++c) s2 += (Sig[c] / two_m) * (Sig[c] / two_m);
    q = sigma / two_m - s2;
  }
  free(Sig);
  return q;
}

/*
 * Modularity, Eq. 1, pair form:
 *   Q = 1/2m * sum_{i,j in V} [ A_ij - K_i K_j / 2m ] delta(C_i, C_j)
 * where A_ij sums the weights of the CSR entries (i,j).  The expected-weight
 * term runs over every ordered pair of vertices (i = j included); only then do
 * the two forms of Eq. 1 agree.  O(n^2): tiny graphs only.
 */
double oracle_modularity_pairs(int64_t n, const int64_t* off,
                               const int32_t* tgt, const float* w,
                               const int32_t* labels) {
  if (n <= 0) return 0.0;
  double* K = (double*)calloc((size_t)n, sizeof(double));
  if (!K) return NAN;
  double two_m = 0.0, a_in = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      K[i] += edge_w(w, e);
      if (labels[tgt[e]] == labels[i]) a_in += edge_w(w, e);
    }
    two_m += K[i];
  }
  double q = 0.0;
  if (two_m > 0.0) {
    double expect = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j)
        if (labels[i] == labels[j]) expect += K[i] * K[j] / two_m;
    q = (a_in - expect) / two_m;
  }
  free(K);
  return q;
}

/*
 * For every vertex i, out[i] = 1 when K_{i->C_i} equals max_c K_{i->c}
 * (Eq. 3 with the current labels; ties allowed) or when i has no neighbour
 * other than itself; out[i] = 0 otherwise.  Returns the number of vertices
 * with out[i] = 0, or -1 on an allocation error.
 */
int64_t oracle_local_optimal(int64_t n, const int64_t* off, const int32_t* tgt,
                             const float* w, const int32_t* labels,
                             unsigned char* out) {
  double* acc = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  unsigned char* seen = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!acc || !seen || !touched) { free(acc); free(seen); free(touched); return -1; }
  int64_t bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t nt = 0;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      const int32_t j = tgt[e];
      if ((int64_t)j == i) continue;
      const int32_t c = labels[j];
      if (!seen[c]) { seen[c] = 1; touched[nt++] = c; acc[c] = 0.0; }
      acc[c] += edge_w(w, e);
    }
    double best = 0.0, own = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
      const int32_t c = touched[t];
      if (acc[c] > best) best = acc[c];
      if (c == labels[i]) own = acc[c];
      seen[c] = 0;
    }
    out[i] = (unsigned char)(nt == 0 || own == best);
    if (!out[i]) ++bad;
  }
  free(acc); free(seen); free(touched);
  return bad;
}
