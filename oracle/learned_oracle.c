/*
 * learned_oracle.c -- CPU oracle for label propagation with a learned
 * change predictor (a project addition on top of Algorithm 1; the paper has
 * no such step).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library.
 *
 * The run is Algorithm 1 in synchronous (Jacobi) order, exactly as
 * oracle_lpa_sync in lpa_oracle.c (Eq. 3 label rule, ties to the smallest
 * label, Pick-Less in iterations l mod rho == 0, pruning, tolerance and cap),
 * with three additions:
 *
 *  1. A per-vertex state record of 8 bytes, rewritten whenever the vertex is
 *     processed (every vertex with min_pred_degree <= D_i <= max_pred_degree,
 *     D_i = row length, min_pred_degree >= 1: the rows that are predicted)
 *     in an iteration l >= pred_start - 1 (the evaluation before the first
 *     prediction on).  From the label sums of that evaluation (fp32 values of the
 *     sums; all sums skip self-loops, labels as at the iteration start):
 *        K     = total neighbour weight,  own = weight of the current label,
 *        best  = maximum label weight,    second = largest weight among the
 *                other labels (0 if none), distinct = number of labels,
 *     and q(x) = floor(255 * x / K) in fp32 (0 when K = 0):
 *        byte 0  q(own)
 *        byte 1  q(best - second)
 *        byte 2  q(best - own)
 *        byte 3  floor(255 * distinct / D_i)            (integer)
 *        byte 4  lq(1 + D_i)                            (integer)
 *        byte 5  lq of the fp32 value 1 + K             (from its bits)
 *        byte 6  change history: bit k = the vertex changed label when it
 *                was evaluated k iterations before byte 7's iteration
 *                (bits 0..6; bit 7 is always 0 here)
 *        byte 7  iteration of this evaluation (at most 254); 255 = never
 *     where lq(u) = min(255, 8 e + m), e = floor(log2 u) and m the three
 *     bits after the leading one (a piecewise-linear log2 in eighths).
 *
 *  2. Features of a flagged vertex at the start of iteration l (fp32):
 *        f0 = byte4 / 64          f1 = byte5 / 64
 *        f2 = byte0 / 255         f3 = byte1 / 255       f4 = byte2 / 255
 *        f5, f6, f7 = changed in iteration l-1, l-2, l-3 (0/1)
 *        f8 = l / cap             f9 = 1 if iteration l is Pick-Less
 *        f10 = min(l - byte7, cap) / cap  (1 if never evaluated)
 *        f11 = byte3 / 255
 *     and the network 12 -> 64 -> 64 -> 1 (ReLU) evaluated in fp64 on bf16
 *     values of the weights and features, the first hidden layer rounded to
 *     bf16 (through fp32), the second not; biases fp32.  The vertex is
 *     predicted unchanged when the logit z is below z_theta.
 *
 *  3. The schedule.  Iteration l "skips" when a predictor is given,
 *     l >= pred_start (>= 1),
 *     l is not a multiple of the guard period (0: no periodic guard), the
 *     previous iteration changed at least 2 * tolerance * N labels (below
 *     that the run is near its stop and the plain sweep is taken, so that
 *     the stop comes where the plain run's would), and the fallback is off.  In a skipping iteration a flagged vertex with
 *     min_pred_degree <= D_i <= max_pred_degree that is predicted unchanged
 *     is not processed and stays flagged; shorter and longer rows are never
 *     predicted.  Every other iteration is plain; in a
 *     plain iteration with l >= pred_start and the fallback off the predictions are
 *     still made, and if more than fn_bound of the vertices predicted
 *     unchanged do change, the fallback turns on for the rest of the run.
 *     The run stops after an iteration that is not Pick-Less and in which
 *     changed + skipped < tolerance * N, or at the cap.  The skipped
 *     vertices bound what the plain sweep of the same iteration could have
 *     changed in addition (every other vertex reads the iteration-start
 *     labels either way), so the test is Algorithm 1's, applied to an upper
 *     bound of the plain count; with nothing skipped it is Algorithm 1's.
 *
 * Traces: in every iteration l >= pred_start, each processed vertex with
 * min_pred_degree <= D_i <= max_pred_degree whose sample draw falls below sample_rate
 * contributes its features (at the iteration start) and whether it changed
 * label.  The draw is SplitMix64 (Steele, Lea and Flood 2014): state =
 * seed + 0x9E3779B97F4A7C15 * (1 + (l << 32 | v)), then the SplitMix64 output
 * mix of that state; the draw is (output >> 11) * 2^-53.
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
  int64_t skipped;        /* flagged vertices left unprocessed */
  int64_t predicted;      /* vertices predicted unchanged */
  int64_t false_neg;      /* of those, processed and changed (plain iterations) */
  int32_t skipping;       /* 1 if this iteration skipped */
  int32_t fallback;       /* fallback state after this iteration */
} oracle_learned_stats;

enum { N_IN = 12, N_H = 64 };

/* bfloat16 value of a float: round to nearest, ties to even, on the bits. */
static float to_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
    u = (u | 0x00400000u) & 0xFFFF0000u;
  } else {
    const uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
  }
  float r;
  memcpy(&r, &u, 4);
  return r;
}

/* Logit of the network for one feature vector.  P: 5,057 fp32 parameters in
 * the order W1[12][64], b1[64], W2[64][64], b2[64], W3[64], b3. */
static double mlp_logit(const float* P, const float f[N_IN]) {
  const float* W1 = P;
  const float* b1 = W1 + N_IN * N_H;
  const float* W2 = b1 + N_H;
  const float* b2 = W2 + N_H * N_H;
  const float* W3 = b2 + N_H;
  const float* b3 = W3 + N_H;
  double x[N_IN], h1[N_H];
  for (int k = 0; k < N_IN; ++k) x[k] = (double)to_bf16(f[k]);
  for (int j = 0; j < N_H; ++j) {
    double a = (double)b1[j];
    for (int k = 0; k < N_IN; ++k) a += x[k] * (double)to_bf16(W1[k * N_H + j]);
    const double r = a > 0.0 ? a : 0.0;
    h1[j] = (double)to_bf16((float)r);
  }
  double z = (double)b3[0];
  for (int j = 0; j < N_H; ++j) {
    double a = (double)b2[j];
    for (int k = 0; k < N_H; ++k) a += h1[k] * (double)to_bf16(W2[k * N_H + j]);
    const double h2 = a > 0.0 ? a : 0.0;
    z += h2 * (double)to_bf16(W3[j]);
  }
  return z;
}

static uint8_t lq_int(uint64_t u) { /* u >= 1 */
  int e = 63;
  while (!((u >> e) & 1u)) --e;
  const uint64_t m = e >= 3 ? (u >> (e - 3)) & 7u : (u << (3 - e)) & 7u;
  const uint64_t q = 8u * (uint64_t)e + m;
  return (uint8_t)(q > 255u ? 255u : q);
}

static uint8_t lq_float(float x) { /* x >= 1 */
  uint32_t b;
  memcpy(&b, &x, 4);
  const int e = (int)(b >> 23) - 127;
  const int q = 8 * e + (int)((b >> 20) & 7u);
  return (uint8_t)(q > 255 ? 255 : (q < 0 ? 0 : q));
}

static uint8_t q255(float x, float K) {
  if (!(K > 0.0f)) return 0;
  const float t = floorf((255.0f * x) / K);
  return (uint8_t)(t > 255.0f ? 255.0f : (t < 0.0f ? 0.0f : t));
}

static double draw(uint64_t seed, int32_t l, int64_t v) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (1ull + (((uint64_t)(uint32_t)l << 32) | (uint64_t)v));
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

/* Features of vertex record r at the start of iteration l. */
static void features(const uint8_t* r, int32_t l, int32_t cap, int32_t rho, float f[N_IN]) {
  const int never = r[7] == 255;
  const int32_t age = never ? cap : l - (int32_t)r[7];
  f[0] = (float)r[4] / 64.0f;
  f[1] = (float)r[5] / 64.0f;
  f[2] = (float)r[0] / 255.0f;
  f[3] = (float)r[1] / 255.0f;
  f[4] = (float)r[2] / 255.0f;
  for (int j = 1; j <= 3; ++j) {
    const int32_t k = j - age; /* bit of the iteration l - j */
    f[4 + j] = (!never && k >= 0 && k <= 6) ? (float)((r[6] >> k) & 1u) : 0.0f;
  }
  f[8] = (float)l / (float)cap;
  f[9] = (rho > 0 && l % rho == 0) ? 1.0f : 0.0f;
  f[10] = (float)(age < cap ? age : cap) / (float)cap;
  f[11] = (float)r[3] / 255.0f;
}

/*
 * n, off, tgt, w (NULL = unit weights): symmetric CSR.  tol, cap, rho, prune
 * as in oracle_lpa_sync.  guard: guard period.  min_pred_degree (>= 1),
 * max_pred_degree: shortest and longest row length that is predicted (and
 * recorded).  pred_start (>= 1): first iteration with predictions.  params: 5,057 fp32 values, or
 * NULL for no predictor (plain schedule, records and traces still kept).
 * z_theta: logit threshold.  fn_bound: fallback bound.  sample_rate, seed,
 * tX (cap x 12), ty, tv, tl, tcap, tcount: trace output (tX NULL = none).
 * labels: output.  rec: 8 n bytes out.  stats: per iteration.  min_margin:
 * smallest |z - z_theta| over every prediction made (INFINITY if none).
 * Returns 0, or -1 on a bad argument or allocation failure.
 */
int oracle_lpa_learned(int64_t n, const int64_t* off, const int32_t* tgt, const float* w,
                       double tol, int32_t cap, int32_t rho, int32_t prune, int32_t guard,
                       int64_t min_pred_degree, int64_t max_pred_degree, int32_t pred_start,
                       const float* params, double z_theta,
                       double fn_bound, double sample_rate, uint64_t seed, float* tX,
                       float* ty, int32_t* tv, int32_t* tl, int64_t tcap, int64_t* tcount,
                       int32_t* labels, uint8_t* rec, oracle_learned_stats* stats,
                       int32_t stats_cap, int32_t* iters_done, double* min_margin) {
  if (n < 0 || cap < 0 || rho < 0 || guard < 0 || min_pred_degree < 1 || pred_start < 1)
    return -1;
  *iters_done = 0;
  *min_margin = INFINITY;
  if (tcount) *tcount = 0;
  if (n == 0) return 0;
  int32_t* C = labels;
  int32_t* Cn = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t* F = (uint8_t*)malloc((size_t)n);
  uint8_t* Fn = (uint8_t*)malloc((size_t)n);
  uint8_t* skip = (uint8_t*)malloc((size_t)n);
  uint8_t* pred = (uint8_t*)malloc((size_t)n);
  double* acc = (double*)calloc((size_t)n, sizeof(double));
  uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!Cn || !F || !Fn || !skip || !pred || !acc || !seen || !touched) {
    free(Cn); free(F); free(Fn); free(skip); free(pred); free(acc); free(seen); free(touched);
    return -1;
  }
  for (int64_t i = 0; i < n; ++i) {
    C[i] = (int32_t)i;
    F[i] = 1;
    memset(rec + 8 * i, 0, 8);
    rec[8 * i + 7] = 255;
  }
  int fallback = 0;
  int64_t changed_prev = -1; /* none before iteration 0 */
  int64_t nt_out = 0;
  for (int32_t l = 0; l < cap; ++l) {
    const int pl = (rho > 0) && (l % rho == 0);
    const int predict = params && !fallback && l >= pred_start;
    const int skipping = predict && (guard == 0 || l % guard != 0) &&
                         !((double)changed_prev < 2.0 * tol * (double)n);
    int64_t changed = 0, processed = 0, scanned = 0, skipped = 0, npred = 0, fneg = 0;
    /* predictions at the iteration start (the frontier) */
    for (int64_t i = 0; i < n; ++i) {
      const int64_t d = off[i + 1] - off[i];
      skip[i] = 0;
      pred[i] = 0;
      if ((prune && !F[i]) || d < min_pred_degree || d > max_pred_degree || !predict) continue;
      float f[N_IN];
      features(rec + 8 * i, l, cap, rho, f);
      const double z = mlp_logit(params, f);
      const double mg = fabs(z - z_theta);
      if (mg < *min_margin) *min_margin = mg;
      if (z < z_theta) {
        pred[i] = 1;
        ++npred;
        if (skipping) { skip[i] = 1; ++skipped; }
      }
    }
    memcpy(Cn, C, sizeof(int32_t) * (size_t)n);
    memset(Fn, 0, (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      if (prune && !F[i]) continue;
      if (skip[i]) { Fn[i] = 1; continue; } /* not processed: stays flagged */
      ++processed;
      const int64_t d = off[i + 1] - off[i];
      int64_t nt = 0;
      double K = 0.0;
      for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        ++scanned;
        const int32_t j = tgt[e];
        if ((int64_t)j == i) continue;
        const int32_t c = C[j];
        const double we = w ? (double)w[e] : 1.0;
        if (!seen[c]) { seen[c] = 1; touched[nt++] = c; acc[c] = 0.0; }
        acc[c] += we;
        K += we;
      }
      int moved = 0;
      int32_t best = -1;
      double own = 0.0, bw = 0.0, second = 0.0;
      if (nt > 0) {
        best = touched[0];
        for (int64_t t = 1; t < nt; ++t) {
          const int32_t c = touched[t];
          if (acc[c] > acc[best] || (acc[c] == acc[best] && c < best)) best = c;
        }
        bw = acc[best];
        for (int64_t t = 0; t < nt; ++t) {
          const int32_t c = touched[t];
          if (c != best && acc[c] > second) second = acc[c];
          if (c == C[i]) own = acc[c];
        }
        for (int64_t t = 0; t < nt; ++t) seen[touched[t]] = 0;
        if (best != C[i] && (!pl || best < C[i])) {
          Cn[i] = best;
          moved = 1;
          ++changed;
          for (int64_t e = off[i]; e < off[i + 1]; ++e) Fn[tgt[e]] = 1;
        }
      }
      if (pred[i] && moved) ++fneg;
      if (d < min_pred_degree || d > max_pred_degree || l < pred_start - 1) continue;
      /* trace sample (features as of the iteration start) */
      if (tX && l >= pred_start && sample_rate > 0.0 && draw(seed, l, i) < sample_rate) {
        if (nt_out < tcap) {
          features(rec + 8 * i, l, cap, rho, tX + N_IN * nt_out);
          ty[nt_out] = (float)moved;
          if (tv) tv[nt_out] = (int32_t)i;
          if (tl) tl[nt_out] = l;
        }
        ++nt_out;
      }
      /* record of this evaluation */
      uint8_t* r = rec + 8 * i;
      const float Kf = (float)K;
      const uint8_t hist = r[6] & 0x7Fu;
      const int32_t shift = r[7] == 255 ? 8 : l - (int32_t)r[7];
      const uint32_t h = (shift >= 8 ? 0u : ((uint32_t)hist << shift)) | (uint32_t)moved;
      r[0] = q255((float)own, Kf);
      r[1] = q255((float)bw - (float)second, Kf);
      r[2] = q255((float)bw - (float)own, Kf);
      r[3] = (uint8_t)((255 * (int64_t)nt) / d);
      r[4] = lq_int((uint64_t)d + 1u);
      r[5] = lq_float(1.0f + Kf);
      r[6] = (uint8_t)(h & 0x7Fu);
      r[7] = (uint8_t)(l < 254 ? l : 254);
    }
    memcpy(C, Cn, sizeof(int32_t) * (size_t)n);
    if (prune) memcpy(F, Fn, (size_t)n);
    else memset(F, 1, (size_t)n);
    if (predict && !skipping && npred > 0 && (double)fneg > fn_bound * (double)npred)
      fallback = 1;
    if (l < stats_cap) {
      oracle_learned_stats* s = &stats[l];
      s->iteration = l;
      s->pick_less = pl;
      s->changed = changed;
      s->processed = processed;
      s->edges_scanned = scanned;
      s->skipped = skipped;
      s->predicted = npred;
      s->false_neg = skipping ? 0 : fneg;
      s->skipping = skipping;
      s->fallback = fallback;
    }
    *iters_done = l + 1;
    changed_prev = changed;
    if (!pl && (double)(changed + skipped) < tol * (double)n) break;
  }
  if (tcount) *tcount = nt_out;
  free(Cn); free(F); free(Fn); free(skip); free(pred); free(acc); free(seen); free(touched);
  return 0;
}

/* The pieces, exported for the oracle's own tests. */
double oracle_mlp_logit(const float* params, const float* f) { return mlp_logit(params, f); }
int oracle_features(const uint8_t* rec, int32_t l, int32_t cap, int32_t rho, float* f) {
  features(rec, l, cap, rho, f);
  return 0;
}
int oracle_lq(uint64_t u, float x, uint8_t* out) {
  out[0] = lq_int(u);
  out[1] = lq_float(x);
  return 0;
}
double oracle_sample_draw(uint64_t seed, int32_t l, int64_t v) { return draw(seed, l, v); }
