/*
 * cpu_async.c -- CPU throughput baseline: label propagation in asynchronous
 * order on all host cores (OpenMP).  NOT the oracle: it is timed beside the
 * GPU by the benchmark (the task's CPU baseline on the host's own cores), and
 * like the oracle it is test / measurement infrastructure that the library
 * never loads.
 *
 * The method is Algorithm 1 with the GPU's asynchronous semantics: labels
 * are updated in place as soon as a vertex moves (Sec. 4 item 1), a moved
 * vertex flags its neighbours for the next iteration and a processed vertex
 * clears its own flag (Sec. 4 item 4), Pick-Less in iterations l mod rho ==
 * 0 (Sec. 4.1), Eq. 3 with ties to the smallest label, self-loops skipped,
 * stop after an iteration that is not Pick-Less with changed < tol * N, or at
 * the cap; the first iteration reads each neighbour's label as its id, the
 * value at the iteration start, as the GPU's first sweep does.  Each thread
 * sums neighbour weights into a dense per-thread array
 * indexed by label (fp32, as the GPU's tables) with a list of the labels it
 * touched, which it clears after each vertex.  Vertices are taken in dynamic
 * blocks of 1024.  Labels and flags written by other threads are read with
 * relaxed atomic loads: any interleaving is a valid asynchronous order.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int32_t ld32(const int32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
static inline void st32(int32_t* p, int32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
static inline uint8_t ld8(const uint8_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
static inline void st8(uint8_t* p, uint8_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }

/*
 * n vertices, off (n + 1 int64), tgt (int32), w (fp32 or NULL: unit).
 * labels: out (n int32).  Returns the iterations run, -1 on allocation
 * failure.  *threads: the OpenMP threads used.
 */
int32_t cpu_lpa_async_omp(int64_t n, const int64_t* off, const int32_t* tgt, const float* w,
                          double tol, int32_t cap, int32_t rho, int32_t* labels,
                          int64_t* changed_last, int32_t* threads) {
  const int T = omp_get_max_threads();
  int64_t dmax = 1;
  for (int64_t i = 0; i < n; ++i)
    if (off[i + 1] - off[i] > dmax) dmax = off[i + 1] - off[i];
  uint8_t* F = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  float** acc = (float**)calloc((size_t)T, sizeof(float*));
  uint8_t** seen = (uint8_t**)calloc((size_t)T, sizeof(uint8_t*));
  int32_t** touched = (int32_t**)calloc((size_t)T, sizeof(int32_t*));
  int failed = !F || !acc || !seen || !touched;
  if (!failed) {
#pragma omp parallel
    {
      const int t = omp_get_thread_num();
      acc[t] = (float*)calloc((size_t)(n > 0 ? n : 1), sizeof(float));
      seen[t] = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
      touched[t] = (int32_t*)malloc(sizeof(int32_t) * (size_t)dmax);
      if (!acc[t] || !seen[t] || !touched[t]) {
#pragma omp atomic write
        failed = 1;
      }
    }
  }
  int32_t iters = 0;
  *threads = T;
  *changed_last = 0;
  for (int64_t i = 0; i < n && !failed; ++i) {
    labels[i] = (int32_t)i;
    F[i] = 1;
  }
  for (int32_t l = 0; l < cap && !failed; ++l) {
    const int pl = rho > 0 && l % rho == 0;
    int64_t changed = 0;
#pragma omp parallel reduction(+ : changed)
    {
      const int t = omp_get_thread_num();
      float* a = acc[t];
      uint8_t* sn = seen[t];
      int32_t* tc = touched[t];
#pragma omp for schedule(dynamic, 1024)
      for (int64_t i = 0; i < n; ++i) {
        if (!ld8(&F[i])) continue;
        st8(&F[i], 0);
        int64_t nt = 0;
        for (int64_t e = off[i]; e < off[i + 1]; ++e) {
          const int32_t j = tgt[e];
          if ((int64_t)j == i) continue;
          /* the first iteration reads the iteration-start labels (the ids),
             as the GPU's asynchronous mode does, so that in-place reads do
             not flood the smallest ids across communities under Pick-Less */
          const int32_t c = l == 0 ? j : ld32(&labels[j]);
          if (!sn[c]) {
            sn[c] = 1;
            tc[nt++] = c;
          }
          a[c] += w ? w[e] : 1.0f;
        }
        if (nt == 0) continue;
        int32_t best = tc[0];
        for (int64_t k = 1; k < nt; ++k) {
          const int32_t c = tc[k];
          if (a[c] > a[best] || (a[c] == a[best] && c < best)) best = c;
        }
        for (int64_t k = 0; k < nt; ++k) {
          a[tc[k]] = 0.0f;
          sn[tc[k]] = 0;
        }
        const int32_t cur = ld32(&labels[i]);
        if (best != cur && (!pl || best < cur)) {
          st32(&labels[i], best);
          ++changed;
          for (int64_t e = off[i]; e < off[i + 1]; ++e) st8(&F[tgt[e]], 1);
        }
      }
    }
    iters = l + 1;
    *changed_last = changed;
    if (!pl && (double)changed < tol * (double)n) break;
  }
  for (int t = 0; t < T; ++t) {
    if (acc) free(acc[t]);
    if (seen) free(seen[t]);
    if (touched) free(touched[t]);
  }
  free(acc);
  free(seen);
  free(touched);
  free(F);
  return failed ? -1 : iters;
}
