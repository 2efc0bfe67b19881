// graph.hip -- set-up and per-iteration bookkeeping kernels around the sweep:
// validation, degree classes, initial labels and flags (Algorithm 1: every
// vertex in its own community and unprocessed), the frontier of flagged
// vertices ("for all unprocessed i ... mark i processed"), the hub slice plan,
// the deterministic-mode label apply, and fp64 modularity (Eq. 1).
#include <mutex>

#include "lpa_device.h"
#include "lpa_mlp.h"
#include "lpa_record.h"

namespace lpa {

namespace {

constexpr int kBT = 256;

__device__ __forceinline__ void set_error(DevStats* st, unsigned int bit) {
  atomicOr(&st->error, bit);
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int grid_for(int64_t n, int per_block, int cap) {
  const int64_t g = (n + per_block - 1) / per_block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

// ---- init ---------------------------------------------------------------------
__global__ void k_init(int64_t n, const int32_t* init, const int32_t* inv, int32_t* C,
                       uint8_t* F, DevStats* st) {
  // ident: every label equals its internal id, so the first sweep may take
  // a neighbour's id for its label
  if (blockIdx.x == 0 && threadIdx.x == 0) st->ident = (init || inv) ? 0 : 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = inv ? (int64_t)inv[i] : i;
    const int32_t c = init ? init[u] : (int32_t)u;
    if (c < 0 || (int64_t)c >= n) set_error(st, 4u);
    C[i] = c;
    F[i] = 1;
  }
}

hipError_t launch_init(int64_t n, const int32_t* init, const int32_t* inv, int32_t* C,
                       uint8_t* F, DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, n, init, inv, C, F,
                     st);
  return hipGetLastError();
}

// ---- run control ---------------------------------------------------------------
// k_run_begin zeroes the counters and stores the run's parameters; every
// per-iteration kernel returns at once when stop is set; k_iter_end records
// the iteration's statistics and applies the stop rule of Algorithm 1 (after
// an iteration that is not Pick-Less with changed < tolerance * N), or, in a
// batched run, stops when every graph has stopped.
__global__ void k_run_begin(DevStats* st, double tol, int cap, int rho, int batched,
                            int graphs, LearnParams lp) {
  uint32_t* w = reinterpret_cast<uint32_t*>(st);
  for (uint32_t i = threadIdx.x; i < sizeof(DevStats) / sizeof(uint32_t); i += blockDim.x)
    w[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->tol = tol;
    st->cap = cap;
    st->rho = rho;
    st->iter = 0;
    st->stop = cap <= 0 ? 1 : 0;
    st->batched = batched;
    st->graphs_left = (unsigned int)graphs;
    st->learn = lp.learn;
    st->pred_cmin = lp.cmin < 1 ? 1 : lp.cmin;
    st->pred_cmax = lp.cmax < 1 || lp.cmax >= kClassHub ? kClassHub - 1 : lp.cmax;
    st->pred_start = lp.pstart < 1 ? 1 : lp.pstart;
    st->guard = lp.guard;
    st->trace = lp.trace;
    st->z_theta = lp.z_theta;
    st->fn_bound = lp.fn_bound;
    st->trace_rate = lp.trace_rate;
    st->trace_seed = lp.trace_seed;
    st->trace_cap = lp.trace_cap;
    st->cand = 1;
  }
}

hipError_t launch_run_begin(DevStats* st, double tol, int cap, int rho, int batched,
                            int graphs, const LearnParams& lp, hipStream_t s) {
  hipLaunchKernelGGL(k_run_begin, dim3(1), dim3(256), 0, s, st, tol, cap, rho, batched, graphs,
                     lp);
  return hipGetLastError();
}

__global__ void k_arm_flags(uint8_t* F, int64_t n, const DevStats* st) {
  if (st->stop) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    F[i] = 1;
}

hipError_t launch_arm_flags(uint8_t* F, int64_t n, const DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_arm_flags, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, F, n, st);
  return hipGetLastError();
}

__global__ void k_iter_end(DevStats* st, DevIterStats* hist, int64_t n) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || st->stop) return;
  unsigned long long changed = 0, edges = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    changed += st->changed[c];
    edges += st->edges[c];
  }
  changed -= st->reverted;  // Cross-Check reverts do not count as changes
  const int l = st->iter;
  // learned skipping: a plain iteration with predictions checks the vertices
  // predicted unchanged; too many of them changing turns skipping off
  if (st->predict && !st->skipping && st->npred > 0 &&
      (double)st->fneg > st->fn_bound * (double)st->npred)
    st->fallback = 1;
  DevIterStats& h = hist[l];
  h.iteration = l;
  h.pick_less = st->pl;
  h.changed = (long long)changed;
  h.processed = (long long)st->processed;
  h.edges = (long long)edges;
  h.skipped = (long long)st->skipped;
  h.npred = (long long)st->npred;
  h.fneg = st->skipping ? 0ll : (long long)st->fneg;
  h.skipping = st->skipping;
  h.fallback = st->fallback;
  int stop = 0;
  if (st->batched) stop = st->graphs_left == 0u;
  // Algorithm 1's test on changed + skipped: the skipped vertices bound what
  // a plain sweep of this iteration could have changed in addition
  else stop = !st->pl && (double)(changed + st->skipped) < st->tol * (double)n;
  // near the stop (changed < 2 tol N) the next iteration is a plain sweep
  st->cand = (double)changed < 2.0 * st->tol * (double)n ? 1 : 0;
  st->iter = l + 1;
  st->stop = (stop || l + 1 >= st->cap) ? 1 : 0;
}

hipError_t launch_iter_end(DevStats* st, DevIterStats* hist, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, s, st, hist, n);
  return hipGetLastError();
}

// ---- batched runs: per-graph stop rule ------------------------------------------
// One workgroup per graph: count the graph's changed vertices, apply Algorithm
// 1's stop test with the graph's own vertex count, and clear the flags of a
// graph that stops so that none of its vertices is processed again.  All
// graphs share the iteration counter, so each follows its solo schedule.
__global__ __launch_bounds__(kBT) void k_batch_step(BatchArgs b, const uint8_t* chg,
                                                    uint8_t* F, DevStats* st) {
  __shared__ unsigned int cnt[kBT / 64];
  __shared__ int fin;
  if (st->stop) return;
  for (int32_t g = blockIdx.x; g < b.G; g += gridDim.x) {
    if (b.done[g]) continue;
    const int64_t v0 = b.v_off[g], v1 = b.v_off[g + 1];
    unsigned int c = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += kBT) c += chg[v];
    for (int ofs = 32; ofs > 0; ofs >>= 1) c += __shfl_xor(c, ofs);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int q = 0; q < kBT / 64; ++q) t += cnt[q];
      b.changed_last[g] = (long long)t;
      const int l = st->iter;
      const bool f = (!st->pl && (double)t < st->tol * (double)(v1 - v0)) || l + 1 >= st->cap;
      if (f) {
        b.done[g] = 1;
        b.iters[g] = l + 1;
      } else {
        atomicAdd(&st->graphs_left, 1u);
      }
      fin = f;
    }
    __syncthreads();
    if (fin)
      for (int64_t v = v0 + threadIdx.x; v < v1; v += kBT) F[v] = 0;
    __syncthreads();
  }
}

hipError_t launch_batch_step(const BatchArgs& b, const uint8_t* chg, uint8_t* F, DevStats* st,
                             hipStream_t s) {
  const int g = b.G < 8192 ? (b.G > 0 ? b.G : 1) : 8192;
  hipLaunchKernelGGL(k_batch_step, dim3(g), dim3(kBT), 0, s, b, chg, F, st);
  return hipGetLastError();
}

__global__ void k_batch_reset(BatchArgs b) {
  for (int32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < b.G; g += gridDim.x * blockDim.x) {
    b.done[g] = b.v_off[g + 1] == b.v_off[g];  // an empty graph performs no iteration
    b.iters[g] = 0;
    b.changed_last[g] = 0;
  }
}

hipError_t launch_batch_reset(const BatchArgs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(grid_for(b.G, kBT, 1024)), dim3(kBT), 0, s, b);
  return hipGetLastError();
}

// every CSR entry of graph g must point into graph g (error bit 16)
template <typename OffT>
__global__ void k_batch_validate(const OffT* off, const int32_t* tgt, BatchArgs b, int64_t n,
                                 DevStats* st) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = b.G - 1;  // graph holding v: largest g with v_off[g] <= v
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (b.v_off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    const int64_t a0 = b.v_off[lo], a1 = b.v_off[lo + 1];
    for (int64_t e = (int64_t)off[v]; e < (int64_t)off[v + 1]; ++e)
      if ((int64_t)tgt[e] < a0 || (int64_t)tgt[e] >= a1) {
        set_error(st, 16u);
        break;
      }
  }
}

hipError_t launch_batch_validate(bool off64, const void* off, const int32_t* tgt,
                                 const BatchArgs& b, int64_t n, DevStats* st, hipStream_t s) {
  const int g = grid_for(n, kBT, 8192);
  if (off64)
    hipLaunchKernelGGL(k_batch_validate<int64_t>, dim3(g), dim3(kBT), 0, s,
                       (const int64_t*)off, tgt, b, n, st);
  else
    hipLaunchKernelGGL(k_batch_validate<int32_t>, dim3(g), dim3(kBT), 0, s,
                       (const int32_t*)off, tgt, b, n, st);
  return hipGetLastError();
}

// ---- validation (error bits: 1 offsets, 2 targets, 8 weights) ----------------
template <typename OffT>
__global__ void k_validate(const OffT* off, const int32_t* tgt, const float* w,
                           int64_t n, int64_t m, DevStats* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t0 == 0 && ((int64_t)off[0] != 0 || (int64_t)off[n] != m)) set_error(st, 1u);
  for (int64_t i = t0; i < n; i += stride)
    if (off[i] > off[i + 1]) set_error(st, 1u);
  for (int64_t e = t0; e < m; e += stride) {
    const int32_t j = tgt[e];
    if (j < 0 || (int64_t)j >= n) set_error(st, 2u);
    if (w) {
      const uint32_t b = __float_as_uint(w[e]);
      // reject negative (sign bit set, including -0.0), infinities and NaN
      if ((b >> 31) || ((b >> 23) & 0xFFu) == 0xFFu) set_error(st, 8u);
    }
  }
}

hipError_t launch_validate(bool off64, const void* off, const int32_t* tgt,
                           const float* w, int64_t n, int64_t m, DevStats* st,
                           hipStream_t s) {
  const int g = grid_for(m > n ? m : n, kBT, 8192);
  if (off64)
    hipLaunchKernelGGL(k_validate<int64_t>, dim3(g), dim3(kBT), 0, s,
                       (const int64_t*)off, tgt, w, n, m, st);
  else
    hipLaunchKernelGGL(k_validate<int32_t>, dim3(g), dim3(kBT), 0, s,
                       (const int32_t*)off, tgt, w, n, m, st);
  return hipGetLastError();
}

// Any weight other than 1.0f: *other receives 1 (else the weights are unit
// weights, and the kernels need not read them).
__global__ void k_unit_weights(const float* w, int64_t m, unsigned int* other) {
  bool any = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x)
    any |= __float_as_uint(__builtin_nontemporal_load(&w[e])) != 0x3F800000u;
  if (__any(any) && (threadIdx.x & 63) == 0) *other = 1u;
}

hipError_t launch_unit_weights(const float* w, int64_t m, unsigned int* other, hipStream_t s) {
  hipError_t e = launch_fill_u32(other, 0u, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unit_weights, dim3(grid_for(m, kBT, 8192)), dim3(kBT), 0, s, w, m, other);
  return hipGetLastError();
}

// Rows with strictly increasing targets (sorted, no repeated neighbour):
// mark the first entry of every non-empty row, then flag any entry whose
// successor in the same row is not larger.  bad receives 1 on a violation.
template <typename OffT>
__global__ void k_mark_row_starts(const OffT* off, int64_t n, uint8_t* mark) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (off[i] < off[i + 1]) mark[off[i]] = 1;
}

__global__ void k_rows_strict(const int32_t* tgt, const uint8_t* mark, int64_t m,
                              unsigned int* bad) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e + 1 < m;
       e += (int64_t)gridDim.x * blockDim.x)
    if (!mark[e + 1] && tgt[e] >= tgt[e + 1]) *bad = 1u;
}

hipError_t launch_rows_strict(bool off64, const void* off, const int32_t* tgt, int64_t n,
                              int64_t m, uint8_t* mark, unsigned int* bad, hipStream_t s) {
  hipError_t e = launch_fill_u8(mark, 0, m, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(bad, 0u, 1, s);
  if (e != hipSuccess) return e;
  if (off64)
    hipLaunchKernelGGL(k_mark_row_starts<int64_t>, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0,
                       s, (const int64_t*)off, n, mark);
  else
    hipLaunchKernelGGL(k_mark_row_starts<int32_t>, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0,
                       s, (const int32_t*)off, n, mark);
  hipLaunchKernelGGL(k_rows_strict, dim3(grid_for(m, kBT, 16384)), dim3(kBT), 0, s, tgt, mark, m,
                     bad);
  return hipGetLastError();
}

// Label-read probe: one pass that only reads every CSR entry's target and
// its neighbour's label, in the order the sweep kernels read them (8 entries
// in flight per lane).  Its rate bounds any sweep that must read them.
__global__ __launch_bounds__(256) void k_label_read_probe(const int32_t* tgt, int64_t m,
                                                          const int32_t* C, uint32_t* sink) {
  constexpr int U = 8;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t T = (int64_t)gridDim.x * 256;
  uint32_t acc = 0;
  int64_t e = t;
  for (; e + (U - 1) * T < m; e += U * T) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = __builtin_nontemporal_load(&tgt[e + u * T]);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (uint32_t)C[j[u]];
  }
  for (; e < m; e += T) acc += (uint32_t)C[__builtin_nontemporal_load(&tgt[e])];
  sink[t] = acc;
}

hipError_t launch_label_read_probe(const int32_t* tgt, int64_t m, const int32_t* C,
                                   uint32_t* sink, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_label_read_probe, dim3(grid), dim3(256), 0, s, tgt, m, C, sink);
  return hipGetLastError();
}

__global__ void k_check_labels(int64_t n, const int32_t* lab, DevStats* st) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (lab[i] < 0 || (int64_t)lab[i] >= n) set_error(st, 4u);
}

hipError_t launch_check_labels(int64_t n, const int32_t* lab, DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_check_labels, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, n, lab, st);
  return hipGetLastError();
}

// ---- degree classes -------------------------------------------------------------
struct Bounds { int32_t hi[kNumClasses]; };

template <typename OffT>
__global__ void k_classify(const OffT* off, int64_t n, Bounds b, uint8_t* cls,
                           unsigned long long* counts, int32_t* hub_out,
                           unsigned int* hub_count) {
  __shared__ unsigned int cnt[kNumClasses];
  if (threadIdx.x < kNumClasses) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
    int c = kClassHub;
    if (d == 0) {
      c = 0;
    } else {
      for (int q = 1; q < kClassHub; ++q)
        if (d <= b.hi[q]) { c = q; break; }
    }
    cls[v] = (uint8_t)c;
    atomicAdd(&cnt[c], 1u);
    if (c == kClassHub) hub_out[atomicAdd(hub_count, 1u)] = (int32_t)v;
  }
  __syncthreads();
  if (threadIdx.x < kNumClasses && cnt[threadIdx.x])
    atomicAdd(&counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

hipError_t launch_classify(bool off64, const void* off, int64_t n, const int32_t* bounds,
                           uint8_t* cls, unsigned long long* counts, int32_t* hub_out,
                           unsigned int* hub_count, hipStream_t s) {
  Bounds b;
  for (int q = 0; q < kNumClasses; ++q) b.hi[q] = bounds[q];
  const int g = grid_for(n, kBT, 8192);
  if (off64)
    hipLaunchKernelGGL(k_classify<int64_t>, dim3(g), dim3(kBT), 0, s, (const int64_t*)off,
                       n, b, cls, counts, hub_out, hub_count);
  else
    hipLaunchKernelGGL(k_classify<int32_t>, dim3(g), dim3(kBT), 0, s, (const int32_t*)off,
                       n, b, cls, counts, hub_out, hub_count);
  return hipGetLastError();
}

template <typename OffT>
__global__ void k_gather_degrees(const OffT* off, const int32_t* vids, int32_t h, int64_t* deg) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < h; i += gridDim.x * blockDim.x)
    deg[i] = (int64_t)off[vids[i] + 1] - (int64_t)off[vids[i]];
}

hipError_t launch_gather_degrees(bool off64, const void* off, const int32_t* vids, int32_t h,
                                 int64_t* deg, hipStream_t s) {
  const int g = grid_for(h, kBT, 4096);
  if (off64)
    hipLaunchKernelGGL(k_gather_degrees<int64_t>, dim3(g), dim3(kBT), 0, s, (const int64_t*)off, vids, h, deg);
  else
    hipLaunchKernelGGL(k_gather_degrees<int32_t>, dim3(g), dim3(kBT), 0, s, (const int32_t*)off, vids, h, deg);
  return hipGetLastError();
}

// Position of each hub slice's middle entry in the id order by entry mass:
// the row offset of its target (the entries of all rows before it).  Slices
// are listed as (hub index, slice index) pairs.
template <typename OffT>
__global__ void k_slice_keys(const OffT* off, const int32_t* tgt, const int32_t* hub_vid,
                             const uint32_t* sl, int64_t ns, int chunk, int64_t* key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int32_t v = hub_vid[sl[2 * i]];
  const int64_t c = sl[2 * i + 1];
  const int64_t o = (int64_t)off[v], d = (int64_t)off[v + 1] - o;
  const int64_t e0 = c * chunk;
  const int64_t n = d - e0 < chunk ? d - e0 : chunk;
  key[i] = (int64_t)off[tgt[o + e0 + n / 2]];
}

hipError_t launch_slice_keys(bool off64, const void* off, const int32_t* tgt,
                             const int32_t* hub_vid, const uint32_t* sl, int64_t ns, int chunk,
                             int64_t* key, hipStream_t s) {
  const int g = grid_for(ns, kBT, 1 << 20);
  if (off64)
    hipLaunchKernelGGL(k_slice_keys<int64_t>, dim3(g), dim3(kBT), 0, s, (const int64_t*)off, tgt,
                       hub_vid, sl, ns, chunk, key);
  else
    hipLaunchKernelGGL(k_slice_keys<int32_t>, dim3(g), dim3(kBT), 0, s, (const int32_t*)off, tgt,
                       hub_vid, sl, ns, chunk, key);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(count, kBT, 8192)), dim3(kBT), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(count, kBT, 8192)), dim3(kBT), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(count, kBT, 8192)), dim3(kBT), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(count, kBT, 8192)), dim3(kBT), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t count,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(grid_for(count, kBT, 8192)), dim3(kBT), 0,
                     s, p, v, count);
  return hipGetLastError();
}

// ---- hub plan: reset the iteration counters, take the flagged hubs, queue
// their slices and their label buckets.  One workgroup of 1024 threads. -------
template <typename OffT>
__global__ __launch_bounds__(1024) void k_hub_plan(HubArgs a, int32_t* C, uint8_t* F) {
  __shared__ uint32_t ws[16], wb[16];
  __shared__ uint32_t run_s, run_b;
  __shared__ uint32_t nproc;
  const int tid = threadIdx.x;
  DevStats* st = a.st;
  if (st->stop) return;
  if (tid == 0) {
    st->processed = 0; st->pending = 0;
    st->pull_scanned = 0; st->pull_mode = 0;
    st->hub_pairs = 0;
    st->reverted = 0;
    st->graphs_left = 0;
    // Pick-Less in iterations l with l mod rho == 0, counting from 0
    st->pl = (st->rho > 0 && st->iter % st->rho == 0) ? 1 : 0;
    // learned skipping: predictions from iteration 1 on until a fallback;
    // skip unless this is a guard iteration or the last one changed few
    const int l = st->iter;
    st->predict = (st->learn && !st->fallback && l >= st->pred_start) ? 1 : 0;
    st->skipping = (st->predict && (st->guard == 0 || l % st->guard != 0) && !st->cand) ? 1 : 0;
    st->skipped = 0; st->npred = 0; st->fneg = 0;
    st->trace_first = st->trace_n;
    run_s = 0; run_b = 0; nproc = 0;
  }
  if (tid < kNumClasses) {
    st->active[tid] = 0;
    st->edges[tid] = 0;
    st->changed[tid] = 0;
    st->flagw[tid] = 0;
  }
  if (a.witems && tid < kXcds) a.wctr[tid * kQueueCtrStride] = 0u;
  __syncthreads();
  const OffT* off = reinterpret_cast<const OffT*>(a.off);
  // each hub's slice count (0 unless flagged), kB tiles of 1024 hubs at a
  // time, so that the dependent loads of kB hubs per thread (hub vertex, its
  // flag, its row offsets) are in flight together; thread tid takes hubs
  // tid mod 1024 in both passes and reads back only what it wrote
  constexpr int kB = 4;
  for (int32_t t0 = 0; t0 < a.H; t0 += 1024 * kB) {
    int32_t hv[kB];
    uint8_t hf[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int32_t h = t0 + q * 1024 + tid;
      hv[q] = h < a.H ? a.hub_vid[h] : -1;
    }
#pragma unroll
    for (int q = 0; q < kB; ++q) hf[q] = hv[q] >= 0 ? F[hv[q]] : (uint8_t)0;
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int32_t h = t0 + q * 1024 + tid;
      if (h >= a.H) continue;
      const int32_t v = hv[q];
      a.hub_best[h] = 0ull;
      a.hub_ovf[h] = 0;
      uint32_t nch = 0;
      if (hf[q]) {
        F[v] = 0;
        a.hub_old[h] = C[v];
        const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
        nch = (uint32_t)((d + a.chunk - 1) / a.chunk);
        atomicAdd(&nproc, 1u);
      }
      a.hub_nch[h] = (int32_t)nch;
    }
  }
  // queue the flagged hubs' slices and buckets: a scan of both counts over
  // each tile of 1024 hubs (within each wave by shuffles, then over the
  // waves' totals); the next tile's counts are loaded during this one's
  const int lane = tid & 63, wv = tid >> 6;
  uint32_t rs = 0, rb = 0;  // slices and buckets queued by earlier tiles
  int32_t nch_n = tid < a.H ? a.hub_nch[tid] : 0;
  int32_t lgb_n = tid < a.H ? a.hub_lgb[tid] : 0;
  for (int32_t tile = 0; tile < a.H; tile += 1024) {
    const int32_t h = tile + tid;
    const uint32_t nch = (uint32_t)nch_n;
    const uint32_t nbk = nch ? 1u << lgb_n : 0u;
    if (h + 1024 < a.H) {
      nch_n = a.hub_nch[h + 1024];
      lgb_n = a.hub_lgb[h + 1024];
    } else {
      nch_n = 0;
      lgb_n = 0;
    }
    uint32_t xs = nch, xb = nbk;  // inclusive scans within the wave
#pragma unroll
    for (int ofs = 1; ofs < 64; ofs <<= 1) {
      const uint32_t ys = __shfl_up(xs, ofs), yb = __shfl_up(xb, ofs);
      if (lane >= ofs) {
        xs += ys;
        xb += yb;
      }
    }
    if (lane == 63) {
      ws[wv] = xs;
      wb[wv] = xb;
    }
    __syncthreads();
    uint32_t bs = 0, bb = 0, ts = 0, tb = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      if (w < wv) {
        bs += ws[w];
        bb += wb[w];
      }
      ts += ws[w];
      tb += wb[w];
    }
    const uint32_t fs = rs + bs + xs - nch;
    const uint32_t fb = rb + bb + xb - nbk;
    for (uint32_t c = 0; c < nch; ++c) {
      a.items[2 * (uint64_t)(fs + c)] = (uint32_t)h;
      a.items[2 * (uint64_t)(fs + c) + 1] = c;
    }
    for (uint32_t b = 0; b < nbk; ++b) {
      a.bitems[2 * (uint64_t)(fb + b)] = (uint32_t)h;
      a.bitems[2 * (uint64_t)(fb + b) + 1] = b;
      a.bsize[fb + b] = 0u;
    }
    if (nbk) a.hub_bq[h] = (int32_t)fb;
    rs += ts;
    rb += tb;
    __syncthreads();  // ws and wb are rewritten by the next tile
  }
  if (tid == 0) {
    run_s = rs;
    run_b = rb;
  }
  __syncthreads();
  if (tid == 0) {
    st->hub_items = run_s;
    st->hub_bitems = run_b;
    st->processed = nproc;
    st->hub_all = (int32_t)nproc == a.H ? 1u : 0u;
  }
}

hipError_t launch_hub_plan(bool off64, const HubArgs& a, int32_t* C, uint8_t* F,
                           hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_hub_plan<int64_t>, dim3(1), dim3(1024), 0, s, a, C, F);
  else
    hipLaunchKernelGGL(k_hub_plan<int32_t>, dim3(1), dim3(1024), 0, s, a, C, F);
  return hipGetLastError();
}

// ---- frontier: append flagged vertices to their class list, clear flags ------
struct ListPtrs { int32_t* p[kNumClasses]; };

__global__ __launch_bounds__(kBT) void k_frontier(int64_t n_all, int64_t n_later, uint8_t* F,
                                                  const uint8_t* cls, ListPtrs lists,
                                                  uint8_t* chg_clear, DevStats* st) {
  // kWords words of four vertices per thread and block step: the block's
  // appends cost one global atomic per class and step
  constexpr int kWords = 8;
  constexpr int64_t kStep = (int64_t)kBT * kWords * 4;
  __shared__ uint32_t cnt[kNumClasses];
  __shared__ uint32_t base[kNumClasses];
  if (st->stop) return;
  // vertices scanned: all in the first iteration, then n_later (the
  // vertices of degree 0, last in the internal order, are flagged only by
  // the initialisation)
  const int64_t n = st->iter == 0 ? n_all : n_later;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t proc = 0;
  for (int64_t chunk = (int64_t)blockIdx.x * kStep; chunk < n; chunk += (int64_t)gridDim.x * kStep) {
    if (tid < kNumClasses) cnt[tid] = 0;
    __syncthreads();
    // word k of this thread holds vertices v0[k] .. v0[k] + 3 (coalesced)
    int64_t v0[kWords];
    uint32_t f4[kWords], c4[kWords];
#pragma unroll
    for (int k = 0; k < kWords; ++k) {
      v0[k] = chunk + ((int64_t)k * kBT + tid) * 4;
      f4[k] = 0u;
      c4[k] = 0u;
      if (v0[k] + 3 < n) {
        f4[k] = *reinterpret_cast<const uint32_t*>(F + v0[k]);
        c4[k] = *reinterpret_cast<const uint32_t*>(cls + v0[k]);
        *reinterpret_cast<uint32_t*>(chg_clear + v0[k]) = 0u;
        if (f4[k]) *reinterpret_cast<uint32_t*>(F + v0[k]) = 0u;
      } else {
        for (int q = 0; q < 4 && v0[k] + q < n; ++q) {
          f4[k] |= (uint32_t)F[v0[k] + q] << (8 * q);
          c4[k] |= (uint32_t)cls[v0[k] + q] << (8 * q);
          chg_clear[v0[k] + q] = 0;
          F[v0[k] + q] = 0;
        }
      }
    }
    int8_t cq[kWords][4];
    uint32_t pos[kWords][4];
#pragma unroll
    for (int k = 0; k < kWords; ++k) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool f = ((f4[k] >> (8 * q)) & 0xFFu) != 0u;
        const int c = (int)((c4[k] >> (8 * q)) & 0xFFu);
        proc += f ? 1u : 0u;
        const int8_t cc0 = (f && c != 0 && c != kClassHub) ? (int8_t)c : (int8_t)-1;
        cq[k][q] = cc0;
        pos[k][q] = 0u;
        // one LDS atomic per class present in the wave
        unsigned long long left = __ballot(cc0 >= 0);
        while (left) {
          const int src = __ffsll((long long)left) - 1;
          const int cc = __shfl((int)cc0, src);
          const unsigned long long m = __ballot(cc0 == cc);
          uint32_t b = 0;
          if (lane == src) b = atomicAdd(&cnt[cc], (uint32_t)__popcll(m));
          b = __shfl(b, src);
          if (cc0 == cc) pos[k][q] = b + (uint32_t)__popcll(m & lt);
          left &= ~m;
        }
      }
    }
    __syncthreads();
    if (tid < kNumClasses) base[tid] = cnt[tid] ? atomicAdd(&st->active[tid], cnt[tid]) : 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kWords; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (cq[k][q] >= 0)
          lists.p[cq[k][q]][base[cq[k][q]] + pos[k][q]] = (int32_t)(v0[k] + q);
    __syncthreads();
  }
  // one atomic per workgroup for the processed count (cnt is free after the
  // last step's barrier; every thread of the workgroup gets here)
  uint32_t x = proc;
  for (int ofs = 32; ofs > 0; ofs >>= 1) x += __shfl_xor(x, ofs);
  if ((tid & 63) == 0) cnt[tid >> 6] = x;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (int q = 0; q < kBT / 64; ++q) t += cnt[q];
    if (t) atomicAdd(&st->processed, (unsigned long long)t);
  }
}

hipError_t launch_frontier(int64_t n, int64_t n_later, uint8_t* F, const uint8_t* cls,
                           int32_t* const* lists, uint8_t* chg_clear, DevStats* st, int grid,
                           hipStream_t s) {
  ListPtrs lp;
  for (int q = 0; q < kNumClasses; ++q) lp.p[q] = lists[q];
  hipLaunchKernelGGL(k_frontier, dim3(grid), dim3(kBT), 0, s, n, n_later, F, cls, lp, chg_clear,
                     st);
  return hipGetLastError();
}

// ---- frontier with the change predictor (learned variant) ------------------------
// One wave per 64 consecutive vertices.  The flagged vertices of classes 1..8
// are compacted within the wave and, when this iteration predicts, run through
// the network 16 at a time (one MFMA tile of samples, operands held in
// registers for the whole kernel).  In a skipping iteration a vertex whose
// logit is below z_theta keeps its flag and is not listed; in a plain one it
// is listed and marked (record byte 6, bit 7) so that the sweep counts it if
// it changes.  Trace samples (features of a listed vertex) are appended here;
// their targets are filled in after the sweep.
namespace {

__device__ __forceinline__ double sample_draw(unsigned long long seed, int l, int64_t v) {
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull *
                                    (1ull + (((unsigned long long)(uint32_t)l << 32) |
                                             (unsigned long long)v));
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

constexpr int kLearnWaves = 4;
constexpr int kLearnChunks = 4;  // 64-vertex chunks per wave and block step

__global__ __launch_bounds__(kLearnWaves * 64) void k_frontier_learned(
    int64_t n_all, int64_t n_later, uint8_t* F, const uint8_t* cls, ListPtrs lists,
    uint8_t* chg_clear, DevStats* st, unsigned long long* rec, const MlpTiles* tiles,
    TraceArgs tr) {
  __shared__ uint8_t lst_all[kLearnWaves][64];
  __shared__ uint8_t dec_all[kLearnWaves][64];
  __shared__ unsigned long long slot_all[kLearnWaves][16];
  __shared__ uint32_t cnt[kNumClasses];
  __shared__ uint32_t cbase[kNumClasses];
  // the network's operand tiles, read from LDS at each use: held in
  // registers they would leave room for two waves per SIMD
  __shared__ MlpTiles wl;
  if (st->stop) return;
  const int64_t n = st->iter == 0 ? n_all : n_later;  // as in k_frontier
  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  uint8_t* lst = lst_all[wv];
  uint8_t* dec = dec_all[wv];
  unsigned long long* slot = slot_all[wv];
  const int l = st->iter;
  const int cap = st->cap, rho = st->rho;
  const bool predict = st->predict != 0;
  const bool skipping = st->skipping != 0;
  // rows of other classes are never predicted or traced
  const int cmin = st->pred_cmin, cmax = st->pred_cmax;
  const bool tracing = st->trace != 0 && l >= st->pred_start && tr.X != nullptr;
  const float z_theta = st->z_theta;
  const double rate = st->trace_rate;
  const unsigned long long seed = st->trace_seed, tcap = st->trace_cap;
  if (predict) {
    static_assert(sizeof(MlpTiles) % 4 == 0, "tiles are copied as words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(tiles);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&wl);
    for (int q = tid; q < (int)(sizeof(MlpTiles) / 4); q += kLearnWaves * 64) dst[q] = src[q];
  }
  __syncthreads();
  const MlpFromTiles W{wl, lane, g};
  uint32_t proc = 0, skipped = 0, npred = 0;
  constexpr int64_t kStep = (int64_t)kLearnWaves * kLearnChunks * 64;
  // the whole workgroup walks the same steps of kStep vertices (barriers
  // inside); the listed vertices of a step are appended with one atomic per
  // class and workgroup, as in the plain frontier
  for (int64_t step0 = (int64_t)blockIdx.x * kStep; step0 < n;
       step0 += (int64_t)gridDim.x * kStep) {
    if (tid < kNumClasses) cnt[tid] = 0;
    __syncthreads();
    int8_t cq[kLearnChunks];
    uint32_t pos[kLearnChunks];
    // flags, classes and records of the wave's chunks, loaded together (the
    // records of listed vertices reach their tile lanes by shuffles)
    uint8_t fq[kLearnChunks], cl[kLearnChunks];
    unsigned long long rq[kLearnChunks];
#pragma unroll
    for (int q = 0; q < kLearnChunks; ++q) {
      const int64_t v = step0 + ((int64_t)wv * kLearnChunks + q) * 64 + lane;
      fq[q] = 0;
      cl[q] = 0;
      rq[q] = kRecordInit;
      if (v < n) {
        fq[q] = F[v];
        cl[q] = cls[v];
        if (predict || tracing) rq[q] = rec[v];
        chg_clear[v] = 0;
      }
    }
#pragma unroll
    for (int q = 0; q < kLearnChunks; ++q) {
      const int64_t base = step0 + ((int64_t)wv * kLearnChunks + q) * 64;
      const int64_t v = base + lane;
      const uint8_t f = fq[q], c = cl[q];
      const bool cand = f && c >= cmin && c <= cmax && (predict || tracing);
      const unsigned long long cm = __ballot(cand);
      const uint32_t ncand = __popcll(cm);
      if (cand) lst[lane_rank(cm)] = (uint8_t)lane;
      dec[lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (uint32_t r0 = 0; r0 < ncand; r0 += 16) {  // uniform trip count
        const uint32_t si = r0 + (uint32_t)(lane & 15);
        const bool has = si < ncand;
        const int src = has ? lst[si] : 0;
        const int64_t u = base + src;
        const uint32_t rlo = (uint32_t)__shfl((int)(uint32_t)rq[q], src);
        const uint32_t rhi = (uint32_t)__shfl((int)(uint32_t)(rq[q] >> 32), src);
        const unsigned long long rr =
            has ? (((unsigned long long)rhi << 32) | rlo) : kRecordInit;
        float x[4];
        rec_features(rr, l, cap, rho, g, x);
        bool pred = false;
        if (predict) {
          const float z = mlp_logit16_src(W, x);
          pred = has && z < z_theta;
        }
        const bool skip = pred && skipping;
        if (lane < 16 && has) dec[src] = (uint8_t)((pred ? 1 : 0) | (skip ? 2 : 0));
        if (tracing) {
          const int64_t uid = tr.inv ? (int64_t)tr.inv[u] : u;  // the caller's id
          const bool take = has && !skip && sample_draw(seed, l, uid) < rate;
          if (lane < 16) slot[lane] = take ? atomicAdd(&st->trace_n, 1ull) : ~0ull;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          const unsigned long long qq = slot[lane & 15];
          if (take && qq < tcap && g < 3) {
#pragma unroll
            for (int j = 0; j < 4; ++j) tr.X[qq * kMlpIn + 4 * g + j] = x[j];
            if (g == 0) {
              tr.v[qq] = (int32_t)uid;
              tr.l[qq] = l;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      const uint8_t dd = dec[lane];
      const bool skip = (dd & 2) != 0;
      const bool keep = f && !skip;
      if (dd & 1) {
        ++npred;
        // plain iteration: mark for the false-negative count of the sweep
        if (!skip) rec[v] = rq[q] | (0x80ull << 48);
      }
      if (skip) ++skipped;
      cq[q] = -1;
      if (keep) {
        F[v] = 0;
        ++proc;
        if (c >= 1 && c < kClassHub) {
          cq[q] = (int8_t)c;
          pos[q] = atomicAdd(&cnt[c], 1u);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    __syncthreads();
    if (tid < kNumClasses) cbase[tid] = cnt[tid] ? atomicAdd(&st->active[tid], cnt[tid]) : 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kLearnChunks; ++q)
      if (cq[q] >= 0)
        lists.p[cq[q]][cbase[cq[q]] + pos[q]] =
            (int32_t)(step0 + ((int64_t)wv * kLearnChunks + q) * 64 + lane);
    __syncthreads();
  }
  // one atomic per counter and workgroup (cnt and cbase are free after the
  // last step's barrier; every thread of the workgroup gets here)
  const uint32_t tp = wave_sum_u32(proc), ts = wave_sum_u32(skipped), tn = wave_sum_u32(npred);
  if (lane == 0) {
    cnt[wv] = tp;
    cnt[kLearnWaves + wv] = ts;
    cbase[wv] = tn;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t sp = 0, ss = 0, sn = 0;
    for (int q = 0; q < kLearnWaves; ++q) {
      sp += cnt[q];
      ss += cnt[kLearnWaves + q];
      sn += cbase[q];
    }
    if (sp) atomicAdd(&st->processed, (unsigned long long)sp);
    if (ss) atomicAdd(&st->skipped, (unsigned long long)ss);
    if (sn) atomicAdd(&st->npred, (unsigned long long)sn);
  }
}

hipError_t launch_frontier_learned(int64_t n, int64_t n_later, uint8_t* F, const uint8_t* cls,
                                   int32_t* const* lists, uint8_t* chg_clear, DevStats* st,
                                   unsigned long long* rec, const MlpTiles* tiles,
                                   const TraceArgs& tr, int grid, hipStream_t s) {
  ListPtrs lp;
  for (int q = 0; q < kNumClasses; ++q) lp.p[q] = lists[q];
  hipLaunchKernelGGL(k_frontier_learned, dim3(grid), dim3(kLearnWaves * 64), 0, s, n, n_later,
                     F, cls, lp, chg_clear, st, rec, tiles, tr);
  return hipGetLastError();
}

// Targets of this iteration's trace samples: 1 if the vertex changed label.
__global__ void k_trace_label(const DevStats* st, const uint8_t* chg, TraceArgs tr) {
  if (st->stop || !st->trace) return;
  const unsigned long long end = st->trace_n < st->trace_cap ? st->trace_n : st->trace_cap;
  for (unsigned long long i = st->trace_first + blockIdx.x * (unsigned long long)blockDim.x +
                              threadIdx.x;
       i < end; i += (unsigned long long)gridDim.x * blockDim.x)
    tr.y[i] = chg[tr.perm ? tr.perm[tr.v[i]] : tr.v[i]] ? 1.0f : 0.0f;
}

hipError_t launch_trace_label(const DevStats* st, const uint8_t* chg, const TraceArgs& tr,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_trace_label, dim3(256), dim3(256), 0, s, st, chg, tr);
  return hipGetLastError();
}

// ---- neighbour flags ------------------------------------------------------------
// The sweep records each changed vertex in chg.  Every CSR neighbour of a
// changed vertex is then flagged for the next iteration (Sec. 4 item 4), in
// one of two equivalent ways on a symmetric CSR:
//   push: each changed vertex writes the flag byte of each neighbour;
//   pull: each vertex reads the change bytes of its neighbours and stops at
//         the first changed one.
// Push costs one scattered byte store (a line's read-modify-write) per entry
// of a changed row; pull costs a read per entry up to the first changed
// neighbour, about 1/p entries per vertex when the changed rows hold a share
// p of the entries.  On R-MAT scale 26 the two cost the same near p = 1/16
// (push of a quarter of the entries: 18.6 ms; pull at p near 1/2: 2.7 ms), so
// k_flag_decide picks pull when the changed rows hold at least 1/pdiv of the
// CSR entries (lpa_tuning.pull_divisor, default 16), push otherwise; the
// kernels of the other way return at once.
__global__ void k_flag_decide(DevStats* st, int64_t m, int64_t n, int force, int pdiv) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || st->stop) return;
  unsigned long long fw = 0, changed = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    fw += st->flagw[c];
    changed += st->changed[c];
  }
  changed -= st->reverted;
  // the run stops after this iteration (k_iter_end's test, same operands):
  // its flags matter only to a later lpa_get_flags, which sets them then
  if (!st->batched) {
    const bool last = (!st->pl && (double)(changed + st->skipped) < st->tol * (double)n) ||
                      st->iter + 1 >= st->cap;
    if (last) {
      st->pull_mode = 2u;
      st->flags_deferred = 1u;
      return;
    }
  }
  st->pull_mode = force == 2   ? 1u
                  : force == 1 ? 0u
                               : ((unsigned long long)pdiv * fw >= (unsigned long long)m ? 1u : 0u);
}

hipError_t launch_flag_decide(DevStats* st, int64_t m, int64_t n, int force, int pdiv,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_flag_decide, dim3(1), dim3(64), 0, s, st, m, n, force, pdiv);
  return hipGetLastError();
}

// ---- Cross-Check (Sec. 4.1) ---------------------------------------------------
__global__ void k_cc_save(const int32_t* C, int32_t* Cp, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    Cp[i] = C[i];
}

// One round of revert decisions.  A changed vertex (caller id u, new label c)
// reverts when vertex c, at its place in id order, does not hold label c:
// for c < u that is c's final label (its previous label if it reverts), for
// c > u its new label.  The decisions depend only on those of smaller ids, so
// repeating rounds until none changes reaches the id-order result.
__global__ void k_cc_round(const int32_t* C, const int32_t* Cp, const uint8_t* chg, uint8_t* R,
                           const int32_t* perm, const int32_t* inv, int64_t n, DevStats* st) {
  bool moved = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!chg[i]) continue;
    const int32_t c = C[i];                       // new label = a caller id
    const int64_t u = inv ? (int64_t)inv[i] : i;  // this vertex's caller id
    const int64_t ci = perm ? (int64_t)perm[c] : (int64_t)c;  // vertex c, internal
    int32_t lab = C[ci];
    if ((int64_t)c < u && chg[ci] && R[ci]) lab = Cp[ci];
    const uint8_t r = lab != c ? 1 : 0;
    if (r != R[i]) {
      R[i] = r;
      moved = true;
    }
  }
  if (__any(moved) && (threadIdx.x & 63) == 0) st->cc_moved = 1u;
}

__global__ void k_cc_apply(int32_t* C, const int32_t* Cp, uint8_t* chg, uint8_t* R, int64_t n,
                           DevStats* st) {
  uint32_t rev = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (chg[i] && R[i]) {
      C[i] = Cp[i];
      chg[i] = 0;
      R[i] = 0;
      ++rev;
    }
  }
  for (int ofs = 32; ofs > 0; ofs >>= 1) rev += __shfl_xor(rev, ofs);
  if ((threadIdx.x & 63) == 0 && rev) atomicAdd(&st->reverted, (unsigned long long)rev);
}

__global__ void k_cc_clear_moved(DevStats* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->cc_moved = 0u;
}

hipError_t launch_cc_save(const int32_t* C, int32_t* Cp, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cc_save, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, C, Cp, n);
  return hipGetLastError();
}
hipError_t launch_cc_round(const int32_t* C, const int32_t* Cp, const uint8_t* chg, uint8_t* R,
                           const int32_t* perm, const int32_t* inv, int64_t n, DevStats* st,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_cc_clear_moved, dim3(1), dim3(64), 0, s, st);
  hipLaunchKernelGGL(k_cc_round, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, C, Cp, chg, R,
                     perm, inv, n, st);
  return hipGetLastError();
}
hipError_t launch_cc_apply(int32_t* C, const int32_t* Cp, uint8_t* chg, uint8_t* R, int64_t n,
                           DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cc_apply, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, C, Cp, chg, R,
                     n, st);
  return hipGetLastError();
}

__global__ void k_flags_resume(DevStats* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->stop = 0;
    st->pull_mode = 1u;
  }
}
__global__ void k_flags_done(DevStats* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->stop = 1;
    st->pull_mode = 2u;
    st->flags_deferred = 0u;
  }
}
hipError_t launch_flags_resume(DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_flags_resume, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}
hipError_t launch_flags_done(DevStats* st, hipStream_t s) {
  hipLaunchKernelGGL(k_flags_done, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

// push: classes 1..4 with 8 lanes per vertex, classes 5..8 with a workgroup
// per vertex (hub rows: k_push_hubs, one workgroup per slice)
template <typename OffT>
__global__ __launch_bounds__(kBT) void k_push_lists(const OffT* off, const int32_t* tgt,
                                                    ListPtrs lists, const uint8_t* chg,
                                                    uint8_t* F, DevStats* st) {
  if (st->stop || st->pull_mode) return;
  const int lane = threadIdx.x & 63;
  const int k = lane & 7;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int c = 1; c <= 4; ++c) {
    const int64_t cnt = st->active[c];
    const int32_t* list = lists.p[c];
    for (int64_t base = wave * 8; base < cnt; base += nwaves * 8) {
      const int64_t idx = base + (lane >> 3);
      if (idx >= cnt) continue;
      const int32_t v = list[idx];
      if (!chg[v]) continue;
      const int64_t o = (int64_t)off[v], d = (int64_t)off[v + 1] - o;
      for (int64_t e = k; e < d; e += 8) F[tgt[o + e]] = 1;
    }
  }
  for (int c = 5; c < kClassHub; ++c) {
    const int64_t cnt = st->active[c];
    const int32_t* list = lists.p[c];
    for (int64_t item = blockIdx.x; item < cnt; item += gridDim.x) {
      const int32_t v = list[item];
      if (!chg[v]) continue;
      const int64_t o = (int64_t)off[v], d = (int64_t)off[v + 1] - o;
      for (int64_t e = threadIdx.x; e < d; e += blockDim.x) F[tgt[o + e]] = 1;
    }
  }
}

hipError_t launch_push_lists(bool off64, const void* off, const int32_t* tgt,
                             int32_t* const* lists, const uint8_t* chg, uint8_t* F,
                             DevStats* st, int grid, hipStream_t s) {
  ListPtrs lp;
  for (int q = 0; q < kNumClasses; ++q) lp.p[q] = lists[q];
  if (off64)
    hipLaunchKernelGGL(k_push_lists<int64_t>, dim3(grid), dim3(kBT), 0, s,
                       (const int64_t*)off, tgt, lp, chg, F, st);
  else
    hipLaunchKernelGGL(k_push_lists<int32_t>, dim3(grid), dim3(kBT), 0, s,
                       (const int32_t*)off, tgt, lp, chg, F, st);
  return hipGetLastError();
}

template <typename OffT>
__global__ __launch_bounds__(kBT) void k_push_hubs(HubArgs a) {
  if (a.st->stop || a.st->pull_mode) return;
  const uint32_t nitems = a.st->hub_items;
  const OffT* off = reinterpret_cast<const OffT*>(a.off);
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t h = (int32_t)a.items[2 * (uint64_t)it];
    const int32_t c = (int32_t)a.items[2 * (uint64_t)it + 1];
    const int32_t v = a.hub_vid[h];
    if (!a.chg[v]) continue;
    const int64_t o = (int64_t)off[v], d = (int64_t)off[v + 1] - o;
    const int64_t e0 = (int64_t)c * a.chunk;
    const int64_t n = (d - e0 < a.chunk) ? d - e0 : a.chunk;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) a.F[a.tgt[o + e0 + e]] = 1;
  }
}

hipError_t launch_push_hubs(bool off64, const HubArgs& a, int grid, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_push_hubs<int64_t>, dim3(grid), dim3(kBT), 0, s, a);
  else
    hipLaunchKernelGGL(k_push_hubs<int32_t>, dim3(grid), dim3(kBT), 0, s, a);
  return hipGetLastError();
}

// pull: non-hub rows with 8 lanes per vertex, 8 entries per step; hub rows
// with one workgroup per hub.
namespace {
__device__ __forceinline__ uint32_t or8(uint32_t x) {
  x |= dpp32<0xB1, 0xF, 0xF, false>(x);   // quad_perm [1,0,3,2]
  x |= dpp32<0x4E, 0xF, 0xF, false>(x);   // quad_perm [2,3,0,1]
  x |= dpp32<0x141, 0xF, 0xF, false>(x);  // row_half_mirror
  return x;
}
}  // namespace

// The change bytes packed into bits (bit v % 32 of word v / 32) for the pull
// kernels: their reads land at data-dependent vertices, and the bitmap
// (n / 8 bytes) keeps far more of them in one cache line than the bytes do.
__global__ __launch_bounds__(kBT) void k_pack_chg(const uint8_t* chg, int64_t n, uint32_t* bits,
                                                  const DevStats* st) {
  if (st->stop || st->pull_mode != 1u) return;
  const int64_t nw = (n + 31) / 32;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw;
       w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t out = 0;
    if (32 * w + 32 <= n) {
      const uint32_t* p = reinterpret_cast<const uint32_t*>(chg + 32 * w);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t x = p[q];
        // the high bit of each byte of nz is set where that byte is nonzero
        const uint32_t nz = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
        out |= (((nz >> 7) & 1u) | ((nz >> 14) & 2u) | ((nz >> 21) & 4u) | ((nz >> 28) & 8u))
               << (4 * q);
      }
    } else {
      for (int64_t v = 32 * w; v < n; ++v)
        if (chg[v]) out |= 1u << (v - 32 * w);
    }
    bits[w] = out;
  }
}

__device__ __forceinline__ bool chg_bit(const uint32_t* bits, int32_t j) {
  return (bits[j >> 5] >> (j & 31)) & 1u;
}

template <typename OffT>
__global__ __launch_bounds__(kBT) void k_pull_flags(const OffT* off, const int32_t* tgt,
                                                    int64_t n, const uint8_t* cls,
                                                    const uint32_t* chg, uint8_t* F,
                                                    DevStats* st) {
  if (st->stop || st->pull_mode != 1u) return;
  const int lane = threadIdx.x & 63;
  const int k = lane & 7;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long scanned = 0;
  constexpr int kFirst = 4;  // entries a lane checks for its own vertex
  // one vertex per lane for its last kFirst entries (most rows find a
  // changed neighbour there); the rows left unresolved are then scanned
  // eight lanes per row, up to eight rows at a time.  Rows are read from
  // their end: with the internal order's rows sorted by target, the last
  // entries are the lowest-degree neighbours, which are the ones that still
  // change late in a run (from the start: 0.58 -> 0.89 ms per launch on
  // R-MAT 26)
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t v = base + lane;
    const bool valid = v < n && cls[v] != kClassHub;
    int64_t o = 0, d = 0;
    if (valid) {
      o = (int64_t)off[v];
      d = (int64_t)off[v + 1] - o;
    }
    int32_t j[kFirst];
#pragma unroll
    for (int u = 0; u < kFirst; ++u) j[u] = (u < d) ? tgt[o + d - 1 - u] : -1;
    bool found = false;
#pragma unroll
    for (int u = 0; u < kFirst; ++u) {
      if (j[u] >= 0 && !found) {
        ++scanned;
        found = chg_bit(chg, j[u]);
      }
    }
    if (found) F[v] = 1;
    unsigned long long pend = __ballot(!found && d > kFirst);
    while (pend) {
      // the g-th pending row of this round goes to lane group g
      const int g = lane >> 3;
      unsigned long long m = pend;
      for (int q = 0; q < g && m; ++q) m &= m - 1;
      const int src = m ? __ffsll((long long)m) - 1 : -1;
      const int sl = src < 0 ? 0 : src;
      const int64_t pv = base + sl;
      const int64_t po = __shfl(o, sl), pd = __shfl(d, sl);
      bool done = src < 0;  // the same for the 8 lanes of a group
      bool hitany = false;
      for (int64_t t = kFirst; __any(!done); t += 8) {
        uint32_t hit = 0;
        const int64_t e = t + k;
        if (!done && e < pd) {
          hit = chg_bit(chg, tgt[po + pd - 1 - e]) ? 1u : 0u;
          ++scanned;
        }
        hit = or8(hit);
        if (!done) {
          if (hit) { hitany = true; done = true; }
          else if (t + 8 >= pd) done = true;
        }
      }
      if (hitany && k == 0) F[pv] = 1;
      // drop the (up to eight) rows taken this round
      for (int q = 0; q < 8 && pend; ++q) pend &= pend - 1;
    }
  }
  // one atomic per workgroup
  __shared__ unsigned long long ws[kBT / 64];
  for (int ofs = 32; ofs > 0; ofs >>= 1) scanned += __shfl_xor(scanned, ofs);
  if (lane == 0) ws[threadIdx.x >> 6] = scanned;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < kBT / 64; ++q) t += ws[q];
    if (t) atomicAdd(&st->pull_scanned, t);
  }
}

template <typename OffT>
__global__ __launch_bounds__(kBT) void k_pull_hubs(const OffT* off, const int32_t* tgt,
                                                   const int32_t* hub_vid, int32_t H,
                                                   const uint32_t* chg, uint8_t* F,
                                                   DevStats* st) {
  constexpr int U = 8;  // entries per thread and step, all in flight at once
  __shared__ unsigned long long ws[kBT / 64];
  if (st->stop || st->pull_mode != 1u) return;
  unsigned long long scanned = 0;
  for (int32_t h = blockIdx.x; h < H; h += gridDim.x) {
    const int32_t v = hub_vid[h];
    const int64_t o = (int64_t)off[v];
    const int64_t d = (int64_t)off[v + 1] - o;
    bool found = false;
    for (int64_t t = 0; t < d && !found; t += (int64_t)kBT * U) {
      int32_t j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = t + (int64_t)u * kBT + threadIdx.x;
        j[u] = e < d ? tgt[o + e] : -1;
      }
      int hit = 0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (j[u] >= 0) {
          ++scanned;
          hit |= chg_bit(chg, j[u]) ? 1 : 0;
        }
      found = __syncthreads_or(hit) != 0;  // uniform over the workgroup
    }
    if (threadIdx.x == 0 && found) F[v] = 1;
  }
  // one atomic per workgroup
  for (int ofs = 32; ofs > 0; ofs >>= 1) scanned += __shfl_xor(scanned, ofs);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = scanned;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < kBT / 64; ++q) t += ws[q];
    if (t) atomicAdd(&st->pull_scanned, t);
  }
}

hipError_t launch_pull_flags(bool off64, const void* off, const int32_t* tgt, int64_t n,
                             const uint8_t* cls, const uint8_t* chg, uint32_t* chg_bits,
                             uint8_t* F, DevStats* st, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_chg, dim3(grid_for((n + 31) / 32, kBT, 8192)), dim3(kBT), 0, s, chg,
                     n, chg_bits, st);
  if (off64)
    hipLaunchKernelGGL(k_pull_flags<int64_t>, dim3(grid), dim3(kBT), 0, s,
                       (const int64_t*)off, tgt, n, cls, chg_bits, F, st);
  else
    hipLaunchKernelGGL(k_pull_flags<int32_t>, dim3(grid), dim3(kBT), 0, s,
                       (const int32_t*)off, tgt, n, cls, chg_bits, F, st);
  return hipGetLastError();
}

// chg_bits: the packed change bits that launch_pull_flags wrote just before
hipError_t launch_pull_hubs(bool off64, const void* off, const int32_t* tgt,
                            const int32_t* hub_vid, int32_t H, const uint32_t* chg,
                            uint8_t* F, DevStats* st, hipStream_t s) {
  const int g = H < 2048 ? H : 2048;
  if (off64)
    hipLaunchKernelGGL(k_pull_hubs<int64_t>, dim3(g), dim3(kBT), 0, s,
                       (const int64_t*)off, tgt, hub_vid, H, chg, F, st);
  else
    hipLaunchKernelGGL(k_pull_hubs<int32_t>, dim3(g), dim3(kBT), 0, s,
                       (const int32_t*)off, tgt, hub_vid, H, chg, F, st);
  return hipGetLastError();
}

// ---- deterministic mode: publish the labels of this iteration -------------
// Every vertex processed by a class kernel wrote its next label to Cn; hubs
// queued their moves.  Copy both into C.
__global__ void k_apply(const DevStats* st, ListPtrs lists, const int32_t* Cn,
                        const int32_t* pv, const int32_t* pc, int32_t* C) {
  if (st->stop) return;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  const unsigned long long t0 = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  const unsigned long long nq = st->pending;
  for (unsigned long long i = t0; i < nq; i += stride) C[pv[i]] = pc[i];
  for (int c = 1; c < kClassHub; ++c) {
    const unsigned long long cnt = st->active[c];
    const int32_t* list = lists.p[c];
    for (unsigned long long i = t0; i < cnt; i += stride) {
      const int32_t v = list[i];
      C[v] = Cn[v];
    }
  }
}

hipError_t launch_apply(const DevStats* st, int32_t* const* lists, const int32_t* Cn,
                        const int32_t* pv, const int32_t* pc, int32_t* C, int grid,
                        hipStream_t s) {
  ListPtrs lp;
  for (int q = 0; q < kNumClasses; ++q) lp.p[q] = lists[q];
  hipLaunchKernelGGL(k_apply, dim3(grid), dim3(kBT), 0, s, st, lp, Cn, pv, pc, C);
  return hipGetLastError();
}

// ---- modularity, Eq. 1 ------------------------------------------------------
// Community form: Q = sigma / 2m - sum_c (Sigma_c / 2m)^2.  Edge-parallel: each
// wave owns a contiguous range of CSR entries and takes 64 consecutive ones
// per step (coalesced target and weight loads).  The row of each entry comes
// from the 64 row ends that follow the wave's current row, searched across
// lanes; an entry adds its weight to 2m, to sigma when both end labels agree,
// and to Sigma of its row's label.  Sigma is summed over each run of lanes
// whose rows share a label, then gathered per wave in a small LDS table of
// labels (a direct-mapped cache flushed with one fp64 atomic per label at the
// end of the wave's range), so that a label shared by many rows -- a large
// community -- costs few atomics on its one address.
namespace {

__device__ __forceinline__ double block_sum_f64(double x, double* sh) {
  for (int ofs = 32; ofs > 0; ofs >>= 1) x += __shfl_xor(x, ofs);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int64_t shfl_i64(int64_t x, int src) {
  const int lo = __shfl((int)(uint32_t)x, src);
  const int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

}  // namespace

constexpr int kModCache = 64;  // label slots per wave

template <typename OffT>
__global__ __launch_bounds__(kBT) void k_mod_edges(const OffT* off, const int32_t* tgt,
                                                   const float* w, int64_t n, int64_t m,
                                                   const int32_t* C, double* sig,
                                                   double* acc) {
  __shared__ double sh[kBT / 64];
  __shared__ int32_t ckey_all[kBT / 64][kModCache];
  __shared__ double cval_all[kBT / 64][kModCache];
  const int lane = threadIdx.x & 63;
  int32_t* ckey = ckey_all[threadIdx.x >> 6];
  double* cval = cval_all[threadIdx.x >> 6];
  ckey[lane] = -1;
  cval[lane] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t S = (((m + nwaves - 1) / nwaves) + 63) & ~(int64_t)63;
  const int64_t e_begin = wave * S;
  const int64_t e_end = (e_begin + S < m) ? e_begin + S : m;
  double sigma = 0.0, two_m = 0.0;
  if (e_begin < e_end) {  // uniform over the wave
    // row of e_begin: the largest i with off[i] <= e_begin
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)off[mid] <= e_begin) lo = mid; else hi = mid - 1;
    }
    int64_t r0 = lo;
    for (int64_t base = e_begin; base < e_end; base += 64) {
      const int64_t e = base + lane;
      const bool valid = e < e_end;
      // row of e: r0 plus the number of row ends <= e, window by window
      int64_t myrow = valid ? -1 : r0;
      for (int64_t rb = r0;; rb += 64) {
        const int64_t idx = rb + 1 + lane;
        const int64_t end_k = idx <= n ? (int64_t)off[idx] : INT64_MAX;
        int pos = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const int64_t v = shfl_i64(end_k, pos + step - 1);
          if (v <= e) pos += step;
        }
        const int cnt = pos + (shfl_i64(end_k, pos) <= e ? 1 : 0);
        if (myrow < 0 && cnt < 64) myrow = rb + cnt;
        if (!__any(myrow < 0)) break;
      }
      int32_t ci = -1;
      double we = 0.0;
      if (valid) {
        ci = C[myrow];
        we = w ? (double)w[e] : 1.0;
        two_m += we;
        if (C[tgt[e]] == ci) sigma += we;
      }
      // segmented sum of we over runs of equal labels, one atomic per run
      const int32_t prev = __shfl_up(ci, 1);
      const int32_t next = __shfl_down(ci, 1);
      int f = (lane == 0 || prev != ci) ? 1 : 0;
      double sm = we;
#pragma unroll
      for (int ofs = 1; ofs < 64; ofs <<= 1) {
        const double ys = __shfl_up(sm, ofs);
        const int yf = __shfl_up(f, ofs);
        if (lane >= ofs && !f) {
          sm += ys;
          f |= yf;
        }
      }
      const bool tail = lane == 63 || next != ci;
      if (tail && ci >= 0 && sm != 0.0) {
        const int slot = (int)(((uint32_t)ci * 0x9E3779B1u) >> 26);  // 64 slots
        int k = __hip_atomic_load(&ckey[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (k == -1) {
          int expected = -1;
          __hip_atomic_compare_exchange_strong(&ckey[slot], &expected, ci, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
          k = expected == -1 ? ci : expected;
        }
        if (k == ci)
          __hip_atomic_fetch_add(&cval[slot], sm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        else
          atomicAdd(&sig[ci], sm);  // slot held by another label
      }
      const int last = (int)((e_end - 1 - base) < 63 ? (e_end - 1 - base) : 63);
      r0 = shfl_i64(myrow, last);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (ckey[lane] >= 0 && cval[lane] != 0.0) atomicAdd(&sig[ckey[lane]], cval[lane]);
  const double s1 = block_sum_f64(sigma, sh);
  const double s2 = block_sum_f64(two_m, sh);
  if (threadIdx.x == 0) {
    atomicAdd(&acc[0], s1);
    atomicAdd(&acc[1], s2);
  }
}

__global__ __launch_bounds__(kBT) void k_mod_sq(const double* sig, int64_t n, double* acc) {
  __shared__ double sh[kBT / 64];
  double s = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    s += sig[c] * sig[c];
  const double t = block_sum_f64(s, sh);
  if (threadIdx.x == 0) atomicAdd(&acc[2], t);
}

// ---- modularity scratch for callers that cannot allocate ----------------------
// Sigma_c (one double per vertex) and the four accumulators of
// lpa_modularity_noalloc live in this file-scope array: one copy per GPU,
// 32 MiB, held until the process ends.  Host code never takes the array's
// name as an address (it is a host-side stand-in); the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) double scratch[kModScratchVertices + 4];

hipError_t modularity_scratch(double** sig, double** acc) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *sig = addr[dev];
  *acc = addr[dev] + kModScratchVertices;
  return hipSuccess;
}

hipError_t launch_modularity(bool off64, const void* off, const int32_t* tgt, const float* w,
                             int64_t n, int64_t m, const int32_t* C, double* sig,
                             double* acc, hipStream_t s) {
  hipError_t e = launch_fill_f64(sig, 0.0, n, s);
  if (e != hipSuccess) return e;
  e = launch_fill_f64(acc, 0.0, 4, s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    const int g = grid_for((m + 63) / 64, kBT, 16384);
    if (off64)
      hipLaunchKernelGGL(k_mod_edges<int64_t>, dim3(g), dim3(kBT), 0, s, (const int64_t*)off,
                         tgt, w, n, m, C, sig, acc);
    else
      hipLaunchKernelGGL(k_mod_edges<int32_t>, dim3(g), dim3(kBT), 0, s, (const int32_t*)off,
                         tgt, w, n, m, C, sig, acc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mod_sq, dim3(grid_for(n, kBT, 8192)), dim3(kBT), 0, s, sig, n, acc);
  return hipGetLastError();
}

}  // namespace lpa
