// queue.hip -- batched label propagation (Algorithm 1 run on many independent
// graphs packed into one CSR) as a persistent work queue.
//
// An item is a chunk of up to 2^chunk_log2 consecutive vertices of one graph.
// Per iteration:
//   k_queue_iter_begin  resets the iteration's counters (one thread);
//   k_queue_sweep       a resident grid (every workgroup the GPU holds at
//                       once) pops items from the queue until it is drained.
//                       For each item the workgroup reads and clears the
//                       chunk's flags, sorts the flagged vertices by row
//                       length into two LDS lists and processes them: rows of
//                       up to group_max entries with 16 lanes and a 127-slot
//                       LDS table each (16 rows at a time), longer ones (up
//                       to 512 entries) with the whole workgroup and a
//                       1023-slot table in the same LDS.  The first sweep
//                       from the ids over strictly increasing rows needs no
//                       table (each label occurs once per row).
//                       Each vertex takes the label of maximum summed weight
//                       (Eq. 3; smallest label on ties), moves under the
//                       Pick-Less rule (Sec. 4.1) and, when it moves, flags
//                       every neighbour for the next iteration (Sec. 4 item
//                       4) and marks their chunks to be queued;
//   k_queue_step        one workgroup per graph applies Algorithm 1's stop
//                       test with the graph's own vertex count and queues
//                       the graph's marked chunks for the next iteration;
//   k_iter_end          (graph.hip) records the iteration and ends the run
//                       when every graph has stopped.
// The iteration boundary is the only barrier: a graph's next iteration reads
// what the previous kernels wrote, and graphs never share a vertex, so no
// ordering is needed inside the sweep beyond the relaxed atomics of the
// queue counters.  The queue has two halves by iteration parity, and each
// half one part per XCD: all chunks of graph g go to part g mod 8, so a
// graph's labels, flags and rows are cached in the L2 of the XCD that works
// on it.  A workgroup pops from its own XCD's part first and takes items
// from the other parts once that is drained.
//
// Deterministic mode keeps two label arrays by iteration parity.  A visited
// chunk writes the next label of every vertex (processed ones their result,
// the others a copy); a chunk in which a label changed is visited again in
// the next iteration, so that the copy catches up.  A chunk left unvisited
// had no change in the previous iteration and therefore holds the same
// labels in both arrays.  A graph's final labels (and its flags for a next
// iteration) are in the arrays of its iteration-count parity;
// k_queue_finish moves the odd ones.
#include "lpa_device.h"

namespace lpa {

namespace {

constexpr int kQBT = 256;                 // threads per sweep workgroup
constexpr int kQGroups = kQBT / 16;       // 16-lane groups per workgroup
constexpr int kQGroupSlots = 127;         // group tables: rows of up to 64 entries
constexpr int kQWaves = kQBT / 64;
constexpr int kQPool = kQGroups * kQGroupSlots;  // LDS table slots per workgroup
constexpr uint32_t kNoItem = 0xFFFFFFFFu;
static_assert(2 * kQueueMaxDegree - 1 <= kQPool, "the pool holds a 512-entry row's table");

__device__ __forceinline__ unsigned int* qhead(unsigned int* ctr, int par, uint32_t x) {
  return ctr + (size_t)((par * kXcds + (int)x) * 2) * kQueueCtrStride;
}
__device__ __forceinline__ unsigned int* qtail(unsigned int* ctr, int par, uint32_t x) {
  return ctr + (size_t)((par * kXcds + (int)x) * 2 + 1) * kQueueCtrStride;
}

// Next item of queue half par for a workgroup, trying part `from` first (its
// own XCD's, later the part it last took an item from), then the others;
// kNoItem once every part is drained.  The tails were written by earlier
// kernels and do not change during the sweep; heads may run past them.
__device__ uint32_t queue_pop(const QueueArgs& q, int par, uint32_t& from) {
  for (int k = 0; k < kXcds; ++k) {
    const uint32_t p = (from + (uint32_t)k) & (uint32_t)(kXcds - 1);
    const unsigned int tail = *qtail(q.qctr, par, p);
    unsigned int* head = qhead(q.qctr, par, p);
    if (__hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tail) continue;
    const unsigned int pos = atomicAdd(head, 1u);
    if (pos < tail) {
      from = p;
      return q.items[(size_t)par * (size_t)q.nchunks + (size_t)q.qbase[p] + pos];
    }
  }
  return kNoItem;
}

}  // namespace

template <typename OffT>
__global__ __launch_bounds__(kQBT) void k_queue_sweep(QueueArgs q) {
  // one LDS pool: 16 group tables of 127 slots, or one 1023-slot table for
  // the workgroup path
  __shared__ uint32_t keys[kQPool];
  __shared__ float vals[kQPool];
  __shared__ uint16_t lsmall[1 << kQueueMaxChunkLog2];
  __shared__ uint16_t llarge[1 << kQueueMaxChunkLog2];
  __shared__ unsigned long long wbest[kQWaves];
  __shared__ uint32_t nsmall, nlarge, ichg, item_sh;
  __shared__ int moved_sh;
  DevStats* st = q.st;
  if (st->stop) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l = st->iter;
  const int par = l & 1;
  const int pl = st->pl;                       // fixed for the whole sweep
  const bool id0 = l == 0 && st->ident;        // labels are still the ids
  // first sweep from the ids over rows with strictly increasing targets:
  // every neighbour label occurs once, so a row's Eq. 3 maximum is its
  // largest (weight, smallest id) entry and no table is needed
  const bool direct = id0 && q.strict_rows;
  int32_t* Cc = par ? q.C1 : q.C0;             // labels at the iteration start
  int32_t* Cw = par ? q.C0 : q.C1;             // deterministic: labels after it
  uint8_t* Fc = par ? q.F1 : q.F0;
  uint8_t* Fn = par ? q.F0 : q.F1;
  const OffT* off = reinterpret_cast<const OffT*>(q.off);
  const int64_t CH = (int64_t)1 << q.chunk_log2;
  const int64_t gm = q.group_max;
  const bool unit = q.w == nullptr;
  const bool det = !q.async_mode;
  for (int s = tid; s < kQPool; s += kQBT) {
    keys[s] = kEmpty;
    vals[s] = 0.0f;
  }
  uint32_t from = xcc_id();
  unsigned long long my_edges = 0, my_proc = 0;
  uint32_t my_changed = 0;
  if (tid == 0) {
    nsmall = 0;
    nlarge = 0;
    ichg = 0;
    item_sh = queue_pop(q, par, from);
  }
  __syncthreads();
  while (true) {
    const uint32_t it = item_sh;
    if (it == kNoItem) break;
    const int32_t g = q.cgraph[it];
    const int64_t gv0 = q.b.v_off[g], gv1 = q.b.v_off[g + 1];
    const int64_t c0 = q.cbase[g], c1 = q.cbase[g + 1];
    const int64_t v0 = gv0 + (((int64_t)it - c0) << q.chunk_log2);
    const int64_t v1 = (v0 + CH < gv1) ? v0 + CH : gv1;
    // 1. the chunk's flags: flagged vertices into the two lists by row
    //    length; in deterministic mode the others carry their label over
    for (int64_t base = v0; base < v1; base += kQBT) {
      const int64_t v = base + tid;
      bool fs = false, fl = false;
      if (v < v1) {
        if (Fc[v]) {
          Fc[v] = 0;
          const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
          ++my_proc;
          fs = d >= 1 && d <= gm;
          fl = d > gm && d <= kQueueMaxDegree;
          // a row longer than the tables (the CSR changed after create):
          // left alone, reported through the error bits
          if (d > kQueueMaxDegree) atomicOr(&st->error, 32u);
          if ((d == 0 || d > kQueueMaxDegree) && det) Cw[v] = Cc[v];
        } else if (det) {
          Cw[v] = Cc[v];
        }
      }
      const unsigned long long ms = __ballot(fs), ml = __ballot(fl);
      uint32_t bs = 0, bl = 0;
      if (lane == 0) {
        if (ms) bs = atomicAdd(&nsmall, (uint32_t)__popcll(ms));
        if (ml) bl = atomicAdd(&nlarge, (uint32_t)__popcll(ml));
      }
      bs = (uint32_t)__shfl((int)bs, 0);
      bl = (uint32_t)__shfl((int)bl, 0);
      if (fs) lsmall[bs + lane_rank(ms)] = (uint16_t)(v - v0);
      if (fl) llarge[bl + lane_rank(ml)] = (uint16_t)(v - v0);
    }
    __syncthreads();
    uint32_t item_changed = 0;
    // 2. rows of up to group_max (<= 64) entries: 16 lanes each
    {
      const int gi = tid >> 4, k = tid & 15;
      uint32_t* tk = keys + gi * kQGroupSlots;
      float* tv = vals + gi * kQGroupSlots;
      const uint32_t ns = nsmall;
      // the 16 lanes of a group are active or inactive together
      for (uint32_t idx = (uint32_t)gi; idx < ns; idx += kQGroups) {
        const int32_t v = (int32_t)(v0 + lsmall[idx]);
        const int64_t o = (int64_t)off[v];
        const int64_t d = (int64_t)off[v + 1] - o;
        const int32_t cur = Cc[v];
        int32_t j[4];
        float wt[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t e = u * 16 + k;
          const bool has = e < d;
          j[u] = has ? __builtin_nontemporal_load(&q.tgt[o + e]) : v;
          wt[u] = has ? edge_weight(q.w, o + e) : 0.0f;
        }
        unsigned long long best = 0;
        if (direct) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j[u] != v) best = umax64(best, pack_key(wt[u], (uint32_t)j[u]));
        } else {
          const uint32_t p1 = table_p1((uint32_t)d);
          uint32_t lab[4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            lab[u] = (j[u] != v) ? (id0 ? (uint32_t)j[u] : (uint32_t)Cc[j[u]]) : kEmpty;
#pragma unroll
          for (int u = 0; u < 4; ++u) merge_lead16(lab[u], wt[u], unit);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (lab[u] != kEmpty) lds_accumulate(tk, tv, p1, lab[u], wt[u], q.probe);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          for (uint32_t s = (uint32_t)k; s < p1; s += 16) {
            const uint32_t kk = tk[s];
            if (kk != kEmpty) {
              best = umax64(best, pack_key(tv[s], kk));
              tk[s] = kEmpty;
              tv[s] = 0.0f;
            }
          }
        }
        best = row16_max_u64(best);
        uint32_t cstar = 0;
        const bool moved = decide(best, cur, pl, &cstar);
        if (k == 0) {
          if (det) Cw[v] = moved ? (int32_t)cstar : cur;
          else if (moved) Cc[v] = (int32_t)cstar;
          my_edges += (unsigned long long)d;
          if (moved) {
            ++my_changed;
            ++item_changed;
          }
        }
        if (moved) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u * 16 + k < d) {
              Fn[j[u]] = 1;
              const int64_t cj = c0 + (((int64_t)j[u] - gv0) >> q.chunk_log2);
              if (cj >= c0 && cj < c1) q.cmark[cj] = 1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    // 3. rows of group_max + 1 .. 512 entries: the whole workgroup, one row
    //    at a time, in a 1023-slot table over the group tables' LDS
    const uint32_t nl = nlarge;
    for (uint32_t idx = 0; idx < nl; ++idx) {
      __syncthreads();  // the previous row's (or the groups') table is clear
      const int32_t v = (int32_t)(v0 + llarge[idx]);
      const int64_t o = (int64_t)off[v];
      const int64_t d = (int64_t)off[v + 1] - o;
      const int32_t cur = Cc[v];
      const uint32_t p1 = table_p1((uint32_t)d);
      unsigned long long best = 0;
      for (int64_t e0 = 0; e0 < d; e0 += kQBT) {
        const int64_t e = e0 + tid;
        const bool has = e < d;
        const int32_t j = has ? __builtin_nontemporal_load(&q.tgt[o + e]) : v;
        float wt = has ? edge_weight(q.w, o + e) : 0.0f;
        if (direct) {
          if (j != v) best = umax64(best, pack_key(wt, (uint32_t)j));
        } else {
          uint32_t lab = (j != v) ? (id0 ? (uint32_t)j : (uint32_t)Cc[j]) : kEmpty;
          merge_lead(lab, wt, unit);
          if (lab != kEmpty) lds_accumulate(keys, vals, p1, lab, wt, q.probe);
        }
      }
      if (!direct) {
        __syncthreads();
        for (uint32_t s = (uint32_t)tid; s < p1; s += kQBT) {
          const uint32_t kk = keys[s];
          if (kk != kEmpty) {
            best = umax64(best, pack_key(vals[s], kk));
            keys[s] = kEmpty;
            vals[s] = 0.0f;
          }
        }
      }
      best = wave_max_u64(best);
      if (lane == 0) wbest[wv] = best;
      __syncthreads();
      if (tid == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < kQWaves; ++w) b = umax64(b, wbest[w]);
        uint32_t cstar = 0;
        const bool moved = decide(b, cur, pl, &cstar);
        if (det) Cw[v] = moved ? (int32_t)cstar : cur;
        else if (moved) Cc[v] = (int32_t)cstar;
        my_edges += (unsigned long long)d;
        if (moved) {
          ++my_changed;
          ++item_changed;
        }
        moved_sh = moved ? 1 : 0;
      }
      __syncthreads();
      if (moved_sh) {
        for (int64_t e = tid; e < d; e += kQBT) {
          const int32_t jj = q.tgt[o + e];
          Fn[jj] = 1;
          const int64_t cj = c0 + (((int64_t)jj - gv0) >> q.chunk_log2);
          if (cj >= c0 && cj < c1) q.cmark[cj] = 1;
        }
      }
    }
    // 4. the item's changes go to the graph's count; a chunk with a change
    //    is visited again next iteration (deterministic copy, see above)
    const uint32_t c = wave_sum_u32(item_changed);
    if (lane == 0 && c) atomicAdd(&ichg, c);
    __syncthreads();
    if (tid == 0) {
      if (ichg) {
        atomicAdd(&q.gchanged[g], ichg);
        q.cmark[it] = 1;
      }
      ichg = 0;
      nsmall = 0;
      nlarge = 0;
      item_sh = queue_pop(q, par, from);
    }
    __syncthreads();
  }
  // one device atomic per counter and workgroup
  flush_stats(my_edges, my_changed, 0ull, st, 0);
  __shared__ unsigned long long wp[kQWaves];
  const unsigned long long p = wave_sum_u64(my_proc);
  if (lane == 0) wp[wv] = p;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kQWaves; ++w) t += wp[w];
    if (t) atomicAdd(&st->processed, t);
  }
}

// Counters of the iteration; the other queue half is emptied for the step
// kernel to refill.
__global__ void k_queue_iter_begin(QueueArgs q) {
  DevStats* st = q.st;
  if (st->stop) return;
  const int tid = threadIdx.x;
  if (tid == 0) {
    st->processed = 0;
    st->pending = 0;
    st->pull_scanned = 0;
    st->pull_mode = 0;
    st->graphs_left = 0;
    // Pick-Less in iterations l with l mod rho == 0, counting from 0
    st->pl = (st->rho > 0 && st->iter % st->rho == 0) ? 1 : 0;
  }
  if (tid < kNumClasses) {
    st->active[tid] = 0;
    st->edges[tid] = 0;
    st->changed[tid] = 0;
    st->flagw[tid] = 0;
  }
  const int np = (st->iter + 1) & 1;
  if (tid < 2 * kXcds) q.qctr[(size_t)(np * 2 * kXcds + tid) * kQueueCtrStride] = 0u;
}

// Per graph still running: Algorithm 1's stop test on its own counts, then
// its marked chunks into the next queue half (one tail atomic per round of
// 256 chunks).
__global__ __launch_bounds__(kQBT) void k_queue_step(QueueArgs q) {
  __shared__ uint32_t wcnt[kQWaves];
  __shared__ uint32_t base_sh;
  __shared__ int state_sh;
  DevStats* st = q.st;
  if (st->stop) return;
  const int l = st->iter;
  const int np = (l + 1) & 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int32_t g = blockIdx.x; g < q.b.G; g += gridDim.x) {
    if (tid == 0) {
      int state = 0;  // 0: stopped earlier, 1: stops now, 2: runs on
      if (!q.b.done[g]) {
        const unsigned int t = q.gchanged[g];
        q.gchanged[g] = 0u;
        const int64_t ng = q.b.v_off[g + 1] - q.b.v_off[g];
        q.b.changed_last[g] = (long long)t;
        const bool f = (!st->pl && (double)t < st->tol * (double)ng) || l + 1 >= st->cap;
        if (f) {
          q.b.done[g] = 1;
          q.b.iters[g] = l + 1;
          state = 1;
        } else {
          atomicAdd(&st->graphs_left, 1u);
          state = 2;
        }
      }
      state_sh = state;
    }
    __syncthreads();
    if (state_sh == 2) {
      const int64_t c0 = q.cbase[g], c1 = q.cbase[g + 1];
      const uint32_t x = (uint32_t)g & (uint32_t)(kXcds - 1);
      uint32_t* out = q.items + (size_t)np * (size_t)q.nchunks + (size_t)q.qbase[x];
      for (int64_t cb = c0; cb < c1; cb += kQBT) {
        const int64_t c = cb + tid;
        bool vis = false;
        if (c < c1 && q.cmark[c]) {
          q.cmark[c] = 0;
          vis = true;
        }
        const unsigned long long m = __ballot(vis);
        if (lane == 0) wcnt[wv] = (uint32_t)__popcll(m);
        __syncthreads();
        if (tid == 0) {
          uint32_t tot = 0;
          for (int w = 0; w < kQWaves; ++w) tot += wcnt[w];
          base_sh = tot ? atomicAdd(qtail(q.qctr, np, x), tot) : 0u;
        }
        __syncthreads();
        uint32_t pos = base_sh;
        for (int w = 0; w < wv; ++w) pos += wcnt[w];
        if (vis) out[pos + lane_rank(m)] = (uint32_t)c;
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// Graphs that stopped after an odd number of iterations hold their flags for
// a next iteration in F1 and, in deterministic mode, their labels in C1:
// both move to the even arrays, which are the handle's.
__global__ __launch_bounds__(kQBT) void k_queue_finish(QueueArgs q) {
  const bool det = q.C1 != q.C0;
  for (int32_t g = blockIdx.x; g < q.b.G; g += gridDim.x) {
    if ((q.b.iters[g] & 1) == 0) continue;
    for (int64_t v = q.b.v_off[g] + threadIdx.x; v < q.b.v_off[g + 1]; v += kQBT) {
      q.F0[v] = q.F1[v];
      if (det) q.C0[v] = q.C1[v];
    }
  }
}

template <typename OffT>
__global__ void k_max_degree(const OffT* off, int64_t n, unsigned long long* dmax) {
  unsigned long long m = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long d = (unsigned long long)((int64_t)off[v + 1] - (int64_t)off[v]);
    m = d > m ? d : m;
  }
  for (int ofs = 32; ofs > 0; ofs >>= 1) {
    const unsigned long long o = __shfl_xor(m, ofs);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax(dmax, m);
}

// The initial queue (every chunk of every non-empty graph, in XCD parts)
// and its counters are built once by the host and copied in; the odd flags,
// the chunk marks and the graphs' counts start at zero; deterministic mode
// starts both label arrays equal.
hipError_t launch_queue_begin(const QueueArgs& q, int64_t n, hipStream_t s) {
  hipError_t e = launch_fill_u8(q.F1, 0, n, s);
  if (e == hipSuccess) e = launch_fill_u8(q.cmark, 0, q.nchunks, s);
  if (e == hipSuccess) e = launch_fill_u32(q.gchanged, 0u, q.b.G, s);
  if (e == hipSuccess && q.C1 != q.C0)
    e = hipMemcpyAsync(q.C1, q.C0, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
  return e;
}

hipError_t launch_queue_iter_begin(const QueueArgs& q, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_iter_begin, dim3(1), dim3(64), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_queue_sweep(bool off64, const QueueArgs& q, int grid, hipStream_t s) {
  if (q.chunk_log2 < 0 || q.chunk_log2 > kQueueMaxChunkLog2 || q.group_max < 1 ||
      q.group_max > 64)
    return hipErrorInvalidValue;
  if (off64)
    hipLaunchKernelGGL(k_queue_sweep<int64_t>, dim3(grid), dim3(kQBT), 0, s, q);
  else
    hipLaunchKernelGGL(k_queue_sweep<int32_t>, dim3(grid), dim3(kQBT), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_queue_step(const QueueArgs& q, hipStream_t s) {
  const int g = q.b.G < 8192 ? (q.b.G > 0 ? q.b.G : 1) : 8192;
  hipLaunchKernelGGL(k_queue_step, dim3(g), dim3(kQBT), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_queue_finish(const QueueArgs& q, hipStream_t s) {
  const int g = q.b.G < 8192 ? (q.b.G > 0 ? q.b.G : 1) : 8192;
  hipLaunchKernelGGL(k_queue_finish, dim3(g), dim3(kQBT), 0, s, q);
  return hipGetLastError();
}

// Seven workgroups per CU: 16 KB of tables and 4 KB of lists each.
int queue_sweep_resident() { return 256 * 7; }

hipError_t launch_max_degree(bool off64, const void* off, int64_t n, unsigned long long* dmax,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const int g = (int)(want < 2048 ? want : 2048);
  if (off64)
    hipLaunchKernelGGL(k_max_degree<int64_t>, dim3(g), dim3(256), 0, s,
                       static_cast<const int64_t*>(off), n, dmax);
  else
    hipLaunchKernelGGL(k_max_degree<int32_t>, dim3(g), dim3(256), 0, s,
                       static_cast<const int32_t*>(off), n, dmax);
  return hipGetLastError();
}

}  // namespace lpa
