// sweep_tv.hip -- the table-value precision ablation of Sec. 4.4: the label
// sweep with 32-bit or 64-bit floating-point hashtable values.
//
// The class kernels of sweep.hip are specialised for fp32 values (packed
// 64-bit arg-max keys, register sums, 8-byte LDS slots sized to the 160 KB of
// a CU).  Comparing fp64 against them would measure those specialisations as
// much as the value width, so the ablation runs one kernel structure
// instantiated with V = float or V = double, and only the width differs:
//   k_tv_wave     one wave per vertex, LDS table (classes 1..4, rows <= 512)
//   k_tv_block    one workgroup per vertex, LDS table of up to 8191 slots
//                 (classes 5..7, rows <= 4096; 8191 x 12 B = 96 KB for fp64)
//   k_tv_hub_*    longer rows: every slice of the row adds into the hub's
//                 global-memory table with device-scope atomics; then each
//                 slice's share of the table yields its largest value, the
//                 smallest label holding the hub's largest value, and k_hub_fin
//                 of sweep.hip makes the move as in the main path.
// Every table holds D keys in 2^m - 1 >= 2D - 1 slots (load <= 1/2) and uses
// the probe sequence of lpa_tuning.probe, like the main kernels.  The arg-max
// reduces (value bits, ~label) pairs: for V >= 0 the bit patterns order like
// the values, and the complemented label makes the smaller label win a tie
// (Eq. 3 with the strict tie rule).  Labels, flags, counters and the move
// rule (Pick-Less, Sec. 4.1) are those of the main kernels.
#include "lpa_device.h"

namespace lpa {

namespace {

template <typename V>
__device__ __forceinline__ unsigned long long value_bits(V x);
template <>
__device__ __forceinline__ unsigned long long value_bits<float>(float x) {
  return (unsigned long long)__float_as_uint(x);
}
template <>
__device__ __forceinline__ unsigned long long value_bits<double>(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

// (vb, nl) <- the larger of the two pairs; (0, 0) is the empty pair.
__device__ __forceinline__ void pair_max(unsigned long long& vb, uint32_t& nl,
                                         unsigned long long ovb, uint32_t onl) {
  if (ovb > vb || (ovb == vb && onl > nl)) {
    vb = ovb;
    nl = onl;
  }
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ void pair_step(unsigned long long& vb, uint32_t& nl) {
  const unsigned long long ovb = dpp64<CTRL, ROW_MASK>(vb);
  const uint32_t onl = dpp32<CTRL, ROW_MASK>(nl);
  pair_max(vb, nl, ovb, onl);
}

// Largest pair over the 64 lanes (every lane active); uniform result.
__device__ __forceinline__ void wave_pair_max(unsigned long long& vb, uint32_t& nl) {
  pair_step<0x111>(vb, nl);        // row_shr:1
  pair_step<0x112>(vb, nl);        // row_shr:2
  pair_step<0x114>(vb, nl);        // row_shr:4
  pair_step<0x118>(vb, nl);        // row_shr:8
  pair_step<0x142, 0xA>(vb, nl);   // row_bcast:15
  pair_step<0x143, 0xC>(vb, nl);   // row_bcast:31
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)vb, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(vb >> 32), 63);
  vb = ((unsigned long long)hi << 32) | lo;
  nl = (uint32_t)__builtin_amdgcn_readlane((int)nl, 63);
}

__device__ __forceinline__ unsigned long long tv_wave_sum_u64(unsigned long long x) {
  x += dpp64<0x111>(x);
  x += dpp64<0x112>(x);
  x += dpp64<0x114>(x);
  x += dpp64<0x118>(x);
  x += dpp64<0x142, 0xA>(x);
  x += dpp64<0x143, 0xC>(x);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ void tv_flush_stats(unsigned long long edges, uint32_t changed,
                                               unsigned long long flagw, DevStats* st, int cls) {
  const unsigned long long e = tv_wave_sum_u64(edges);
  const uint32_t c = wave_sum_u32(changed);
  const unsigned long long f = tv_wave_sum_u64(flagw);
  if ((threadIdx.x & 63) == 0) {
    if (e) atomicAdd(&st->edges[cls], e);
    if (c) atomicAdd(&st->changed[cls], (unsigned long long)c);
    if (f) atomicAdd(&st->flagw[cls], f);
  }
}

// Move rule of the main kernels on a reduced pair: no key (only self-loops)
// keeps the label; otherwise move to a different label, under Pick-Less only
// to a smaller one.
__device__ __forceinline__ bool tv_decide(uint32_t nl, int32_t cur, int pl, uint32_t* cstar) {
  if (nl == 0u) return false;
  const uint32_t c = ~nl;
  *cstar = c;
  return (int32_t)c != cur && (!pl || (int32_t)c < cur);
}

// Algorithm 2, shared branch, in LDS: claim the key's slot by compare-and-swap
// and add the value atomically.
template <typename V>
__device__ __forceinline__ void tv_lds_accumulate(uint32_t* keys, V* vals, uint32_t p1,
                                                  uint32_t k, V v, ProbeCfg pc) {
  const uint32_t p2 = 2u * p1 + 1u;
  uint32_t s = k % p1;
  uint32_t step = 1u % p1;
  const uint32_t r = (k % p2) % p1;
  for (int t = 0;; ++t) {
    uint32_t cur = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == kEmpty) {
      uint32_t expected = kEmpty;
      __hip_atomic_compare_exchange_strong(&keys[s], &expected, k, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      cur = (expected == kEmpty) ? k : expected;
    }
    if (cur == k) {
      __hip_atomic_fetch_add(&vals[s], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    probe_next(s, step, r, p1, t, pc);
  }
}

// The same in a global-memory table shared by workgroups on every XCD.
template <typename V>
__device__ __forceinline__ void tv_global_accumulate(uint32_t* keys, V* vals, uint32_t p1,
                                                     uint32_t k, V v, ProbeCfg pc) {
  const uint32_t p2 = 2u * p1 + 1u;
  uint32_t s = k % p1;
  uint32_t step = 1u % p1;
  const uint32_t r = (k % p2) % p1;
  for (int t = 0;; ++t) {
    uint32_t cur = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kEmpty) {
      uint32_t expected = kEmpty;
      __hip_atomic_compare_exchange_strong(&keys[s], &expected, k, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      cur = (expected == kEmpty) ? k : expected;
    }
    if (cur == k) {
      __hip_atomic_fetch_add(&vals[s], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    probe_next(s, step, r, p1, t, pc);
  }
}

constexpr int kTvWaves = 4;     // waves (vertices) per workgroup of k_tv_wave
constexpr int kTvHubBT = 256;   // threads per workgroup of the hub kernels

// ---- one wave per vertex ----------------------------------------------------
template <typename OffT, typename V, int SLOTS>
__global__ __launch_bounds__(kTvWaves * 64) void k_tv_wave(SweepArgs a) {
  __shared__ uint32_t keys_all[kTvWaves][SLOTS];
  __shared__ V vals_all[kTvWaves][SLOTS];
  if (a.st->stop) return;
  const int pl = a.st->pl;
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  uint32_t* keys = keys_all[wv];
  V* vals = vals_all[wv];
  for (int s = lane; s < SLOTS; s += 64) { keys[s] = kEmpty; vals[s] = (V)0; }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0;
  for (uint32_t item = blockIdx.x * kTvWaves + wv; item < count;
       item += gridDim.x * kTvWaves) {
    const int32_t v = a.active[item];
    int64_t o, d;
    row_of<OffT>(a.off, v, &o, &d);
    const int32_t cur = a.C[v];
    const uint32_t p1 = table_p1((uint32_t)d);
    for (int64_t e = lane; e < d; e += 64) {
      const int32_t j = __builtin_nontemporal_load(&a.tgt[o + e]);
      if (j == v) continue;
      const uint32_t lab = id0 ? (uint32_t)j : (uint32_t)a.C[j];
      tv_lds_accumulate<V>(keys, vals, p1, lab, (V)edge_weight(a.w, o + e), a.probe);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long vb = 0;
    uint32_t nl = 0;
    for (uint32_t s = lane; s < p1; s += 64) {
      const uint32_t kk = keys[s];
      if (kk != kEmpty) {
        pair_max(vb, nl, value_bits<V>(vals[s]), ~kk);
        keys[s] = kEmpty;
        vals[s] = (V)0;
      }
    }
    wave_pair_max(vb, nl);
    uint32_t cstar = 0;
    const bool moved = tv_decide(nl, cur, pl, &cstar);
    if (lane == 0) {
      if (a.async_mode) {
        if (moved) a.C[v] = (int32_t)cstar;
      } else {
        a.Cn[v] = moved ? (int32_t)cstar : cur;
      }
      if (moved) a.chg[v] = 1;
      my_edges += (unsigned long long)d;
      my_changed += moved ? 1u : 0u;
      my_flagw += moved ? (unsigned long long)d : 0ull;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  tv_flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
}

// ---- one workgroup per vertex -------------------------------------------------
template <typename OffT, typename V, int SLOTS, int BT>
__global__ __launch_bounds__(BT) void k_tv_block(SweepArgs a) {
  constexpr int NW = BT / 64;
  __shared__ uint32_t keys[SLOTS];
  __shared__ V vals[SLOTS];
  __shared__ unsigned long long red_v[NW];
  __shared__ uint32_t red_l[NW];
  if (a.st->stop) return;
  const int pl = a.st->pl;
  const bool id0 = a.st->iter == 0 && a.st->ident;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int s = tid; s < SLOTS; s += BT) { keys[s] = kEmpty; vals[s] = (V)0; }
  __syncthreads();
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const int32_t v = a.active[item];
    int64_t o, d;
    row_of<OffT>(a.off, v, &o, &d);
    // read before the barriers: in asynchronous mode thread 0 overwrites it
    const int32_t cur = a.C[v];
    const uint32_t p1 = table_p1((uint32_t)d);
    for (int64_t e = tid; e < d; e += BT) {
      const int32_t j = __builtin_nontemporal_load(&a.tgt[o + e]);
      if (j == v) continue;
      const uint32_t lab = id0 ? (uint32_t)j : (uint32_t)a.C[j];
      tv_lds_accumulate<V>(keys, vals, p1, lab, (V)edge_weight(a.w, o + e), a.probe);
    }
    __syncthreads();
    unsigned long long vb = 0;
    uint32_t nl = 0;
    for (uint32_t s = tid; s < p1; s += BT) {
      const uint32_t kk = keys[s];
      if (kk != kEmpty) {
        pair_max(vb, nl, value_bits<V>(vals[s]), ~kk);
        keys[s] = kEmpty;
        vals[s] = (V)0;
      }
    }
    wave_pair_max(vb, nl);
    if (lane == 0) {
      red_v[tid >> 6] = vb;
      red_l[tid >> 6] = nl;
    }
    __syncthreads();
    vb = red_v[0];
    nl = red_l[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) pair_max(vb, nl, red_v[q], red_l[q]);
    uint32_t cstar = 0;
    const bool moved = tv_decide(nl, cur, pl, &cstar);
    if (tid == 0) {
      if (a.async_mode) {
        if (moved) a.C[v] = (int32_t)cstar;
      } else {
        a.Cn[v] = moved ? (int32_t)cstar : cur;
      }
      if (moved) a.chg[v] = 1;
      my_edges += (unsigned long long)d;
      my_changed += moved ? 1u : 0u;
      my_flagw += moved ? (unsigned long long)d : 0ull;
    }
    __syncthreads();
  }
  tv_flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
}

// ---- rows longer than the LDS tables ----------------------------------------
// Slice c of hub h covers entries [c chunk, (c + 1) chunk) of its row and the
// share [p1 c / ns, p1 (c + 1) / ns) of its table (ns slices).
struct HubSlice {
  int32_t h, v;
  int64_t o, d, e0, e1, s0, s1;
  uint32_t p1;
};

template <typename OffT>
__device__ __forceinline__ HubSlice hub_slice(const HubArgs& a, uint32_t it) {
  HubSlice q;
  q.h = (int32_t)a.items[2 * (uint64_t)it];
  const int64_t c = (int64_t)a.items[2 * (uint64_t)it + 1];
  q.v = a.hub_vid[q.h];
  row_of<OffT>(a.off, q.v, &q.o, &q.d);
  q.e0 = c * a.chunk;
  q.e1 = (q.d - q.e0 < a.chunk) ? q.d : q.e0 + a.chunk;
  q.p1 = table_p1((uint32_t)q.d);
  const int64_t ns = (q.d + a.chunk - 1) / a.chunk;
  q.s0 = (int64_t)q.p1 * c / ns;
  q.s1 = (int64_t)q.p1 * (c + 1) / ns;
  return q;
}

// Each queued slice adds its entries into the hub's table.
template <typename OffT, typename V>
__global__ __launch_bounds__(kTvHubBT) void k_tv_hub_acc(HubArgs a, V* gvals) {
  if (a.st->stop) return;
  const bool id0 = a.st->iter == 0 && a.st->ident;
  const uint32_t nitems = a.st->hub_items;
  unsigned long long my_edges = 0;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const HubSlice q = hub_slice<OffT>(a, it);
    uint32_t* gk = a.gkeys + a.hub_tab[q.h];
    V* gv = gvals + a.hub_tab[q.h];
    for (int64_t e = q.e0 + threadIdx.x; e < q.e1; e += kTvHubBT) {
      const int32_t j = __builtin_nontemporal_load(&a.tgt[q.o + e]);
      if (j == q.v) continue;
      const uint32_t lab = id0 ? (uint32_t)j : (uint32_t)a.C[j];
      tv_global_accumulate<V>(gk, gv, q.p1, lab, (V)edge_weight(a.w, q.o + e), a.probe);
    }
    if (threadIdx.x == 0) my_edges += (unsigned long long)(q.e1 - q.e0);
  }
  if (threadIdx.x == 0 && my_edges) atomicAdd(&a.st->edges[kClassHub], my_edges);
}

// Each queued slice: the largest value in its share of the hub's table.
template <typename OffT, typename V>
__global__ __launch_bounds__(kTvHubBT) void k_tv_hub_max(HubArgs a, const V* gvals,
                                                        unsigned long long* vmax) {
  __shared__ unsigned long long red[kTvHubBT / 64];
  if (a.st->stop) return;
  const int tid = threadIdx.x;
  const uint32_t nitems = a.st->hub_items;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const HubSlice q = hub_slice<OffT>(a, it);
    const uint32_t* gk = a.gkeys + a.hub_tab[q.h];
    const V* gv = gvals + a.hub_tab[q.h];
    unsigned long long best = 0;
    for (int64_t s = q.s0 + tid; s < q.s1; s += kTvHubBT)
      if (gk[s] != kEmpty) best = umax64(best, value_bits<V>(gv[s]));
    best = wave_max_u64(best);
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kTvHubBT / 64; ++w) best = umax64(best, red[w]);
      if (best) atomicMax(&vmax[q.h], best);
    }
    __syncthreads();
  }
}

// Each queued slice: the smallest label in its share that holds the hub's
// largest value (as the complement's maximum); the share is cleared.
template <typename OffT, typename V>
__global__ __launch_bounds__(kTvHubBT) void k_tv_hub_arg(HubArgs a, V* gvals,
                                                        const unsigned long long* vmax,
                                                        uint32_t* hub_nl) {
  __shared__ unsigned long long red[kTvHubBT / 64];
  if (a.st->stop) return;
  const int tid = threadIdx.x;
  const uint32_t nitems = a.st->hub_items;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const HubSlice q = hub_slice<OffT>(a, it);
    uint32_t* gk = a.gkeys + a.hub_tab[q.h];
    V* gv = gvals + a.hub_tab[q.h];
    const unsigned long long top = vmax[q.h];
    unsigned long long nl = 0;
    for (int64_t s = q.s0 + tid; s < q.s1; s += kTvHubBT) {
      const uint32_t kk = gk[s];
      if (kk != kEmpty) {
        if (value_bits<V>(gv[s]) == top) nl = umax64(nl, (unsigned long long)~kk);
        gk[s] = kEmpty;
        gv[s] = (V)0;
      }
    }
    nl = wave_max_u64(nl);
    if ((tid & 63) == 0) red[tid >> 6] = nl;
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kTvHubBT / 64; ++w) nl = umax64(nl, red[w]);
      if (nl) atomicMax(&hub_nl[q.h], (uint32_t)nl);
    }
    __syncthreads();
  }
}

// Per hub: the result as the packed key k_hub_fin reads (nonzero, with the
// label's complement in the low word); the per-hub state is reset.
__global__ void k_tv_hub_pack(HubArgs a, unsigned long long* vmax, uint32_t* hub_nl) {
  if (a.st->stop) return;
  for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < a.H;
       h += gridDim.x * blockDim.x) {
    const uint32_t nl = hub_nl[h];
    a.hub_best[h] = nl ? ((1ull << 32) | (unsigned long long)nl) : 0ull;
    vmax[h] = 0ull;
    hub_nl[h] = 0u;
  }
}

template <typename OffT, typename V>
hipError_t sweep_tv_t(int cls, const SweepArgs& a, int grid, hipStream_t s) {
  switch (cls) {
    case 1: case 2: case 3:
      hipLaunchKernelGGL((k_tv_wave<OffT, V, 127>), dim3(grid), dim3(kTvWaves * 64), 0, s, a);
      break;
    case 4:
      hipLaunchKernelGGL((k_tv_wave<OffT, V, 1023>), dim3(grid), dim3(kTvWaves * 64), 0, s, a);
      break;
    case 5:
      hipLaunchKernelGGL((k_tv_block<OffT, V, 2047, 256>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 6:
      hipLaunchKernelGGL((k_tv_block<OffT, V, 4095, 512>), dim3(grid), dim3(512), 0, s, a);
      break;
    case 7:
      hipLaunchKernelGGL((k_tv_block<OffT, V, 8191, 1024>), dim3(grid), dim3(1024), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;  // class 8 is empty when table_values is set
  }
  return hipGetLastError();
}

template <typename OffT, typename V>
hipError_t tv_hub_acc_t(const HubArgs& a, void* gvals, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_tv_hub_acc<OffT, V>), dim3(grid), dim3(kTvHubBT), 0, s, a,
                     static_cast<V*>(gvals));
  return hipGetLastError();
}

template <typename OffT, typename V>
hipError_t tv_hub_select_t(const HubArgs& a, void* gvals, unsigned long long* vmax,
                           uint32_t* hub_nl, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_tv_hub_max<OffT, V>), dim3(grid), dim3(kTvHubBT), 0, s, a,
                     static_cast<const V*>(gvals), vmax);
  hipLaunchKernelGGL((k_tv_hub_arg<OffT, V>), dim3(grid), dim3(kTvHubBT), 0, s, a,
                     static_cast<V*>(gvals), (const unsigned long long*)vmax, hub_nl);
  const int pg = (a.H + 255) / 256;
  hipLaunchKernelGGL(k_tv_hub_pack, dim3(pg < 1 ? 1 : pg), dim3(256), 0, s, a, vmax, hub_nl);
  return hipGetLastError();
}

// LDS bytes of one workgroup of each class's kernel.
int64_t tv_lds_bytes(int cls, int bits) {
  const int64_t slot = 4 + bits / 8;
  switch (cls) {
    case 1: case 2: case 3: return kTvWaves * 127 * slot;
    case 4: return kTvWaves * 1023 * slot;
    case 5: return 2047 * slot;
    case 6: return 4095 * slot;
    case 7: return 8191 * slot;
    default: return 0;
  }
}

int tv_threads(int cls) {
  switch (cls) {
    case 6: return 512;
    case 7: return 1024;
    default: return 256;
  }
}

}  // namespace

int tv_items_per_block(int cls) { return cls <= 4 ? kTvWaves : 1; }

// Workgroups resident on the whole GPU: 256 CUs, 160 KB of LDS and 2048
// threads per CU.
int tv_max_resident(int cls, int bits) {
  const int64_t lds = tv_lds_bytes(cls, bits);
  int64_t per_cu = 2048 / tv_threads(cls);
  if (lds > 0 && (160 * 1024) / lds < per_cu) per_cu = (160 * 1024) / lds;
  if (per_cu < 1) per_cu = 1;
  return (int)(256 * per_cu);
}

hipError_t launch_sweep_tv(bool off64, int cls, int bits, const SweepArgs& a, int grid,
                           hipStream_t s) {
  if (bits == 64)
    return off64 ? sweep_tv_t<int64_t, double>(cls, a, grid, s)
                 : sweep_tv_t<int32_t, double>(cls, a, grid, s);
  return off64 ? sweep_tv_t<int64_t, float>(cls, a, grid, s)
               : sweep_tv_t<int32_t, float>(cls, a, grid, s);
}

hipError_t launch_tv_hub_acc(bool off64, int bits, const HubArgs& a, void* gvals, int grid,
                             hipStream_t s) {
  if (bits == 64)
    return off64 ? tv_hub_acc_t<int64_t, double>(a, gvals, grid, s)
                 : tv_hub_acc_t<int32_t, double>(a, gvals, grid, s);
  return off64 ? tv_hub_acc_t<int64_t, float>(a, gvals, grid, s)
               : tv_hub_acc_t<int32_t, float>(a, gvals, grid, s);
}

hipError_t launch_tv_hub_select(bool off64, int bits, const HubArgs& a, void* gvals,
                                unsigned long long* vmax, uint32_t* hub_nl, int grid,
                                hipStream_t s) {
  if (bits == 64)
    return off64 ? tv_hub_select_t<int64_t, double>(a, gvals, vmax, hub_nl, grid, s)
                 : tv_hub_select_t<int32_t, double>(a, gvals, vmax, hub_nl, grid, s);
  return off64 ? tv_hub_select_t<int64_t, float>(a, gvals, vmax, hub_nl, grid, s)
               : tv_hub_select_t<int32_t, float>(a, gvals, vmax, hub_nl, grid, s);
}

}  // namespace lpa
