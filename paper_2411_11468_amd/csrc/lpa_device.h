// lpa_device.h -- device helpers for the label sweep on gfx950 (wave64).
//
//  * packed arg-max keys: (fp32 weight bits << 32) | ~label.  Weights are
//    >= 0, so their bit patterns order like the values; the complemented
//    label makes the smaller label win a tie (the reading of the "strict"
//    rule of Sec. 4 item 5 used throughout).  An empty key packs to 0, below
//    every real entry.
//  * DPP cross-lane reductions and rotations (no LDS traffic).
//  * the per-vertex hashtable of Sec. 4.2 / Algorithm 2 with a Mersenne
//    capacity p1 = 2^m - 1 and secondary modulus p2 = 2 p1 + 1 (co-prime with
//    p1), first slot k mod p1, probe step starting at 1 and updated as
//    step <- 2 step + (k mod p2) (hybrid quadratic-double probing).  After
//    max_retries probes the walk continues linearly, which visits every slot,
//    so an insert always lands and no weight is ever dropped.  The capacity
//    for a row of D entries is the smallest 2^m >= 2D, minus one: the paper
//    reserves 2D slots per vertex but sizes the table nextPow2(D) - 1, which
//    runs near full load when every neighbour label is distinct (always the
//    case in the first iteration); using the reserved 2D keeps the load at or
//    below one half.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpa_internal.h"

namespace lpa {

__device__ __forceinline__ unsigned long long pack_key(float w, uint32_t label) {
  return ((unsigned long long)__float_as_uint(w) << 32) | (unsigned long long)(~label);
}
__device__ __forceinline__ uint32_t unpack_label(unsigned long long k) {
  return ~(uint32_t)k;
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a,
                                                     unsigned long long b) {
  return a > b ? a : b;
}

// Table capacity for a row of d >= 1 entries: smallest 2^m >= 2d, minus one
// (so 2d - 1 <= p1 <= 4d - 3: load at most one half).  d <= 2^30.
__device__ __forceinline__ uint32_t table_p1(uint32_t d) {
  return (d <= 1u) ? 1u : ((1u << (32 - __clz(2u * d - 1u))) - 1u);
}

// Capacity under a load bound of 1/load for a row of d >= 1 entries in a
// table of `slots` slots (2^m - 1): load 1 = smallest 2^m > d, minus one
// (the paper's nextPow2(d) - 1: up to full load), 2 = table_p1 (the
// default: load <= 1/2), 4 = smallest 2^m >= 4d, minus one (load <= 1/4);
// never above `slots`, which every class sizes for load <= 1/2.
__device__ __forceinline__ uint32_t table_p1_load(uint32_t d, int load, uint32_t slots) {
  uint32_t p;
  if (load == 1) p = (d <= 1u) ? 1u : ((1u << (32 - __clz(d))) - 1u);
  else if (load == 4) p = table_p1(2u * d);
  else p = table_p1(d);
  return p < slots ? p : slots;
}

// ---- DPP -------------------------------------------------------------------
// dpp_ctrl encodings (GCN/CDNA): quad_perm 0x00-0xFF, row_shr:n 0x110+n,
// row_ror:n 0x120+n, row_bcast:15 0x142, row_bcast:31 0x143.
template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF, bool BOUND_ZERO = true>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, BANK_MASK,
                                               BOUND_ZERO);
}
template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF, bool BOUND_ZERO = true>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long x) {
  const uint32_t lo = dpp32<CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO>((uint32_t)x);
  const uint32_t hi = dpp32<CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO>((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
template <int CTRL>
__device__ __forceinline__ float dppf(float x) {
  return __uint_as_float(dpp32<CTRL>(__float_as_uint(x)));
}

// Max over all 64 lanes; every lane must be active.  Result is uniform.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
  x = umax64(x, dpp64<0x111>(x));             // row_shr:1
  x = umax64(x, dpp64<0x112>(x));             // row_shr:2
  x = umax64(x, dpp64<0x114>(x));             // row_shr:4
  x = umax64(x, dpp64<0x118>(x));             // row_shr:8  -> lane 15 of a row
  x = umax64(x, dpp64<0x142, 0xA>(x));        // row_bcast:15 into rows 1, 3
  x = umax64(x, dpp64<0x143, 0xC>(x));        // row_bcast:31 into rows 2, 3
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Sum over all 64 lanes of a small integer (uniform result).
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  x += dpp32<0x111>(x);
  x += dpp32<0x112>(x);
  x += dpp32<0x114>(x);
  x += dpp32<0x118>(x);
  x += dpp32<0x142, 0xA>(x);
  x += dpp32<0x143, 0xC>(x);
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Lane rank among the lanes of the wave whose bit is set in mask.
__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Max within each 16-lane row, result in every lane of the row.
__device__ __forceinline__ unsigned long long row16_max_u64(unsigned long long x) {
  x = umax64(x, dpp64<0x128>(x));  // row_ror:8
  x = umax64(x, dpp64<0x124>(x));  // row_ror:4
  x = umax64(x, dpp64<0x122>(x));  // row_ror:2
  x = umax64(x, dpp64<0x121>(x));  // row_ror:1
  return x;
}
// Max within each quad, result in every lane of the quad.
__device__ __forceinline__ unsigned long long quad_max_u64(unsigned long long x) {
  x = umax64(x, dpp64<0xB1>(x));  // quad_perm [1,0,3,2]
  x = umax64(x, dpp64<0x4E>(x));  // quad_perm [2,3,0,1]
  return x;
}

// ---- hashtable probing -------------------------------------------------------
// Probe sequences of Sec. 4.2: mode 0 quadratic-double (step 1, then
// 2*step + (k mod p2), the method's), 1 linear (step 1), 2 quadratic (step
// 1, doubled on each collision), 3 double hashing (step (k mod p2) mod p1, 1
// when that is 0).  After max_retries probes every mode continues linearly,
// which visits every slot, so an insert into a table with a free slot ends.
// Next probe slot.  t counts probes already made.  s, step < p1; r = (k mod p2)
// mod p1.
__device__ __forceinline__ void probe_next(uint32_t& s, uint32_t& step, uint32_t r,
                                           uint32_t p1, int t, ProbeCfg pc) {
  if (t < pc.max_retries) {
    if (pc.mode == 1) {
      s = (s + 1u == p1) ? 0u : s + 1u;
      return;
    }
    if (pc.mode == 3) {
      s += (r == 0u) ? 1u : r;
      if (s >= p1) s -= p1;
      return;
    }
    s += step;
    if (s >= p1) s -= p1;
    step = 2u * step + (pc.mode == 0 ? r : 0u);
    if (step >= p1) step -= p1;
    if (step >= p1) step -= p1;
  } else {
    s = (s + 1u == p1) ? 0u : s + 1u;
  }
}

// Accumulate (k, v) into an LDS table of p1 slots shared by the lanes of one
// wave or workgroup: atomic compare-and-swap claims an empty key slot, atomic
// add accumulates the weight (Algorithm 2, shared branch).
__device__ __forceinline__ void lds_accumulate(uint32_t* keys, float* vals, uint32_t p1,
                                               uint32_t k, float v, ProbeCfg pc) {
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

// lds_accumulate that also reports the slot this lane claimed for a new key
// (-1 when the key was there already), so that the caller can list the
// occupied slots instead of scanning the whole table afterwards.
__device__ __forceinline__ int32_t lds_accumulate_claim(uint32_t* keys, float* vals, uint32_t p1,
                                                        uint32_t k, float v, ProbeCfg pc) {
  const uint32_t p2 = 2u * p1 + 1u;
  uint32_t s = k % p1;
  uint32_t step = 1u % p1;
  const uint32_t r = (k % p2) % p1;
  for (int t = 0;; ++t) {
    uint32_t cur = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    bool mine = false;
    if (cur == kEmpty) {
      uint32_t expected = kEmpty;
      __hip_atomic_compare_exchange_strong(&keys[s], &expected, k, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      mine = expected == kEmpty;
      cur = mine ? k : expected;
    }
    if (cur == k) {
      __hip_atomic_fetch_add(&vals[s], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return mine ? (int32_t)s : -1;
    }
    probe_next(s, step, r, p1, t, pc);
  }
}

// Append the slots the lanes of one wave claimed (claimed >= 0) to a list
// of occupied slots: one LDS atomic per wave on the list's length.  Entries
// past cap are not stored (the length still counts them: a caller whose
// list overflowed reads back the whole table).
__device__ __forceinline__ void list_claimed(int32_t claimed, uint16_t* lst, uint32_t* lst_n,
                                             uint32_t cap = 0xFFFFFFFFu) {
  const unsigned long long m = __ballot(claimed >= 0);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int first = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == first)
    base = __hip_atomic_fetch_add(lst_n, (uint32_t)__popcll(m), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
  base = (uint32_t)__shfl((int)base, first);
  const uint32_t pos = base + lane_rank(m);
  if (claimed >= 0 && pos < cap) lst[pos] = (uint16_t)claimed;
}

// Accumulate (k, v) into a global-memory table; returns the slot and the
// value the slot holds after this add (values only grow, so the largest value
// ever returned for a key is its final sum).  SCOPE is the atomics' memory
// scope: agent when workgroups on several XCDs share the table, workgroup when
// every access comes from one XCD (the atomics then resolve in its L2).
template <int SCOPE>
__device__ __forceinline__ uint32_t global_accumulate(uint32_t* keys, float* vals,
                                                      uint32_t p1, uint32_t k, float v,
                                                      ProbeCfg pc, float* after) {
  const uint32_t p2 = 2u * p1 + 1u;
  uint32_t s = k % p1;
  uint32_t step = 1u % p1;
  const uint32_t r = (k % p2) % p1;
  for (int t = 0;; ++t) {
    uint32_t cur = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, SCOPE);
    if (cur == kEmpty) {
      uint32_t expected = kEmpty;
      __hip_atomic_compare_exchange_strong(&keys[s], &expected, k, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, SCOPE);
      cur = (expected == kEmpty) ? k : expected;
    }
    if (cur == k) {
      const float old = __hip_atomic_fetch_add(&vals[s], v, __ATOMIC_RELAXED, SCOPE);
      *after = old + v;
      return s;
    }
    probe_next(s, step, r, p1, t, pc);
  }
}

// ---- shared by the sweep kernels (sweep.hip, queue.hip) ----------------------
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
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


// Adds a workgroup's counters to the iteration's: sums over each wave, then
// over the waves in LDS, then one device atomic per counter and workgroup
// (atomics on one address from every wave of a full grid serialise at the
// memory side: tens of microseconds per kernel).  Every thread of the
// workgroup calls it, at the end of the kernel.
__device__ __forceinline__ void flush_stats(unsigned long long edges, uint32_t changed,
                                            unsigned long long flagw, DevStats* st,
                                            int cls) {
  __shared__ unsigned long long fs_e[16], fs_f[16];
  __shared__ uint32_t fs_c[16];
  const unsigned long long e = wave_sum_u64(edges);
  const uint32_t c = wave_sum_u32(changed);
  const unsigned long long f = wave_sum_u64(flagw);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    fs_e[w] = e;
    fs_c[w] = c;
    fs_f[w] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long te = 0, tf = 0;
    uint32_t tc = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      te += fs_e[q];
      tc += fs_c[q];
      tf += fs_f[q];
    }
    if (te) atomicAdd(&st->edges[cls], te);
    if (tc) atomicAdd(&st->changed[cls], (unsigned long long)tc);
    if (tf) atomicAdd(&st->flagw[cls], tf);
  }
}

// Wave-level merge before the LDS inserts of one unrolled step: the lanes
// holding the same label as the wave's first lane with an entry hand their
// weights to that lane (a popcount for unit weights, else a wave sum) and
// drop their own entries.  Atomic adds to one LDS slot from one wave
// instruction are serialised; after the first iteration a row's labels
// concentrate on a few values, and the first lane's label is most often the
// step's most frequent one.  The table then receives the same per-label sums
// (exactly so for integer weights).  All 64 lanes must be active.
__device__ __forceinline__ void merge_lead(uint32_t& lab, float& wt, bool unit) {
  const unsigned long long act = __ballot(lab != kEmpty);
  if (act == 0ull) return;
  const int first = __ffsll((long long)act) - 1;
  const uint32_t lead = (uint32_t)__builtin_amdgcn_readlane((int)lab, first);
  const bool mine = lab == lead;
  const unsigned long long m = __ballot(mine);
  float sum;
  if (unit) {
    sum = (float)__popcll(m);
  } else {
    float x = mine ? wt : 0.0f;
    for (int ofs = 32; ofs > 0; ofs >>= 1) x += __shfl_xor(x, ofs);
    sum = x;
  }
  if (mine) {
    if ((int)(threadIdx.x & 63) == first) wt = sum;
    else lab = kEmpty;
  }
}

// merge_lead within each 16-lane row, for k_sweep_group (one row per vertex;
// the lanes of a row are active or inactive together).
__device__ __forceinline__ void merge_lead16(uint32_t& lab, float& wt, bool unit) {
  const unsigned long long act = __ballot(lab != kEmpty);
  const int lane = (int)(threadIdx.x & 63);
  const int row0 = lane & ~15;
  const uint32_t ract = (uint32_t)(act >> row0) & 0xFFFFu;
  const int first = row0 + (ract ? __ffs((int)ract) - 1 : 0);
  const uint32_t lead = (uint32_t)__shfl((int)lab, first);
  const bool mine = ract != 0u && lab == lead;
  const unsigned long long m = __ballot(mine);
  float sum;
  if (unit) {
    sum = (float)__popc((uint32_t)(m >> row0) & 0xFFFFu);
  } else {
    float x = mine ? wt : 0.0f;
    x += dppf<0x128>(x);  // row_ror:8
    x += dppf<0x124>(x);
    x += dppf<0x122>(x);
    x += dppf<0x121>(x);
    sum = x;
  }
  if (mine) {
    if (lane == first) wt = sum;
    else lab = kEmpty;
  }
}

__device__ __forceinline__ bool decide(unsigned long long best, int32_t cur, int pl,
                                       uint32_t* cstar) {
  if (best == 0ull) return false;  // no neighbour other than itself
  const uint32_t c = unpack_label(best);
  *cstar = c;
  return (int32_t)c != cur && (!pl || (int32_t)c < cur);
}

// Index of the accelerator complex die (XCD) this wave runs on.
__device__ __forceinline__ uint32_t xcc_id() {
  uint32_t x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  return x & (uint32_t)(kXcds - 1);
}

template <typename OffT>
__device__ __forceinline__ void row_of(const void* off, int32_t v, int64_t* o, int64_t* d) {
  const OffT* p = reinterpret_cast<const OffT*>(off);
  const int64_t a = (int64_t)p[v];
  const int64_t b = (int64_t)p[v + 1];
  *o = a;
  *d = b - a;
}

// A wave-uniform index pinned to a VGPR.  The result of a load from a
// uniform address is moved into SGPRs, which waits for the load there and
// then; a load through this index stays a vector load whose result stays in
// VGPRs until it is read, so that it can be issued a whole row ahead.
__device__ __forceinline__ uint32_t vgpr_u32(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The first lane's value of x (wave-uniform values held in VGPRs).
__device__ __forceinline__ int32_t first_lane_i32(int32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ int64_t first_lane_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A row's start and end offsets, left unsubtracted so that nothing waits for
// the loads until the row is processed.
template <typename OffT>
__device__ __forceinline__ void row_bounds(const void* off, int32_t v, int64_t* o, int64_t* e) {
  const OffT* p = reinterpret_cast<const OffT*>(off);
  *o = (int64_t)p[v];
  *e = (int64_t)p[v + 1];
}

// Targets and weights are read once per sweep: streaming (non-temporal)
// loads keep them from displacing the gathered labels in the caches.
__device__ __forceinline__ float edge_weight(const float* w, int64_t e) {
  return w ? __builtin_nontemporal_load(&w[e]) : 1.0f;
}

}  // namespace lpa
