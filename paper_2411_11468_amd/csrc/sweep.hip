// sweep.hip -- the per-vertex label sweep (one iteration of lpaMove,
// Algorithm 1) for gfx950, split by degree class.
//
// Every kernel processes the active vertices of its class (built by the
// frontier kernel) and, per vertex i:
//   1. sums the weight towards each neighbour label, skipping self-loops
//      (Eq. 3; Algorithm 1 neighbour scan, Algorithm 2 accumulation),
//   2. takes the label of maximum sum, smallest label on ties,
//   3. moves if the label differs and, under Pick-Less, is strictly smaller
//      (Sec. 4.1),
//   4. on a move, records the change (one byte per vertex) and counts it;
//      the neighbours of changed vertices are flagged for the next iteration
//      (Sec. 4 item 4) after the sweep, by the flag kernels of graph.hip.
// In asynchronous mode the new label is stored in place; in deterministic
// mode it is queued and applied after the sweep, so every vertex reads the
// iteration-start labels.  In the first iteration of a run that starts from
// labels = vertex ids (Algorithm 1's initialisation) a neighbour's label is
// its id and is not gathered: the deterministic result is unchanged, and in
// asynchronous mode this is the read of the iteration-start value, which an
// asynchronous sweep is free to make.  When, moreover, every row's targets
// strictly increase (checked once at create), the host runs that first sweep
// with k_sweep_direct / k_hub_direct, which need no table.  Flags are cleared only by the frontier kernel
// before the sweep and set only after it, so a neighbour that read an old
// label is always flagged for the next iteration and no fence is needed
// between a label store and anything else.  (An agent-scope fence would
// also write back the XCD's L2 on every move.)
//
// Classes:
//   k_sweep_lane4     rows of up to 4 entries, one lane per row, sums in
//                     registers (learned variant: k_sweep_small<4>).
//   k_sweep_small<G>  G lanes per vertex (G = 4 or 16), one edge per lane,
//                     per-label sums by DPP rotations inside the group; no
//                     hashtable is needed for rows this short.
//   k_sweep_group     rows of up to 64 entries, 16 lanes and an LDS table per
//                     vertex, four vertices per wave.
//   k_sweep_wave_pipe  one wave per vertex, LDS hashtable per wave, the next
//                     row's head loaded during the table scan.
//   k_sweep_block(_pipe)  one workgroup per vertex, LDS hashtable per
//                     workgroup; the _pipe forms load the next row's head
//                     during the table scan.
//   k_hub_part/reduce/spill/fin   rows longer than the largest LDS table:
//                     each slice of the row is reduced in an LDS table and
//                     its (label, sum) pairs written grouped by label bucket;
//                     each bucket is summed in an LDS table (a full table
//                     spills into the hub's global table) and its maximum
//                     folded into the hub's packed best; k_hub_fin moves.
#include "lpa_device.h"
#include "lpa_record.h"

namespace lpa {

namespace {

// One rotation step of the per-label sums inside a 16-lane row (R) or a quad
// (quad_perm Q): add the other lane's weight if it holds the same label.
// FEAT: also count the lanes holding the lane's label (its multiplicity).
template <int R, bool FEAT>
__device__ __forceinline__ void rot16_accum(uint32_t lab, float wt, float& sum, float& mult) {
  const uint32_t ol = dpp32<0x120 + R, 0xF, 0xF, false>(lab);
  const float ow = __uint_as_float(dpp32<0x120 + R, 0xF, 0xF, false>(__float_as_uint(wt)));
  if (ol == lab) {
    sum += ow;
    if constexpr (FEAT) mult += 1.0f;
  }
}
template <int Q, bool FEAT>
__device__ __forceinline__ void rot4_accum(uint32_t lab, float wt, float& sum, float& mult) {
  const uint32_t ol = dpp32<Q, 0xF, 0xF, false>(lab);
  const float ow = __uint_as_float(dpp32<Q, 0xF, 0xF, false>(__float_as_uint(wt)));
  if (ol == lab) {
    sum += ow;
    if constexpr (FEAT) mult += 1.0f;
  }
}

// Reductions over a group of G = 4 (quad) or 16 (row) lanes, result in every
// lane of the group.
template <int G>
__device__ __forceinline__ unsigned long long group_max(unsigned long long x) {
  if constexpr (G == 16) return row16_max_u64(x);
  else return quad_max_u64(x);
}
template <int G>
__device__ __forceinline__ float group_sum_f32(float x) {
  if constexpr (G == 16) {
    x += dppf<0x128>(x);  // row_ror:8
    x += dppf<0x124>(x);
    x += dppf<0x122>(x);
    x += dppf<0x121>(x);
  } else {
    x += dppf<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dppf<0x4E>(x);   // quad_perm [2,3,0,1]
  }
  return x;
}
template <int G>
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t x) {
  if constexpr (G == 16) {
    x += dpp32<0x128>(x);
    x += dpp32<0x124>(x);
    x += dpp32<0x122>(x);
    x += dpp32<0x121>(x);
  } else {
    x += dpp32<0xB1>(x);
    x += dpp32<0x4E>(x);
  }
  return x;
}

// fp32 sum over the wave (uniform result).
__device__ __forceinline__ float wave_sum_f32(float x) {
  for (int ofs = 32; ofs > 0; ofs >>= 1) x += __shfl_xor(x, ofs);
  return x;
}

// The learned variant's false-negative count, one atomic per workgroup as in
// flush_stats (every thread calls it, at the end of the kernel).
__device__ __forceinline__ void flush_fneg(uint32_t fneg, DevStats* st) {
  __shared__ uint32_t fn_w[16];
  const uint32_t f = wave_sum_u32(fneg);
  if ((threadIdx.x & 63) == 0) fn_w[threadIdx.x >> 6] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += fn_w[q];
    if (t) atomicAdd(&st->fneg, (unsigned long long)t);
  }
}

}  // namespace

// ---- small rows: G lanes per vertex, registers only -------------------------
// FEAT: the learned variant, which also rewrites the state record of every
// vertex it evaluates (lpa_record.h).
template <typename OffT, int G, bool FEAT>
__global__ __launch_bounds__(256) void k_sweep_small(SweepArgs a) {
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int lane = threadIdx.x & 63;
  const int k = lane & (G - 1);
  const uint32_t count = a.st->active[a.cls];
  const int l = a.st->iter;
  constexpr uint32_t kVpw = 64 / G;
  const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0, my_fneg = 0;
  for (uint64_t base = (uint64_t)wave_id * kVpw; base < count;
       base += (uint64_t)nwaves * kVpw) {
    const uint64_t idx = base + (uint32_t)lane / G;
    const bool valid = idx < count;
    int32_t v = valid ? a.active[idx] : 0;
    int64_t o = 0, d = 0;
    if (valid) row_of<OffT>(a.off, v, &o, &d);
    [[maybe_unused]] const unsigned long long rold = (FEAT && valid && k == 0) ? a.rec[v] : 0ull;
    const bool has = valid && k < d;
    const int32_t j = has ? __builtin_nontemporal_load(&a.tgt[o + k]) : -1;
    const float wt = has ? edge_weight(a.w, o + k) : 0.0f;
    uint32_t lab = kEmpty;
    if (has && j != v) lab = id0 ? (uint32_t)j : (uint32_t)a.C[j];
    // Per-label sum seen from this lane: its own weight plus every other lane
    // of the group holding the same label.  FEAT: mult = lanes holding it.
    float sum = wt, mult = 1.0f;
    if constexpr (G == 16) {
      rot16_accum<1, FEAT>(lab, wt, sum, mult);  rot16_accum<2, FEAT>(lab, wt, sum, mult);
      rot16_accum<3, FEAT>(lab, wt, sum, mult);  rot16_accum<4, FEAT>(lab, wt, sum, mult);
      rot16_accum<5, FEAT>(lab, wt, sum, mult);  rot16_accum<6, FEAT>(lab, wt, sum, mult);
      rot16_accum<7, FEAT>(lab, wt, sum, mult);  rot16_accum<8, FEAT>(lab, wt, sum, mult);
      rot16_accum<9, FEAT>(lab, wt, sum, mult);  rot16_accum<10, FEAT>(lab, wt, sum, mult);
      rot16_accum<11, FEAT>(lab, wt, sum, mult); rot16_accum<12, FEAT>(lab, wt, sum, mult);
      rot16_accum<13, FEAT>(lab, wt, sum, mult); rot16_accum<14, FEAT>(lab, wt, sum, mult);
      rot16_accum<15, FEAT>(lab, wt, sum, mult);
    } else {
      rot4_accum<0x39, FEAT>(lab, wt, sum, mult);  // quad_perm [1,2,3,0]
      rot4_accum<0x4E, FEAT>(lab, wt, sum, mult);  // quad_perm [2,3,0,1]
      rot4_accum<0x93, FEAT>(lab, wt, sum, mult);  // quad_perm [3,0,1,2]
    }
    const unsigned long long packed = (lab != kEmpty) ? pack_key(sum, lab) : 0ull;
    const unsigned long long best = group_max<G>(packed);
    uint32_t cstar = 0;
    const int32_t cur = valid ? a.C[v] : 0;
    const bool moved = valid && decide(best, cur, pl, &cstar);
    const bool leader = valid && k == 0;
    if constexpr (FEAT) {
      // every lane takes part in the group reductions
      const float K = group_sum_f32<G>(lab != kEmpty ? wt : 0.0f);
      const unsigned long long ownk =
          (lab != kEmpty && (int32_t)lab == cur) ? (unsigned long long)__float_as_uint(sum) : 0ull;
      const float own = __uint_as_float((uint32_t)group_max<G>(ownk));
      const uint32_t bl = best ? unpack_label(best) : kEmpty;
      const unsigned long long sk = (lab != kEmpty && lab != bl) ? pack_key(sum, lab) : 0ull;
      const float second = __uint_as_float((uint32_t)(group_max<G>(sk) >> 32));
      const float bw = __uint_as_float((uint32_t)(best >> 32));
      // each label's lanes contribute 1/mult each: the group sum is the
      // number of distinct labels up to rounding (at most 16 terms)
      const uint32_t distinct =
          (uint32_t)rintf(group_sum_f32<G>(lab != kEmpty ? 1.0f / mult : 0.0f));
      if (leader && d >= 1)
        my_fneg += rec_write(a.rec, v, rold, l, K, own, bw, second, distinct, (uint32_t)d, moved);
    }
    if (leader) {
      if (a.async_mode) {
        if (moved) a.C[v] = (int32_t)cstar;
      } else {
        a.Cn[v] = moved ? (int32_t)cstar : cur;
      }
    }
    if (moved && leader) a.chg[v] = 1;
    if (leader) {
      my_edges += (unsigned long long)d;
      my_changed += moved ? 1u : 0u;
      my_flagw += moved ? (unsigned long long)d : 0ull;
    }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
  if constexpr (FEAT) flush_fneg(my_fneg, a.st);
}

// Plain k_sweep_small<16> with R wave steps in flight (three; two gained
// less): the list entries, offsets, targets and neighbour labels of all R
// steps are loaded before any is reduced (a step is a chain of four
// dependent loads).
template <typename OffT>
__global__ __launch_bounds__(256) void k_sweep_small16x2(SweepArgs a) {
  constexpr int G = 16, R = 3;
  constexpr uint32_t kVpw = 64 / G;
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int lane = threadIdx.x & 63;
  const int k = lane & (G - 1);
  const uint32_t count = a.st->active[a.cls];
  const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0;
  for (uint64_t base = (uint64_t)wave_id * kVpw; base < count;
       base += (uint64_t)R * nwaves * kVpw) {
    bool valid[R];
    int32_t v[R], j[R];
    int64_t o[R], d[R];
    float wt[R];
    uint32_t lab[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t idx = base + (uint64_t)r * nwaves * kVpw + (uint32_t)lane / G;
      valid[r] = idx < count;
      v[r] = valid[r] ? a.active[idx] : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      o[r] = 0;
      d[r] = 0;
      if (valid[r]) row_of<OffT>(a.off, v[r], &o[r], &d[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool has = valid[r] && k < d[r];
      j[r] = has ? __builtin_nontemporal_load(&a.tgt[o[r] + k]) : -1;
      wt[r] = has ? edge_weight(a.w, o[r] + k) : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      lab[r] = kEmpty;
      if (j[r] >= 0 && j[r] != v[r]) lab[r] = id0 ? (uint32_t)j[r] : (uint32_t)a.C[j[r]];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float sum = wt[r], mult = 1.0f;
      rot16_accum<1, false>(lab[r], wt[r], sum, mult);  rot16_accum<2, false>(lab[r], wt[r], sum, mult);
      rot16_accum<3, false>(lab[r], wt[r], sum, mult);  rot16_accum<4, false>(lab[r], wt[r], sum, mult);
      rot16_accum<5, false>(lab[r], wt[r], sum, mult);  rot16_accum<6, false>(lab[r], wt[r], sum, mult);
      rot16_accum<7, false>(lab[r], wt[r], sum, mult);  rot16_accum<8, false>(lab[r], wt[r], sum, mult);
      rot16_accum<9, false>(lab[r], wt[r], sum, mult);  rot16_accum<10, false>(lab[r], wt[r], sum, mult);
      rot16_accum<11, false>(lab[r], wt[r], sum, mult); rot16_accum<12, false>(lab[r], wt[r], sum, mult);
      rot16_accum<13, false>(lab[r], wt[r], sum, mult); rot16_accum<14, false>(lab[r], wt[r], sum, mult);
      rot16_accum<15, false>(lab[r], wt[r], sum, mult);
      const unsigned long long packed = (lab[r] != kEmpty) ? pack_key(sum, lab[r]) : 0ull;
      const unsigned long long best = row16_max_u64(packed);
      uint32_t cstar = 0;
      const int32_t cur = valid[r] ? a.C[v[r]] : 0;
      const bool moved = valid[r] && decide(best, cur, pl, &cstar);
      if (valid[r] && k == 0) {
        if (a.async_mode) {
          if (moved) a.C[v[r]] = (int32_t)cstar;
        } else {
          a.Cn[v[r]] = moved ? (int32_t)cstar : cur;
        }
        if (moved) a.chg[v[r]] = 1;
        my_edges += (unsigned long long)d[r];
        my_changed += moved ? 1u : 0u;
        my_flagw += moved ? (unsigned long long)d[r] : 0ull;
      }
    }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
}

// ---- rows of at most 4 entries: one lane per vertex -------------------------
// Plain variant for the smallest class: each lane loads its rows' (up to 4)
// targets, weights and labels at once and sums equal labels among them in
// registers.  A lane takes two rows per step (the second one grid-stride
// further), so that a wave has 128 rows' reads in flight.
template <typename OffT>
__global__ __launch_bounds__(256) void k_sweep_lane4(SweepArgs a) {
  constexpr int R = 2;  // rows per lane and step
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0;
  const uint64_t T = (uint64_t)gridDim.x * 256;
  for (uint64_t idx0 = (uint64_t)blockIdx.x * 256 + threadIdx.x; idx0 < count; idx0 += R * T) {
    int32_t v[R], j[R][4], cur[R];
    int64_t o[R], d[R];
    float wt[R][4];
    uint32_t lab[R][4];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      valid[r] = idx0 + r * T < count;
      v[r] = valid[r] ? a.active[idx0 + r * T] : 0;
      o[r] = 0;
      d[r] = 0;
      if (valid[r]) row_of<OffT>(a.off, v[r], &o[r], &d[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool has = u < d[r];
        j[r][u] = has ? __builtin_nontemporal_load(&a.tgt[o[r] + u]) : v[r];
        wt[r][u] = has ? edge_weight(a.w, o[r] + u) : 0.0f;
      }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        lab[r][u] = (j[r][u] != v[r]) ? (id0 ? (uint32_t)j[r][u] : (uint32_t)a.C[j[r][u]]) : kEmpty;
      cur[r] = valid[r] ? a.C[v[r]] : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!valid[r]) continue;
      unsigned long long best = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (lab[r][u] == kEmpty) continue;
        float sum = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) sum += (lab[r][q] == lab[r][u]) ? wt[r][q] : 0.0f;
        best = umax64(best, pack_key(sum, lab[r][u]));
      }
      uint32_t cstar = 0;
      const bool moved = decide(best, cur[r], pl, &cstar);
      if (a.async_mode) {
        if (moved) a.C[v[r]] = (int32_t)cstar;
      } else {
        a.Cn[v[r]] = moved ? (int32_t)cstar : cur[r];
      }
      if (moved) a.chg[v[r]] = 1;
      my_edges += (unsigned long long)d[r];
      my_changed += moved ? 1u : 0u;
      my_flagw += moved ? (unsigned long long)d[r] : 0ull;
    }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
}

// Learned variant, table kernels: per-lane partials of the record quantities
// gathered while the table is read back (each slot holds one label).
struct RecPartial {
  unsigned long long b1 = 0, b2 = 0;  // two largest packed keys of the lane
  float own = 0.0f;                   // weight of the vertex's own label
  float K = 0.0f;                     // lane's share of the total weight
  uint32_t distinct = 0;              // occupied slots read by the lane
  __device__ __forceinline__ void slot(unsigned long long pk, uint32_t key, float val,
                                       int32_t cur) {
    if (pk > b1) { b2 = b1; b1 = pk; } else if (pk > b2) { b2 = pk; }
    if ((int32_t)key == cur) own = val;
    ++distinct;
  }
};

// ---- one wave per vertex, next row's head loaded during the table scan ------
// Rows of 65-512 entries, one wave per vertex; the wave issues the
// loads of its next vertex (list entry, row offsets, first 64U targets and
// weights) before it scans and clears the current vertex's table, so that
// those loads are in flight while the scan runs.  Labels are not
// prefetched: they are read when the row is accumulated, as before.
// FEAT: the learned variant, which also rewrites the state record.
template <typename OffT, int SLOTS, int WAVES, int U, bool FEAT>
__global__ __launch_bounds__(WAVES * 64) void k_sweep_wave_pipe(SweepArgs a) {
  __shared__ uint32_t keys_all[WAVES][SLOTS];
  __shared__ float vals_all[WAVES][SLOTS];
  // per wave: the slots its current row claimed, read back instead of all
  // p1 slots (a row holds at most (SLOTS + 1) / 2 labels); the count is
  // wave-uniform and lives in a register
  __shared__ uint16_t lst_all[WAVES][(SLOTS + 1) / 2];
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int l = a.st->iter;
  uint32_t* keys = keys_all[wv];
  float* vals = vals_all[wv];
  uint16_t* lst = lst_all[wv];
  uint32_t nl = 0;
  auto claim = [&](int32_t cl) {
    const unsigned long long m = __ballot(cl >= 0);
    if (cl >= 0) lst[nl + lane_rank(m)] = (uint16_t)cl;
    nl += (uint32_t)__popcll(m);
  };
  for (int s = lane; s < SLOTS; s += 64) { keys[s] = kEmpty; vals[s] = 0.0f; }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const uint32_t count = a.st->active[a.cls];
  const uint32_t stride = gridDim.x * WAVES;
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0, my_fneg = 0;
  int32_t vq = 0, j[U];  // the current row's vertex and offsets
  int64_t oq = 0, eq = 0;
  float wt[U];
  // a row's first 64*U targets and weights, its offsets known
  auto head = [&](int32_t hv, int64_t ho, int64_t hd, int32_t* hj, float* hw) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = u * 64 + lane;
      const bool has = e < hd;
      hj[u] = has ? __builtin_nontemporal_load(&a.tgt[ho + e]) : hv;
      hw[u] = has ? edge_weight(a.w, ho + e) : 0.0f;
    }
  };
  uint32_t item = blockIdx.x * WAVES + wv;
  if (item < count) {
    vq = first_lane_i32(a.active[vgpr_u32(item)]);
    row_bounds<OffT>(a.off, vq, &oq, &eq);
    oq = first_lane_i64(oq);
    eq = first_lane_i64(eq);
    head(vq, oq, eq - oq, j, wt);
  }
  // the next row's list entry and offsets (v1, o1, e1): loaded one row
  // earlier than its targets, so that neither dependent load waits in line
  // before the table scan
  int32_t v1 = 0;
  int64_t o1 = 0, e1 = 0;
  if (item + stride < count) {
    v1 = first_lane_i32(a.active[vgpr_u32(item + stride)]);
    row_bounds<OffT>(a.off, v1, &o1, &e1);
    o1 = first_lane_i64(o1);
    e1 = first_lane_i64(e1);
  }
  while (item < count) {
    const int32_t v = vq;
    const int64_t o = oq, d = eq - o;
    const uint32_t nitem = item + stride;
    const uint32_t n2item = nitem + stride;
    const int32_t v2 = n2item < count ? a.active[vgpr_u32(n2item)] : 0;
    // own label, a vector load: used only by the decision at the row's end
    const int32_t cur = a.C[vgpr_u32((uint32_t)v)];
    [[maybe_unused]] const unsigned long long rold = (FEAT && lane == 0) ? a.rec[v] : 0ull;
    const uint32_t p1 = table_p1_load((uint32_t)d, a.tload, (uint32_t)SLOTS);
    RecPartial rp;
    uint32_t lab[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      lab[u] = (j[u] != v) ? (id0 ? (uint32_t)j[u] : (uint32_t)a.C[j[u]]) : kEmpty;
    #pragma unroll
    for (int u = 0; u < U; ++u) merge_lead(lab[u], wt[u], a.w == nullptr);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int32_t cl = -1;
      if (lab[u] != kEmpty) {
        cl = lds_accumulate_claim(keys, vals, p1, lab[u], wt[u], a.probe);
        if constexpr (FEAT) rp.K += wt[u];
      }
      claim(cl);
    }
    for (int64_t base = 64 * U; base < d; base += 64 * U) {
      int32_t jj[U];
      float ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = base + u * 64 + lane;
        const bool has = e < d;
        jj[u] = has ? __builtin_nontemporal_load(&a.tgt[o + e]) : v;
        ww[u] = has ? edge_weight(a.w, o + e) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        lab[u] = (jj[u] != v) ? (id0 ? (uint32_t)jj[u] : (uint32_t)a.C[jj[u]]) : kEmpty;
      #pragma unroll
      for (int u = 0; u < U; ++u) merge_lead(lab[u], ww[u], a.w == nullptr);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int32_t cl = -1;
        if (lab[u] != kEmpty) {
          cl = lds_accumulate_claim(keys, vals, p1, lab[u], ww[u], a.probe);
          if constexpr (FEAT) rp.K += ww[u];
        }
        claim(cl);
      }
    }
    // next vertex's head and the offsets of the one after, in flight during
    // the scan below
    int32_t nj[U];
    float nw[U];
    if (nitem < count) head(v1, o1, e1 - o1, nj, nw);
    int64_t o2 = 0, e2 = 0;
    if (n2item < count) row_bounds<OffT>(a.off, v2, &o2, &e2);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long best = 0;
    for (uint32_t i = lane; i < nl; i += 64) {
      const uint32_t s = lst[i];
      const uint32_t kk = keys[s];
      const unsigned long long pk = pack_key(vals[s], kk);
      if constexpr (FEAT) rp.slot(pk, kk, vals[s], cur);
      best = umax64(best, pk);
      keys[s] = kEmpty;
      vals[s] = 0.0f;
    }
    nl = 0;
    best = wave_max_u64(best);
    uint32_t cstar = 0;
    const bool moved = decide(best, cur, pl, &cstar);
    if constexpr (FEAT) {
      const float second =
          __uint_as_float((uint32_t)(wave_max_u64(rp.b1 == best ? rp.b2 : rp.b1) >> 32));
      const float own = __uint_as_float((uint32_t)wave_max_u64(__float_as_uint(rp.own)));
      const uint32_t distinct = wave_sum_u32(rp.distinct);
      const float K = wave_sum_f32(rp.K);
      if (lane == 0)
        my_fneg += rec_write(a.rec, v, rold, l, K, own, __uint_as_float((uint32_t)(best >> 32)),
                             second, distinct, (uint32_t)d, moved);
    }
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
    item = nitem;
    vq = v1; oq = o1; eq = e1;
    // complete by now (the rotation of the head's registers waits for them)
    v1 = first_lane_i32(v2);
    o1 = first_lane_i64(o2);
    e1 = first_lane_i64(e2);
#pragma unroll
    for (int u = 0; u < U; ++u) { j[u] = nj[u]; wt[u] = nw[u]; }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
  if constexpr (FEAT) flush_fneg(my_fneg, a.st);
}

// ---- G lanes per vertex, LDS table per lane group ----------------------------
// Rows of up to 4G entries: a wave takes 64/G vertices at once, each group of
// G lanes with a table of its own, so that four rows' label reads are in
// flight per wave where the one-wave-per-vertex kernel has one.  G = 16 is
// one DPP row, whose reductions stay inside the group.  FEAT: the learned
// variant, which also reduces the record quantities over the group.
template <typename OffT, int SLOTS, int G, bool FEAT>
__global__ __launch_bounds__(256) void k_sweep_group(SweepArgs a) {
  static_assert(G == 16, "group reductions are DPP-row wide");
  constexpr int NG = 256 / G;
  constexpr int U = 4;
  __shared__ uint32_t keys_all[NG][SLOTS];
  __shared__ float vals_all[NG][SLOTS];
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int tid = threadIdx.x;
  const int gi = tid / G, k = tid & (G - 1);
  [[maybe_unused]] const int l = a.st->iter;
  uint32_t* keys = keys_all[gi];
  float* vals = vals_all[gi];
  for (int s = k; s < SLOTS; s += G) { keys[s] = kEmpty; vals[s] = 0.0f; }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0, my_fneg = 0;
  // the 16 lanes of a group are active or inactive together
  for (uint64_t item = (uint64_t)blockIdx.x * NG + gi; item < count;
       item += (uint64_t)gridDim.x * NG) {
    const int32_t v = a.active[item];
    int64_t o, d;
    row_of<OffT>(a.off, v, &o, &d);
    const int32_t cur = a.C[v];
    [[maybe_unused]] const unsigned long long rold = (FEAT && k == 0) ? a.rec[v] : 0ull;
    const uint32_t p1 = table_p1_load((uint32_t)d, a.tload, (uint32_t)SLOTS);
    RecPartial rp;
    for (int64_t base = 0; base < d; base += G * U) {
      int32_t j[U];
      float wt[U];
      uint32_t lab[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = base + u * G + k;
        const bool has = e < d;
        j[u] = has ? __builtin_nontemporal_load(&a.tgt[o + e]) : v;
        wt[u] = has ? edge_weight(a.w, o + e) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        lab[u] = (j[u] != v) ? (id0 ? (uint32_t)j[u] : (uint32_t)a.C[j[u]]) : kEmpty;
#pragma unroll
      for (int u = 0; u < U; ++u) merge_lead16(lab[u], wt[u], a.w == nullptr);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (lab[u] != kEmpty) {
          lds_accumulate(keys, vals, p1, lab[u], wt[u], a.probe);
          if constexpr (FEAT) rp.K += wt[u];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long best = 0;
    for (uint32_t s = k; s < p1; s += G) {
      const uint32_t kk = keys[s];
      if (kk != kEmpty) {
        const unsigned long long pk = pack_key(vals[s], kk);
        if constexpr (FEAT) rp.slot(pk, kk, vals[s], cur);
        best = umax64(best, pk);
        keys[s] = kEmpty;
        vals[s] = 0.0f;
      }
    }
    best = row16_max_u64(best);
    uint32_t cstar = 0;
    const bool moved = decide(best, cur, pl, &cstar);
    if constexpr (FEAT) {
      const float second =
          __uint_as_float((uint32_t)(row16_max_u64(rp.b1 == best ? rp.b2 : rp.b1) >> 32));
      const float own = __uint_as_float((uint32_t)row16_max_u64(__float_as_uint(rp.own)));
      const uint32_t distinct = group_sum_u32<G>(rp.distinct);
      const float K = group_sum_f32<G>(rp.K);
      if (k == 0)
        my_fneg += rec_write(a.rec, v, rold, l, K, own, __uint_as_float((uint32_t)(best >> 32)),
                             second, distinct, (uint32_t)d, moved);
    }
    if (k == 0) {
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
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
  if constexpr (FEAT) flush_fneg(my_fneg, a.st);
}

// ---- one workgroup per vertex, LDS table per workgroup ---------------------
template <typename OffT, int SLOTS, int BT, int U, bool FEAT>
__global__ __launch_bounds__(BT) void k_sweep_block(SweepArgs a) {
  constexpr int NW = BT / 64;
  __shared__ uint32_t keys[SLOTS];
  __shared__ float vals[SLOTS];
  __shared__ unsigned long long red[NW];
  __shared__ unsigned long long red2[FEAT ? NW : 1], redo[FEAT ? NW : 1];
  __shared__ uint32_t redc[FEAT ? NW : 1];
  __shared__ float redk[FEAT ? NW : 1];
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int l = a.st->iter;
  for (int s = tid; s < SLOTS; s += BT) { keys[s] = kEmpty; vals[s] = 0.0f; }
  __syncthreads();
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0, my_fneg = 0;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const int32_t v = a.active[item];
    int64_t o, d;
    row_of<OffT>(a.off, v, &o, &d);
    // Own label, read before the barriers below: in asynchronous mode thread 0
    // overwrites it, and every thread must reach the same move decision.
    const int32_t cur = a.C[v];
    [[maybe_unused]] const unsigned long long rold = (FEAT && tid == 0) ? a.rec[v] : 0ull;
    const uint32_t p1 = table_p1_load((uint32_t)d, a.tload, (uint32_t)SLOTS);
    RecPartial rp;
    unsigned long long best = 0;
    for (int64_t base = 0; base < d; base += (int64_t)BT * U) {
      int32_t j[U];
      float wt[U];
      uint32_t lab[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = base + u * BT + tid;
        const bool has = e < d;
        j[u] = has ? __builtin_nontemporal_load(&a.tgt[o + e]) : v;
        wt[u] = has ? edge_weight(a.w, o + e) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        lab[u] = (j[u] != v) ? (id0 ? (uint32_t)j[u] : (uint32_t)a.C[j[u]]) : kEmpty;
      // rows sorted by target put runs of equal labels into one wave's lanes
#pragma unroll
      for (int u = 0; u < U; ++u) merge_lead(lab[u], wt[u], a.w == nullptr);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (lab[u] != kEmpty) {
          lds_accumulate(keys, vals, p1, lab[u], wt[u], a.probe);
          if constexpr (FEAT) rp.K += wt[u];
        }
    }
    __syncthreads();
    for (uint32_t s = tid; s < p1; s += BT) {
      const uint32_t kk = keys[s];
      if (kk != kEmpty) {
        const unsigned long long pk = pack_key(vals[s], kk);
        if constexpr (FEAT) rp.slot(pk, kk, vals[s], cur);
        best = umax64(best, pk);
        keys[s] = kEmpty;
        vals[s] = 0.0f;
      }
    }
    best = wave_max_u64(best);
    if (lane == 0) red[tid >> 6] = best;
    __syncthreads();
    best = red[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) best = umax64(best, red[q]);
    uint32_t cstar = 0;
    const bool moved = decide(best, cur, pl, &cstar);
    if constexpr (FEAT) {
      const unsigned long long ws = wave_max_u64(rp.b1 == best ? rp.b2 : rp.b1);
      const unsigned long long wo = wave_max_u64(__float_as_uint(rp.own));
      const uint32_t wc = wave_sum_u32(rp.distinct);
      const float wk = wave_sum_f32(rp.K);
      if (lane == 0) {
        red2[tid >> 6] = ws;
        redo[tid >> 6] = wo;
        redc[tid >> 6] = wc;
        redk[tid >> 6] = wk;
      }
      __syncthreads();
      if (tid == 0) {
        unsigned long long sec = red2[0], ow = redo[0];
        uint32_t distinct = redc[0];
        float K = redk[0];
        for (int q = 1; q < NW; ++q) {
          sec = umax64(sec, red2[q]);
          ow = umax64(ow, redo[q]);
          distinct += redc[q];
          K += redk[q];
        }
        my_fneg += rec_write(a.rec, v, rold, l, K, __uint_as_float((uint32_t)ow),
                             __uint_as_float((uint32_t)(best >> 32)),
                             __uint_as_float((uint32_t)(sec >> 32)), distinct, (uint32_t)d,
                             moved);
      }
    }
    if (tid == 0) {
      if (a.async_mode) {
        if (moved) a.C[v] = (int32_t)cstar;
      } else {
        a.Cn[v] = moved ? (int32_t)cstar : cur;
      }
    }
    if (moved && tid == 0) a.chg[v] = 1;
    if (tid == 0) {
      my_edges += (unsigned long long)d;
      my_changed += moved ? 1u : 0u;
      my_flagw += moved ? (unsigned long long)d : 0ull;
    }
    __syncthreads();
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
  if constexpr (FEAT) flush_fneg(my_fneg, a.st);
}

// ---- one workgroup per vertex, next row's head loaded during the scan -------
// Plain variant of k_sweep_block: as k_sweep_wave_pipe, the workgroup issues
// the loads of its next vertex's head (the first BT*U targets and weights)
// before the barrier that ends the current row's accumulation, so that they
// are in flight while the table is scanned and cleared (the barriers wait on
// LDS traffic only).
template <typename OffT, int SLOTS, int BT, int U>
__global__ __launch_bounds__(BT) void k_sweep_block_pipe(SweepArgs a) {
  constexpr int NW = BT / 64;
  __shared__ uint32_t keys[SLOTS];
  __shared__ float vals[SLOTS];
  __shared__ unsigned long long red[NW];
  // the slots occupied by the current row, listed as they are claimed: the
  // table read-back visits these instead of all p1 slots (a row of d
  // entries holds at most d labels, and SLOTS >= 2 d - 1)
  __shared__ uint16_t lst[(SLOTS + 1) / 2];
  __shared__ uint32_t lst_n;
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int s = tid; s < SLOTS; s += BT) { keys[s] = kEmpty; vals[s] = 0.0f; }
  if (tid == 0) lst_n = 0u;
  __syncthreads();
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0;
  int32_t vq = 0, j[U];  // the current row's vertex and offsets
  int64_t oq = 0, eq = 0;
  float wt[U];
  // a row's first BT*U targets and weights, its offsets known
  auto head = [&](int32_t hv, int64_t ho, int64_t hd, int32_t* hj, float* hw) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = (int64_t)u * BT + tid;
      const bool has = e < hd;
      hj[u] = has ? __builtin_nontemporal_load(&a.tgt[ho + e]) : hv;
      hw[u] = has ? edge_weight(a.w, ho + e) : 0.0f;
    }
  };
  uint32_t item = blockIdx.x;
  if (item < count) {
    vq = first_lane_i32(a.active[vgpr_u32(item)]);
    row_bounds<OffT>(a.off, vq, &oq, &eq);
    oq = first_lane_i64(oq);
    eq = first_lane_i64(eq);
    head(vq, oq, eq - oq, j, wt);
  }
  // the next row's list entry and offsets (v1, o1, e1), loaded one row
  // earlier than its targets (as in k_sweep_wave_pipe)
  int32_t v1 = 0;
  int64_t o1 = 0, e1 = 0;
  if (item + gridDim.x < count) {
    v1 = first_lane_i32(a.active[vgpr_u32(item + gridDim.x)]);
    row_bounds<OffT>(a.off, v1, &o1, &e1);
    o1 = first_lane_i64(o1);
    e1 = first_lane_i64(e1);
  }
  while (item < count) {
    const int32_t v = vq;
    const int64_t o = oq, d = eq - o;
    const uint32_t nitem = item + gridDim.x;
    const uint32_t n2item = nitem + gridDim.x;
    const int32_t v2 = n2item < count ? a.active[vgpr_u32(n2item)] : 0;
    // own label, read before the barriers below: in asynchronous mode thread
    // 0 overwrites it, and every thread must reach the same move decision (a
    // vector load: used only by the decision at the row's end)
    const int32_t cur = a.C[vgpr_u32((uint32_t)v)];
    const uint32_t p1 = table_p1_load((uint32_t)d, a.tload, (uint32_t)SLOTS);
    // rows longer than the head: each further chunk's targets are loaded
    // before the labels of the chunk ahead of it are read, so that the two
    // loads overlap
    constexpr bool kLong = (SLOTS + 1) / 2 > BT * U;
    constexpr int64_t kStep = (int64_t)BT * U;
    int32_t jn[U];
    float wn[U];
    auto chunk = [&](int64_t base) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = base + u * BT + tid;
        const bool has = e < d;
        jn[u] = has ? __builtin_nontemporal_load(&a.tgt[o + e]) : v;
        wn[u] = has ? edge_weight(a.w, o + e) : 0.0f;
      }
    };
    if constexpr (kLong) {
      if (kStep < d) chunk(kStep);
    }
    uint32_t lab[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      lab[u] = (j[u] != v) ? (id0 ? (uint32_t)j[u] : (uint32_t)a.C[j[u]]) : kEmpty;
    #pragma unroll
    for (int u = 0; u < U; ++u) merge_lead(lab[u], wt[u], a.w == nullptr);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t cl =
          lab[u] != kEmpty ? lds_accumulate_claim(keys, vals, p1, lab[u], wt[u], a.probe) : -1;
      list_claimed(cl, lst, &lst_n);
    }
    for (int64_t base = kStep; kLong && base < d; base += kStep) {
      int32_t jj[U];
      float ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) { jj[u] = jn[u]; ww[u] = wn[u]; }
      if (base + kStep < d) chunk(base + kStep);
#pragma unroll
      for (int u = 0; u < U; ++u)
        lab[u] = (jj[u] != v) ? (id0 ? (uint32_t)jj[u] : (uint32_t)a.C[jj[u]]) : kEmpty;
      #pragma unroll
      for (int u = 0; u < U; ++u) merge_lead(lab[u], ww[u], a.w == nullptr);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t cl =
            lab[u] != kEmpty ? lds_accumulate_claim(keys, vals, p1, lab[u], ww[u], a.probe) : -1;
        list_claimed(cl, lst, &lst_n);
      }
    }
    int32_t nj[U];
    float nw[U];
    if (nitem < count) head(v1, o1, e1 - o1, nj, nw);
    int64_t o2 = 0, e2 = 0;
    if (n2item < count) row_bounds<OffT>(a.off, v2, &o2, &e2);
    __syncthreads();
    unsigned long long best = 0;
    const uint32_t nl = lst_n;
    for (uint32_t i = tid; i < nl; i += BT) {
      const uint32_t s = lst[i];
      best = umax64(best, pack_key(vals[s], keys[s]));
      keys[s] = kEmpty;
      vals[s] = 0.0f;
    }
    best = wave_max_u64(best);
    if (lane == 0) red[tid >> 6] = best;
    __syncthreads();
    best = red[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) best = umax64(best, red[q]);
    uint32_t cstar = 0;
    const bool moved = decide(best, cur, pl, &cstar);
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
      lst_n = 0u;  // every thread read it before the last barrier
    }
    __syncthreads();  // red[] and the slot list are rewritten by the next vertex
    item = nitem;
    vq = v1; oq = o1; eq = e1;
    // complete by now (the rotation of the head's registers waits for them)
    v1 = first_lane_i32(v2);
    o1 = first_lane_i64(o2);
    e1 = first_lane_i64(e2);
#pragma unroll
    for (int u = 0; u < U; ++u) { j[u] = nj[u]; wt[u] = nw[u]; }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
}

// ---- hubs: slices reduced in LDS, partitioned by label bucket, buckets
// reduced in LDS ----------------------------------------------------------------
// A hub row is cut into slices of chunk entries.  k_hub_part reduces a slice
// in an LDS table and writes its distinct (label, partial sum) pairs grouped
// by bucket (label hash >> (32 - lgb)), with the bucket offsets of the slice.
// k_hub_reduce takes one (hub, bucket): it reads that bucket's run from every
// slice of the hub, sums the runs in an LDS table and folds the bucket's
// packed maximum into the hub's best.  Every label of a hub lies in exactly
// one bucket, so the largest bucket maximum is the hub's Eq. 3 maximum.  The
// pairs move through HBM once each way, coalesced; no global atomics are
// made on label sums.  A bucket that finds its LDS table full spills the new
// labels into the hub's global table (each such label wholly, since a full
// table stays full), which k_hub_spill scans and clears.
namespace {

__device__ __forceinline__ uint32_t bucket_of(uint32_t label, int lgb) {
  uint32_t x = label;  // MurmurHash3 32-bit finaliser
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return lgb == 0 ? 0u : (x >> (32 - lgb));
}

// In-place exclusive scan of a[0..n) (n <= BT * PER) by one workgroup;
// returns the total.  Ends with a barrier.
template <int BT, int PER>
__device__ uint32_t block_exclusive_scan(uint32_t* a, uint32_t n, uint32_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t v[PER];
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = (uint32_t)tid * PER + q;
    v[q] = i < n ? a[i] : 0u;
    mine += v[q];
  }
  // inclusive scan of the per-thread sums within the wave
  uint32_t x = mine;
#pragma unroll
  for (int ofs = 1; ofs < 64; ofs <<= 1) {
    const uint32_t y = __shfl_up(x, ofs);
    if (lane >= ofs) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int q = 0; q < BT / 64; ++q) {
    if (q < wv) before += wsum[q];
    total += wsum[q];
  }
  uint32_t run = before + x - mine;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = (uint32_t)tid * PER + q;
    if (i < n) a[i] = run;
    run += v[q];
  }
  __syncthreads();
  return total;
}

// lds_accumulate that gives up (returns false) when the table holds neither
// the key nor an empty slot: after max_retries probes the linear
// continuation has visited every slot once.
__device__ __forceinline__ bool lds_accumulate_bounded(uint32_t* keys, float* vals, uint32_t p1,
                                                       uint32_t k, float v, ProbeCfg pc) {
  const uint32_t p2 = 2u * p1 + 1u;
  uint32_t s = k % p1;
  uint32_t step = 1u % p1;
  const uint32_t r = (k % p2) % p1;
  const int limit = pc.max_retries + (int)p1;
  for (int t = 0; t < limit; ++t) {
    uint32_t cur = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == kEmpty) {
      uint32_t expected = kEmpty;
      __hip_atomic_compare_exchange_strong(&keys[s], &expected, k, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      cur = (expected == kEmpty) ? k : expected;
    }
    if (cur == k) {
      __hip_atomic_fetch_add(&vals[s], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return true;
    }
    probe_next(s, step, r, p1, t, pc);
  }
  return false;
}

}  // namespace

template <typename OffT, int SLOTS, int BT>
__global__ __launch_bounds__(BT) void k_hub_part(HubArgs a) {
  constexpr int kMaxB = 1 << kHubMaxBucketLog2;
  __shared__ uint32_t keys[SLOTS];
  __shared__ float vals[SLOTS];
  __shared__ uint32_t hist[kMaxB];
  __shared__ uint32_t wsum[BT / 64];
  // the slots the current slice claimed: the histogram and partition passes
  // visit these instead of all p1c slots.  The list holds a little less
  // than a full slice's labels (the LDS budget): a slice with more distinct
  // labels than kLst reads back its whole table instead.
  constexpr uint32_t kLst = (SLOTS + 1) / 2 - 256;
  __shared__ uint16_t lst[kLst];
  __shared__ uint32_t lst_n;
  if (a.st->stop) return;
  const bool id0 = a.st->iter == 0 && a.st->ident;  // labels are still the ids
  const int tid = threadIdx.x;
  for (int s = tid; s < SLOTS; s += BT) { keys[s] = kEmpty; vals[s] = 0.0f; }
  if (tid == 0) lst_n = 0u;
  __syncthreads();
  const uint32_t nitems = a.st->hub_items;
  // with every hub flagged, the slices grouped by target window: group x
  // first on XCD x, then the others (the results do not depend on which
  // workgroup takes a slice)
  const bool grouped = a.witems != nullptr && a.st->hub_all != 0;
  const uint32_t* isrc = grouped ? a.witems : a.items;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  __shared__ uint32_t s_next[2];
  uint32_t home = grouped ? xcc_id() : 0u, done_groups = 0u, seq = 0u;
  // the next slice for this workgroup (thread 0 only)
  auto fetch = [&]() -> uint32_t {
    if (!grouped) {
      const uint32_t i = blockIdx.x + seq * gridDim.x;
      ++seq;
      return i < nitems ? i : kNone;
    }
    for (int k = 0; k < kXcds; ++k) {
      const uint32_t x = (home + (uint32_t)k) & (uint32_t)(kXcds - 1);
      if (done_groups & (1u << x)) continue;
      const uint32_t i = atomicAdd(&a.wctr[x * kQueueCtrStride], 1u);
      if (i < a.wbase[x + 1] - a.wbase[x]) return a.wbase[x] + i;
      done_groups |= 1u << x;
    }
    return kNone;
  };
  unsigned long long my_edges = 0, my_pairs = 0;
  // U entries per thread in flight: targets, then their labels, then the
  // table inserts.  The first BT*U targets of the next slice (its head) are
  // loaded before the barrier that ends the current slice's accumulation, so
  // that they are in flight during its partition phase.
  constexpr int U = 4;
  constexpr int64_t kStep = (int64_t)BT * U;
  struct Head {
    int32_t c, v, lgb, bq;
    int64_t o, e0, n, boff0, slice0;
    int32_t j[U];
    float wt[U];
  };
  // a slice's extent from its hub's row end, and its first BT*U targets
  auto head_tgt = [&](Head& H, int64_t end) {
    const int64_t d = end - H.o;
    H.e0 = (int64_t)H.c * a.chunk;
    H.n = (d - H.e0 < a.chunk) ? d - H.e0 : a.chunk;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = (int64_t)u * BT + tid;
      const bool has = e < H.n;
      H.j[u] = has ? __builtin_nontemporal_load(&a.tgt[H.o + H.e0 + e]) : H.v;
      H.wt[u] = has ? edge_weight(a.w, H.o + H.e0 + e) : 0.0f;
    }
  };
  if (tid == 0) {
    s_next[0] = fetch();
    s_next[1] = s_next[0] != kNone ? fetch() : kNone;
  }
  __syncthreads();
  uint32_t it = s_next[0], nit = s_next[1];
  int par = 0;
  __syncthreads();
  Head cur{};
  if (it != kNone) {
    const int32_t h = (int32_t)isrc[2 * (uint64_t)it];
    cur.c = (int32_t)isrc[2 * (uint64_t)it + 1];
    cur.v = a.hub_vid[h];
    cur.lgb = a.hub_lgb[h];
    cur.bq = a.hub_bq[h];
    cur.boff0 = a.hub_boff0[h];
    cur.slice0 = a.hub_slice0[h];
    int64_t end;
    row_bounds<OffT>(a.off, cur.v, &cur.o, &end);
    head_tgt(cur, end);
  }
  while (it != kNone) {
    const int32_t c = cur.c, v = cur.v, lgb = cur.lgb, bq = cur.bq;
    const int64_t o = cur.o, e0 = cur.e0, n = cur.n, boff0 = cur.boff0, slice0 = cur.slice0;
    // the next slice's header in three dependent steps (its item; its hub's
    // vertex and bucket parameters; the row offsets), vector loads each
    // issued while a chunk's labels of this slice are in flight
    const bool more = nit != kNone;
    uint32_t h1 = 0u, c1 = 0u;
    if (more) {
      const uint64_t q = 2 * (uint64_t)vgpr_u32(nit);
      h1 = isrc[q];
      c1 = isrc[q + 1];
    }
    int32_t v1 = 0, lgb1 = 0, bq1 = 0;
    int64_t boff1 = 0, sl1 = 0, o1 = 0, end1 = 0;
    const uint32_t nb = 1u << lgb;
    for (uint32_t b = tid; b < nb; b += BT) hist[b] = 0u;
    const uint32_t p1c = table_p1((uint32_t)n);
    int32_t jn[U];
    float wn[U];
    auto chunk = [&](int64_t base) {  // targets of the chunk at base
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = base + u * BT + tid;
        const bool has = e < n;
        jn[u] = has ? __builtin_nontemporal_load(&a.tgt[o + e0 + e]) : v;
        wn[u] = has ? edge_weight(a.w, o + e0 + e) : 0.0f;
      }
    };
    auto accumulate = [&](const int32_t* j, const float* wsrc, int step) {
      uint32_t lab[U];
      float wt[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        lab[u] = (j[u] != v) ? (id0 ? (uint32_t)j[u] : (uint32_t)a.C[j[u]]) : kEmpty;
        wt[u] = wsrc[u];
      }
      if (more && step == 0) {
        v1 = a.hub_vid[h1];
        lgb1 = a.hub_lgb[h1];
        bq1 = a.hub_bq[h1];
        boff1 = a.hub_boff0[h1];
        sl1 = a.hub_slice0[h1];
      } else if (more && step == 1) {
        row_bounds<OffT>(a.off, v1, &o1, &end1);
      }
      #pragma unroll
      for (int u = 0; u < U; ++u) merge_lead(lab[u], wt[u], a.w == nullptr);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t cl =
            lab[u] != kEmpty ? lds_accumulate_claim(keys, vals, p1c, lab[u], wt[u], a.probe) : -1;
        list_claimed(cl, lst, &lst_n, kLst);
      }
    };
    // the head chunk, then the rest, each chunk's targets loaded while the
    // labels of the chunk ahead of it are read
    if (kStep < n) chunk(kStep);
    accumulate(cur.j, cur.wt, 0);
    for (int64_t base = kStep; base < n; base += kStep) {
      int32_t jj[U];
      float ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) { jj[u] = jn[u]; ww[u] = wn[u]; }
      if (base + kStep < n) chunk(base + kStep);
      accumulate(jj, ww, base == kStep ? 1 : 2);
    }
    if (more && n <= kStep) row_bounds<OffT>(a.off, v1, &o1, &end1);
    Head nxt{};
    if (more) {
      nxt.c = first_lane_i32((int32_t)c1);
      nxt.v = first_lane_i32(v1);
      nxt.lgb = first_lane_i32(lgb1);
      nxt.bq = first_lane_i32(bq1);
      nxt.boff0 = first_lane_i64(boff1);
      nxt.slice0 = first_lane_i64(sl1);
      nxt.o = first_lane_i64(o1);
      head_tgt(nxt, first_lane_i64(end1));
    }
    // the slice after the next one, read by every thread after the last
    // barrier of this slice (two words: a slow thread may still read the
    // previous one while thread 0 writes this one)
    if (tid == 0) s_next[par] = nit != kNone ? fetch() : kNone;
    __syncthreads();
    const uint32_t nl = lst_n;
    const bool listed = nl <= kLst;  // else: the whole table, as p1c slots
    const uint32_t nv = listed ? nl : p1c;
    for (uint32_t i = tid; i < nv; i += BT) {
      const uint32_t kk = keys[listed ? lst[i] : i];
      if (kk != kEmpty) atomicAdd(&hist[bucket_of(kk, lgb)], 1u);
    }
    __syncthreads();
    // the bucket totals over all slices, which size the reduction's tables
    for (uint32_t b = tid; b < nb; b += BT)
      if (hist[b]) atomicAdd(&a.bsize[bq + b], hist[b]);
    __syncthreads();
    const uint32_t total = block_exclusive_scan<BT, kMaxB / BT>(hist, nb, wsum);
    uint32_t* bo = a.boff + boff0 + (int64_t)c * (nb + 1);
    for (uint32_t b = tid; b < nb; b += BT) bo[b] = hist[b];
    if (tid == 0) {
      bo[nb] = total;
      my_pairs += total;
    }
    const int64_t base = (slice0 + c) * (int64_t)a.chunk;
    for (uint32_t i = tid; i < nv; i += BT) {
      const uint32_t s = listed ? lst[i] : i;
      const uint32_t kk = keys[s];
      if (kk == kEmpty) continue;
      const uint32_t pos = atomicAdd(&hist[bucket_of(kk, lgb)], 1u);
      a.part_keys[base + pos] = kk;
      a.part_vals[base + pos] = vals[s];
      keys[s] = kEmpty;
      vals[s] = 0.0f;
    }
    if (tid == 0) {
      my_edges += (unsigned long long)n;
      lst_n = 0u;  // read by every thread before the barriers above
    }
    __syncthreads();
    const uint32_t nn = s_next[par];
    par ^= 1;
    it = nit;
    nit = nn;
    cur = nxt;
  }
  // one atomic per workgroup (my_pairs lives in thread 0: the (label, sum)
  // pairs its slices wrote, read back by k_hub_reduce)
  __shared__ unsigned long long we[BT / 64];
  const unsigned long long e = wave_sum_u64(my_edges);
  if ((tid & 63) == 0) we[tid >> 6] = e;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < BT / 64; ++q) t += we[q];
    if (t) atomicAdd(&a.st->edges[kClassHub], t);
    if (my_pairs) atomicAdd(&a.st->hub_pairs, my_pairs);
  }
}

// Two instantiations share the queued buckets: the small one (SLOTS 4095,
// several workgroups per CU) takes the buckets of at most SMALL_E pairs, the
// large one the rest; a bucket with no pairs is skipped by both.
constexpr uint32_t kHubSmallE = 2048;
template <typename OffT, int SLOTS, int BT, bool LARGE>
__global__ __launch_bounds__(BT) void k_hub_reduce(HubArgs a) {
  constexpr int kRuns = 4 * BT;  // slice runs staged per pass
  __shared__ uint32_t keys[SLOTS];
  __shared__ float vals[SLOTS];
  __shared__ uint32_t start[kRuns];
  __shared__ unsigned long long red[BT / 64];
  __shared__ uint32_t wsum[BT / 64];
  __shared__ int spilled;
  if (a.st->stop) return;
  const int tid = threadIdx.x, lane = tid & 63;
  for (int s = tid; s < SLOTS; s += BT) { keys[s] = kEmpty; vals[s] = 0.0f; }
  if (tid == 0) spilled = 0;
  __syncthreads();
  const uint32_t nitems = a.st->hub_bitems;
  // xcd_map: workgroup w runs on XCD w % 8 (round-robin dispatch); give each
  // XCD a contiguous range of buckets so that the runs of neighbouring
  // buckets, which share cache lines, are read through one L2
  const uint32_t nx = a.xcd_map ? (uint32_t)kXcds : 1u;
  const uint32_t x = blockIdx.x % nx, lw = blockIdx.x / nx, nlw = gridDim.x / nx;
  if (lw >= nlw) return;  // workgroups past the last full round of XCDs
  const uint32_t per = (nitems + nx - 1) / nx;
  // The workgroup's buckets are x * per + j for j = lw, lw + nlw, ...  They
  // are taken BT at a time: each thread reads one bucket's pair count
  // (counted by k_hub_part), the buckets of this size class that hold pairs
  // are listed in order, and the listed buckets are reduced one after the
  // other, the next one's header loaded while the current one's pairs are
  // in flight.
  __shared__ uint32_t ilist[BT], elist[BT], wcnt[BT / 64];
  const int wv = tid >> 6;
  for (uint32_t j0 = lw; j0 < per; j0 += (uint32_t)BT * nlw) {
    {
      const uint64_t jt = (uint64_t)j0 + (uint64_t)tid * nlw;
      const uint64_t itt = (uint64_t)x * per + jt;
      uint32_t E = 0;
      if (jt < per && itt < nitems) E = a.bsize[itt];
      const bool q = E != 0 && (E > kHubSmallE) == LARGE;
      const unsigned long long m = __ballot(q);
      if (lane == 0) wcnt[wv] = (uint32_t)__popcll(m);
      __syncthreads();
      uint32_t pos = 0;
      for (int w = 0; w < wv; ++w) pos += wcnt[w];
      if (q) {
        ilist[pos + lane_rank(m)] = (uint32_t)itt;
        elist[pos + lane_rank(m)] = E;
      }
      __syncthreads();
    }
    uint32_t nlist = 0;
    for (int w = 0; w < BT / 64; ++w) nlist += wcnt[w];
    // header of the listed bucket k: its hub and bucket index (step 1), then
    // the hub's bucket count, run offsets, first slice, spill table and
    // slice count (step 2); vector loads, made uniform when the bucket is
    // reached
    auto step1 = [&](uint32_t k, uint32_t& hh, uint32_t& bb) {
      const uint64_t q = 2 * (uint64_t)vgpr_u32(ilist[k]);
      hh = a.bitems[q];
      bb = a.bitems[q + 1];
    };
    struct Hub2 { int32_t lgb, nch; int64_t boff0, slice0, tab; };
    auto step2 = [&](uint32_t hh, Hub2& r) {
      r.lgb = a.hub_lgb[hh];
      r.nch = a.hub_nch[hh];
      r.boff0 = a.hub_boff0[hh];
      r.slice0 = a.hub_slice0[hh];
      r.tab = a.hub_tab[hh];
    };
    uint32_t hq = 0u, bq = 0u;
    Hub2 cq{};
    if (nlist > 0) {
      step1(0, hq, bq);
      step2(hq, cq);
    }
    for (uint32_t k = 0; k < nlist; ++k) {
      const int32_t h = first_lane_i32((int32_t)hq);
      const uint32_t b = (uint32_t)first_lane_i32((int32_t)bq);
      const uint32_t E = elist[k];
      const uint32_t nch = (uint32_t)first_lane_i32(cq.nch);
      const int lgb = first_lane_i32(cq.lgb);
      const int64_t boff0 = first_lane_i64(cq.boff0);
      const int64_t slice0 = first_lane_i64(cq.slice0);
      const int64_t tab = first_lane_i64(cq.tab);
      const bool more = k + 1 < nlist;
      uint32_t h1 = 0u, b1 = 0u;
      if (more) step1(k + 1, h1, b1);
      Hub2 c1{};
      bool c1_done = false;
      const uint32_t nb1 = (1u << lgb) + 1u;
      const uint32_t* bo = a.boff + boff0;
      uint32_t p1 = E <= (uint32_t)(SLOTS + 1) / 2 ? table_p1(E > 0 ? E : 1u) : (uint32_t)SLOTS;
      if (p1 > a.table_cap) p1 = a.table_cap;
      uint32_t* gk = a.gkeys + tab;
      float* gv = a.gvals + tab;
      bool my_spill = false;
      // the bucket's runs, kRuns slices at a time: their lengths are scanned
      // into start[], and the workgroup's threads take the pass's entries
      // evenly, each finding its slice by binary search in start[]
      for (uint32_t c0 = 0; c0 < nch; c0 += kRuns) {
        const uint32_t cn = (nch - c0 < (uint32_t)kRuns) ? nch - c0 : (uint32_t)kRuns;
        for (uint32_t i = tid; i < cn; i += BT) {
          const uint32_t c = c0 + i;
          start[i] = bo[c * nb1 + b + 1] - bo[c * nb1 + b];
        }
        if (more && !c1_done) {
          step2(h1, c1);
          c1_done = true;
        }
        __syncthreads();
        const uint32_t total = block_exclusive_scan<BT, kRuns / BT>(start, cn, wsum);
        // whole-wave steps (the last one partial), so that the lanes holding
        // the label of the wave's first pair can merge before the inserts:
        // the runs of different slices repeat the same labels
        for (uint32_t g0 = 0; g0 < total; g0 += BT) {
          const uint32_t g = g0 + tid;
          uint32_t kk = kEmpty;
          float vv = 0.0f;
          if (g < total) {
            uint32_t lo = 0, hi = cn - 1;  // largest i with start[i] <= g
            while (lo < hi) {
              const uint32_t mid = (lo + hi + 1) >> 1;
              if (start[mid] <= g) lo = mid; else hi = mid - 1;
            }
            const uint32_t c = c0 + lo;
            const uint32_t e = bo[c * nb1 + b] + (g - start[lo]);
            const int64_t idx = (slice0 + c) * (int64_t)a.chunk + e;
            kk = a.part_keys[idx];
            vv = a.part_vals[idx];
          }
          merge_lead(kk, vv, false);
          if (kk == kEmpty) continue;
          if (!lds_accumulate_bounded(keys, vals, p1, kk, vv, a.probe)) {
            // the hub's spill table holds table_p1(degree) slots
            int64_t o, d;
            row_of<OffT>(a.off, a.hub_vid[h], &o, &d);
            float after;
            (void)global_accumulate<__HIP_MEMORY_SCOPE_AGENT>(gk, gv, table_p1((uint32_t)d), kk,
                                                              vv, a.probe, &after);
            my_spill = true;
          }
        }
        __syncthreads();  // start[] is rewritten by the next pass
      }
      if (more && !c1_done) step2(h1, c1);
      if (my_spill) spilled = 1;
      __syncthreads();
      unsigned long long best = 0;
      for (uint32_t s = tid; s < p1; s += BT) {
        const uint32_t kk = keys[s];
        if (kk != kEmpty) {
          best = umax64(best, pack_key(vals[s], kk));
          keys[s] = kEmpty;
          vals[s] = 0.0f;
        }
      }
      best = wave_max_u64(best);
      if (lane == 0) red[tid >> 6] = best;
      __syncthreads();
      if (tid == 0) {
        unsigned long long bb = red[0];
        for (int q = 1; q < BT / 64; ++q) bb = umax64(bb, red[q]);
        if (bb) atomicMax(&a.hub_best[h], bb);
        if (spilled) a.hub_ovf[h] = 1;
        spilled = 0;
      }
      __syncthreads();
      hq = h1; bq = b1; cq = c1;
    }
    __syncthreads();  // ilist, elist and wcnt are rewritten by the next batch
  }
}

// Labels spilled into a hub's global table: each slice of the hub scans a
// stripe of the table, folds its maximum into the hub's best and clears it.
template <typename OffT, int BT>
__global__ __launch_bounds__(BT) void k_hub_spill(HubArgs a) {
  __shared__ unsigned long long red[BT / 64];
  if (a.st->stop) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t nitems = a.st->hub_items;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t h = (int32_t)a.items[2 * (uint64_t)it];
    if (!a.hub_ovf[h]) continue;  // uniform over the workgroup
    const int32_t c = (int32_t)a.items[2 * (uint64_t)it + 1];
    int64_t o, d;
    row_of<OffT>(a.off, a.hub_vid[h], &o, &d);
    const int64_t ns = (d + a.chunk - 1) / a.chunk;
    const int64_t p1g = table_p1((uint32_t)d);
    const int64_t s0 = p1g * c / ns, s1 = p1g * (c + 1) / ns;
    uint32_t* gk = a.gkeys + a.hub_tab[h];
    float* gv = a.gvals + a.hub_tab[h];
    unsigned long long best = 0;
    for (int64_t s = s0 + tid; s < s1; s += BT) {
      const uint32_t kk = gk[s];
      if (kk != kEmpty) {
        best = umax64(best, pack_key(gv[s], kk));
        gk[s] = kEmpty;
        gv[s] = 0.0f;
      }
    }
    best = wave_max_u64(best);
    if (lane == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
      unsigned long long bb = red[0];
      for (int q = 1; q < BT / 64; ++q) bb = umax64(bb, red[q]);
      if (bb) atomicMax(&a.hub_best[h], bb);
    }
    __syncthreads();
  }
}

// Move decision of each hub from its packed best (slice 0 of the hub writes
// the label; every slice adds its entry count to the flag work).
template <typename OffT, int BT>
__global__ __launch_bounds__(BT) void k_hub_fin(HubArgs a) {
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const int tid = threadIdx.x;
  const uint32_t nitems = a.st->hub_items;
  for (uint32_t it = blockIdx.x * BT + tid; it < nitems; it += gridDim.x * BT) {
    const int32_t h = (int32_t)a.items[2 * (uint64_t)it];
    const int32_t c = (int32_t)a.items[2 * (uint64_t)it + 1];
    const int32_t v = a.hub_vid[h];
    int64_t o, d;
    row_of<OffT>(a.off, v, &o, &d);
    const int64_t e0 = (int64_t)c * a.chunk;
    const int64_t n = (d - e0 < a.chunk) ? d - e0 : a.chunk;
    uint32_t cstar = 0;
    const bool moved = decide(a.hub_best[h], a.hub_old[h], pl, &cstar);
    if (!moved) continue;
    if (c == 0) {
      if (a.async_mode) {
        a.C[v] = (int32_t)cstar;
      } else {
        const unsigned long long pos = atomicAdd(&a.st->pending, 1ull);
        a.pend_v[pos] = v;
        a.pend_c[pos] = (int32_t)cstar;
      }
      atomicAdd(&a.st->changed[kClassHub], 1ull);
      a.chg[v] = 1;
    }
    atomicAdd(&a.st->flagw[kClassHub], (unsigned long long)n);
  }
}

// ---- the first sweep from identity labels over strict rows ------------------
// Every neighbour label occurs once in such a row and its sum is the entry's
// weight, so the row's Eq. 3 maximum (ties to the smallest label) is the
// largest packed (weight, target) entry: a streaming maximum, no table.  The
// rows are read in the caller's order and numbering (uoff/utgt/uw), where
// the targets are the labels; results go to the internal slots.  G
// lanes per vertex (4, 16 or 64 for the wave-sized classes, a whole
// workgroup of BT for the larger ones); hub slices fold their maximum into the
// hub's best, decided by k_hub_fin as usual.
//
// FEAT: the learned variant, which also writes each vertex's state record:
// with every label of the row distinct and none equal to the vertex's own,
// the record's label weights are entry weights — own label 0, best and
// second best the two largest entries, distinct labels the non-self entries.
// INT: read the internal row instead and take each target's label from inv
// (rows of at most 4 entries: such a row in the caller's order costs a cache
// line of its own, while the internal rows of the class are contiguous; for
// longer rows the inv reads cost more than they save, measured).
template <typename OffT, int G, int BT, bool FEAT, bool INT>
__global__ __launch_bounds__(BT) void k_sweep_direct(SweepArgs a) {
  __shared__ unsigned long long red[BT / 64];
  __shared__ unsigned long long red2[FEAT ? BT / 64 : 1];
  __shared__ float redk[FEAT ? BT / 64 : 1];
  __shared__ uint32_t redc[FEAT ? BT / 64 : 1];
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const int l = a.st->iter;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t count = a.st->active[a.cls];
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0, my_fneg = 0;
  constexpr int kPer = (G >= 64) ? 1 : 64 / G;        // vertices per wave step
  const int k = (G >= 64) ? ((G == 64) ? lane : tid) : (lane & (G - 1));
  const uint64_t nsteps_wave = (G > 64) ? 1 : (uint64_t)(BT / 64);
  const uint64_t unit0 = (G > 64) ? blockIdx.x : (uint64_t)blockIdx.x * nsteps_wave + (tid >> 6);
  const uint64_t nunits = (G > 64) ? gridDim.x : (uint64_t)gridDim.x * nsteps_wave;
  for (uint64_t base = unit0 * kPer; base < count; base += nunits * kPer) {
    const uint64_t idx = base + ((G >= 64) ? 0 : (uint32_t)lane / G);
    const bool valid = idx < count;
    const int32_t vi = valid ? a.active[idx] : 0;       // internal id
    const int32_t v = a.inv ? a.inv[vi] : vi;            // caller's id = its label
    int64_t o = 0, d = 0;
    // cint: the internal rows carry the caller's ids (no inv reads, rows of
    // one class contiguous)
    const bool cint = a.ctgt != nullptr;
    const bool irow = INT || cint;
    if (valid) row_of<OffT>(irow ? a.off : a.uoff, irow ? vi : v, &o, &d);
    [[maybe_unused]] const unsigned long long rold = (FEAT && valid && k == 0) ? a.rec[vi] : 0ull;
    unsigned long long best = 0, b2 = 0;  // this lane's two largest entries
    float K = 0.0f;
    uint32_t nd = 0;
    const int32_t* rt = cint ? a.ctgt : (INT ? a.tgt : a.utgt);
    const float* rw = irow ? a.w : a.uw;
    const bool remap = INT && !cint && a.inv != nullptr;
    const int32_t self = (INT && !cint) ? vi : v;
    auto take = [&](int32_t jr, float wj) {
      if (jr == self) return;
      const int32_t j = remap ? a.inv[jr] : jr;
      const unsigned long long pk = pack_key(wj, (uint32_t)j);
      if constexpr (FEAT) {
        if (pk > best) { b2 = best; best = pk; } else if (pk > b2) { b2 = pk; }
        K += wj;
        ++nd;
      } else {
        best = umax64(best, pk);
      }
    };
    // four entries per lane in flight, then the remainder
    constexpr int UD = 4;
    int64_t e = k;
    if constexpr (G == 1) {
      // rows of at most 4 entries (the smallest class): one predicated load
      // per slot, all in flight at once
      int32_t jr[4];
      float wj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        jr[u] = (u < d) ? __builtin_nontemporal_load(&rt[o + u]) : self;
        wj[u] = (u < d) ? edge_weight(rw, o + u) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) take(jr[u], wj[u]);
      e = d;
    }
    for (; e + (UD - 1) * G < d; e += UD * G) {
      int32_t jr[UD];
      float wj[UD];
#pragma unroll
      for (int u = 0; u < UD; ++u) {
        jr[u] = __builtin_nontemporal_load(&rt[o + e + u * G]);
        wj[u] = edge_weight(rw, o + e + u * G);
      }
#pragma unroll
      for (int u = 0; u < UD; ++u) take(jr[u], wj[u]);
    }
    for (; e < d; e += G) take(__builtin_nontemporal_load(&rt[o + e]), edge_weight(rw, o + e));
    const unsigned long long mine = best;
    if constexpr (G == 1) {
      // one lane per vertex: nothing to combine
    } else if constexpr (G == 4) {
      best = quad_max_u64(best);
    } else if constexpr (G == 8) {
      // the two quads of each half row: quad maxima, then row_half_mirror
      best = quad_max_u64(best);
      best = umax64(best, dpp64<0x141>(best));
    } else if constexpr (G == 16) {
      best = row16_max_u64(best);
    } else {
      best = wave_max_u64(best);
    }
    if constexpr (G > 64) {
      if (lane == 0) red[tid >> 6] = best;
      __syncthreads();
      best = red[0];
#pragma unroll
      for (int q = 1; q < BT / 64; ++q) best = umax64(best, red[q]);
      __syncthreads();
    }
    // the vertex's own label is its caller id in this sweep
    uint32_t cstar = 0;
    const bool moved = valid && decide(best, v, pl, &cstar);
    const bool leader = valid && k == 0;
    if constexpr (FEAT) {
      unsigned long long sc = (mine == best) ? b2 : mine;
      if constexpr (G == 1) {
        // the lane's own top two and sums are the row's
      } else if constexpr (G == 4) {
        sc = quad_max_u64(sc); K = group_sum_f32<4>(K); nd = group_sum_u32<4>(nd);
      } else if constexpr (G == 8) {
        sc = quad_max_u64(sc);
        sc = umax64(sc, dpp64<0x141>(sc));
        K = group_sum_f32<4>(K);
        K += dppf<0x141>(K);
        nd = group_sum_u32<4>(nd);
        nd += dpp32<0x141>(nd);
      } else if constexpr (G == 16) {
        sc = row16_max_u64(sc); K = group_sum_f32<16>(K); nd = group_sum_u32<16>(nd);
      } else {
        sc = wave_max_u64(sc); K = wave_sum_f32(K); nd = wave_sum_u32(nd);
      }
      if constexpr (G > 64) {
        if (lane == 0) { red2[tid >> 6] = sc; redk[tid >> 6] = K; redc[tid >> 6] = nd; }
        __syncthreads();
        sc = red2[0]; K = redk[0]; nd = redc[0];
#pragma unroll
        for (int q = 1; q < BT / 64; ++q) { sc = umax64(sc, red2[q]); K += redk[q]; nd += redc[q]; }
        __syncthreads();
      }
      if (leader && d >= 1)
        my_fneg += rec_write(a.rec, vi, rold, l, K, 0.0f, __uint_as_float((uint32_t)(best >> 32)),
                             __uint_as_float((uint32_t)(sc >> 32)), nd, (uint32_t)d, moved);
    }
    if (leader) {
      if (a.async_mode) {
        if (moved) a.C[vi] = (int32_t)cstar;
      } else {
        a.Cn[vi] = moved ? (int32_t)cstar : v;
      }
      if (moved) a.chg[vi] = 1;
      my_edges += (unsigned long long)d;
      my_changed += moved ? 1u : 0u;
      my_flagw += moved ? (unsigned long long)d : 0ull;
    }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
  if constexpr (FEAT) flush_fneg(my_fneg, a.st);
}

// Plain first sweep of the rows of 5-64 entries, R wave steps at a time:
// the list entries, row offsets and first targets of all R steps are loaded
// before any step is reduced.  A step is a chain of three
// dependent loads (list, offsets, targets), which the one-step loop of
// k_sweep_direct waits for in turn.  Labels are the caller's ids, read from
// the internal rows that hold them (ctgt) or from the caller's rows.
template <typename OffT, int G, int BT>
__global__ __launch_bounds__(BT) void k_sweep_direct2(SweepArgs a) {
  static_assert(G == 4 || G == 8, "the classes that gain from it");
  constexpr int kPer = 64 / G;  // vertices per wave step
  constexpr int UD = 4;         // entries per lane loaded with the step's head
  constexpr int R = 3;          // steps in flight
  if (a.st->stop) return;
  const int pl = a.st->pl;  // fixed for the whole sweep
  const int tid = threadIdx.x, lane = tid & 63;
  const int k = lane & (G - 1);
  const uint32_t count = a.st->active[a.cls];
  const uint64_t unit0 = (uint64_t)blockIdx.x * (BT / 64) + (tid >> 6);
  const uint64_t nunits = (uint64_t)gridDim.x * (BT / 64);
  const bool cint = a.ctgt != nullptr;
  const void* roff = cint ? a.off : a.uoff;
  const int32_t* rt = cint ? a.ctgt : a.utgt;
  const float* rw = cint ? a.w : a.uw;
  unsigned long long my_edges = 0, my_flagw = 0;
  uint32_t my_changed = 0;
  for (uint64_t base = unit0 * kPer; base < count; base += (uint64_t)R * nunits * kPer) {
    bool valid[R];
    int32_t vi[R], v[R];
    int64_t o[R], d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t idx = base + (uint64_t)r * nunits * kPer + (uint32_t)lane / G;
      valid[r] = idx < count;
      vi[r] = valid[r] ? a.active[idx] : 0;  // internal id
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a.inv ? a.inv[vi[r]] : vi[r];  // caller id = label
#pragma unroll
    for (int r = 0; r < R; ++r) {
      o[r] = 0;
      d[r] = 0;
      if (valid[r]) row_of<OffT>(roff, cint ? vi[r] : v[r], &o[r], &d[r]);
    }
    int32_t jr[R][UD];
    float wj[R][UD];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < UD; ++u) {
        const int64_t e = (int64_t)u * G + k;
        const bool has = e < d[r];
        jr[r][u] = has ? __builtin_nontemporal_load(&rt[o[r] + e]) : v[r];
        wj[r][u] = has ? edge_weight(rw, o[r] + e) : 0.0f;
      }
    unsigned long long best[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      best[r] = 0;
#pragma unroll
      for (int u = 0; u < UD; ++u)
        if (jr[r][u] != v[r]) best[r] = umax64(best[r], pack_key(wj[r][u], (uint32_t)jr[r][u]));
      // the rest of a row longer than UD * G entries
      int64_t e = (int64_t)UD * G + k;
      for (; e + (UD - 1) * G < d[r]; e += UD * G) {
        int32_t j2[UD];
        float w2[UD];
#pragma unroll
        for (int u = 0; u < UD; ++u) {
          j2[u] = __builtin_nontemporal_load(&rt[o[r] + e + u * G]);
          w2[u] = edge_weight(rw, o[r] + e + u * G);
        }
#pragma unroll
        for (int u = 0; u < UD; ++u)
          if (j2[u] != v[r]) best[r] = umax64(best[r], pack_key(w2[u], (uint32_t)j2[u]));
      }
      for (; e < d[r]; e += G) {
        const int32_t j = __builtin_nontemporal_load(&rt[o[r] + e]);
        if (j != v[r]) best[r] = umax64(best[r], pack_key(edge_weight(rw, o[r] + e), (uint32_t)j));
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      unsigned long long b = quad_max_u64(best[r]);
      if constexpr (G == 8) b = umax64(b, dpp64<0x141>(b));  // row_half_mirror: the other quad
      // the vertex's own label is its caller id in this sweep
      uint32_t cstar = 0;
      const bool moved = valid[r] && decide(b, v[r], pl, &cstar);
      if (valid[r] && k == 0) {
        if (a.async_mode) {
          if (moved) a.C[vi[r]] = (int32_t)cstar;
        } else {
          a.Cn[vi[r]] = moved ? (int32_t)cstar : v[r];
        }
        if (moved) a.chg[vi[r]] = 1;
        my_edges += (unsigned long long)d[r];
        my_changed += moved ? 1u : 0u;
        my_flagw += moved ? (unsigned long long)d[r] : 0ull;
      }
    }
  }
  flush_stats(my_edges, my_changed, my_flagw, a.st, a.cls);
}

template <typename OffT, int BT>
__global__ __launch_bounds__(BT) void k_hub_direct(HubArgs a) {
  if (a.st->stop) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t nitems = a.st->hub_items;
  unsigned long long my_edges = 0;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int32_t h = (int32_t)a.items[2 * (uint64_t)it];
    const int32_t c = (int32_t)a.items[2 * (uint64_t)it + 1];
    const int32_t vi = a.hub_vid[h];
    const int32_t v = a.inv ? a.inv[vi] : vi;  // the caller's row, same length
    // the internal row with the caller's ids, when the handle keeps one
    const bool cint = a.ctgt != nullptr;
    const int32_t* rt = cint ? a.ctgt : a.utgt;
    const float* rw = cint ? a.w : a.uw;
    int64_t o, d;
    row_of<OffT>(cint ? a.off : a.uoff, cint ? vi : v, &o, &d);
    const int64_t e0 = (int64_t)c * a.chunk;
    const int64_t n = (d - e0 < a.chunk) ? d - e0 : a.chunk;
    unsigned long long best = 0;
    constexpr int UD = 4;  // entries per thread in flight
    int64_t e = tid;
    for (; e + (UD - 1) * BT < n; e += UD * BT) {
      int32_t j[UD];
      float wj[UD];
#pragma unroll
      for (int u = 0; u < UD; ++u) {
        j[u] = __builtin_nontemporal_load(&rt[o + e0 + e + u * BT]);
        wj[u] = edge_weight(rw, o + e0 + e + u * BT);
      }
#pragma unroll
      for (int u = 0; u < UD; ++u)
        if (j[u] != v) best = umax64(best, pack_key(wj[u], (uint32_t)j[u]));
    }
    for (; e < n; e += BT) {
      const int32_t j = __builtin_nontemporal_load(&rt[o + e0 + e]);
      if (j != v) best = umax64(best, pack_key(edge_weight(rw, o + e0 + e), (uint32_t)j));
    }
    best = wave_max_u64(best);
    if (lane == 0 && best) atomicMax(&a.hub_best[h], best);
    if (tid == 0) my_edges += (unsigned long long)n;
  }
  const unsigned long long e = wave_sum_u64(my_edges);
  if (lane == 0 && e) atomicAdd(&a.st->edges[kClassHub], e);
}

// ---- launch wrappers ----------------------------------------------------------
namespace {
constexpr int kWaveWaves = 4;
constexpr int kBlockBig = 1024;   // threads for the 16383-slot table
constexpr int kBlockMid = 512;
constexpr int kHubThreads = 1024;
constexpr int kHubSlots = 16383;  // slice of up to 8192 edges
}  // namespace

int sweep_block_threads(int cls) {
  switch (cls) {
    case 1: case 2: case 3: case 4: return 256;
    case 5: case 6: return 256;
    case 7: return kBlockMid;
    case 8: return kBlockBig;
    default: return 256;
  }
}
int sweep_items_per_block(int cls) {
  switch (cls) {
    case 1: return 256 / 4;
    case 2: case 3: return 256 / 16;
    case 4: return kWaveWaves;
    default: return 1;
  }
}
int sweep_direct_items_per_block(int cls) {
  switch (cls) {
    case 1: return 256;
    case 2: return 256 / 4;
    case 3: return 256 / 8;
    case 4: return 256 / 16;
    case 5: case 6: return 256 / 64;
    default: return 1;
  }
}
// Workgroups resident on the whole GPU (256 CUs) for each class; LDS bound
// for the table kernels (160 KB per CU).
int sweep_max_resident(int cls) {
  switch (cls) {
    case 1: case 2: return 256 * 8;   // 32 waves per CU
    case 3: return 256 * 8;           // 16 KB LDS per workgroup (16 tables)
    case 4: return 256 * 4;           // 32 KB
    case 5: return 256 * 8;           // 16 KB
    case 6: return 256 * 4;           // 32 KB
    case 7: return 256 * 2;           // 64 KB
    case 8: return 256 * 1;           // 128 KB
    default: return 256;
  }
}
int hub_block_threads() { return kHubThreads; }
int hub_max_resident() { return 256; }

// Workgroup classes with another thread count (lpa_tuning.block_threads).
template <typename OffT, int BT>
static hipError_t sweep_block_bt(int cls, const SweepArgs& a, int grid, hipStream_t s) {
  switch (cls) {
    case 5: hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 2047, BT, 4>), dim3(grid), dim3(BT), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 4095, BT, 4>), dim3(grid), dim3(BT), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 8191, BT, 4>), dim3(grid), dim3(BT), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 16383, BT, 4>), dim3(grid), dim3(BT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename OffT, bool FEAT>
static hipError_t sweep_t(int cls, const SweepArgs& a, int grid, hipStream_t s) {
  if (!FEAT && cls >= 5 && cls <= 8 && a.block_threads != 0) {
    switch (a.block_threads) {
      case 256: return sweep_block_bt<OffT, 256>(cls, a, grid, s);
      case 512: return sweep_block_bt<OffT, 512>(cls, a, grid, s);
      case 1024: return sweep_block_bt<OffT, 1024>(cls, a, grid, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (cls) {
    case 1:
      if constexpr (FEAT) hipLaunchKernelGGL((k_sweep_small<OffT, 4, true>), dim3(grid), dim3(256), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_lane4<OffT>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 2:
      if constexpr (FEAT) hipLaunchKernelGGL((k_sweep_small<OffT, 16, true>), dim3(grid), dim3(256), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_small16x2<OffT>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 3:
      hipLaunchKernelGGL((k_sweep_group<OffT, 127, 16, FEAT>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 4:
      hipLaunchKernelGGL((k_sweep_wave_pipe<OffT, 1023, kWaveWaves, 4, FEAT>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 5:
      if constexpr (FEAT) hipLaunchKernelGGL((k_sweep_block<OffT, 2047, 256, 4, true>), dim3(grid), dim3(256), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 2047, 256, 4>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 6:
      if constexpr (FEAT) hipLaunchKernelGGL((k_sweep_block<OffT, 4095, 256, 4, true>), dim3(grid), dim3(256), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 4095, 256, 8>), dim3(grid), dim3(256), 0, s, a);
      break;
    case 7:
      if constexpr (FEAT) hipLaunchKernelGGL((k_sweep_block<OffT, 8191, kBlockMid, 4, true>), dim3(grid), dim3(kBlockMid), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 8191, kBlockMid, 4>), dim3(grid), dim3(kBlockMid), 0, s, a);
      break;
    case 8:
      if constexpr (FEAT) hipLaunchKernelGGL((k_sweep_block<OffT, 16383, kBlockBig, 4, true>), dim3(grid), dim3(kBlockBig), 0, s, a);
      else hipLaunchKernelGGL((k_sweep_block_pipe<OffT, 16383, kBlockBig, 4>), dim3(grid), dim3(kBlockBig), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename OffT, bool FEAT>
static hipError_t direct_t(int cls, const SweepArgs& a, int grid, hipStream_t s) {
  // three steps in flight: 5-16-entry rows 0.43 -> 0.23 ms, 17-64-entry
  // rows 0.57 -> 0.44 ms on R-MAT 26 (two: 0.24 and 0.45 ms); with two, the
  // rows of up to 4 entries measured the same and those of 65-512 entries
  // slower (0.48 -> 0.58 ms)
  if constexpr (!FEAT) {
    switch (cls) {
      case 2: hipLaunchKernelGGL((k_sweep_direct2<OffT, 4, 256>), dim3(grid), dim3(256), 0, s, a); return hipGetLastError();
      case 3: hipLaunchKernelGGL((k_sweep_direct2<OffT, 8, 256>), dim3(grid), dim3(256), 0, s, a); return hipGetLastError();
      default: break;
    }
  }
  switch (cls) {
    case 1: hipLaunchKernelGGL((k_sweep_direct<OffT, 1, 256, FEAT, true>), dim3(grid), dim3(256), 0, s, a); break;
    case 2:
      hipLaunchKernelGGL((k_sweep_direct<OffT, 4, 256, FEAT, false>), dim3(grid), dim3(256), 0, s, a); break;
    case 3:
      hipLaunchKernelGGL((k_sweep_direct<OffT, 8, 256, FEAT, false>), dim3(grid), dim3(256), 0, s, a); break;
    case 4:
      hipLaunchKernelGGL((k_sweep_direct<OffT, 16, 256, FEAT, false>), dim3(grid), dim3(256), 0, s, a); break;
    case 5: case 6:
      hipLaunchKernelGGL((k_sweep_direct<OffT, 64, 256, FEAT, false>), dim3(grid), dim3(256), 0, s, a); break;
    case 7: case 8:
      hipLaunchKernelGGL((k_sweep_direct<OffT, 256, 256, FEAT, false>), dim3(grid), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweep_direct(bool off64, int cls, const SweepArgs& a, int grid, bool feat,
                               hipStream_t s) {
  if (feat)
    return off64 ? direct_t<int64_t, true>(cls, a, grid, s) : direct_t<int32_t, true>(cls, a, grid, s);
  return off64 ? direct_t<int64_t, false>(cls, a, grid, s) : direct_t<int32_t, false>(cls, a, grid, s);
}

hipError_t launch_hub_direct(bool off64, const HubArgs& a, int grid, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL((k_hub_direct<int64_t, 256>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_hub_direct<int32_t, 256>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep(bool off64, int cls, const SweepArgs& a, int grid, bool feat,
                        hipStream_t s) {
  if (feat && !a.rec) return hipErrorInvalidValue;
  if (off64) return feat ? sweep_t<int64_t, true>(cls, a, grid, s) : sweep_t<int64_t, false>(cls, a, grid, s);
  return feat ? sweep_t<int32_t, true>(cls, a, grid, s) : sweep_t<int32_t, false>(cls, a, grid, s);
}

int hub_bucket_log2(int64_t d, int chunk) {
  int lgb = 0;
  while (lgb < kHubMaxBucketLog2 && ((int64_t)chunk << lgb) < d) ++lgb;
  return lgb;
}

hipError_t launch_hub_part(bool off64, const HubArgs& a, int grid, hipStream_t s) {
  if (a.chunk > (kHubSlots + 1) / 2) return hipErrorInvalidValue;
  if (off64)
    hipLaunchKernelGGL((k_hub_part<int64_t, kHubSlots, kHubThreads>), dim3(grid), dim3(kHubThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_hub_part<int32_t, kHubSlots, kHubThreads>), dim3(grid), dim3(kHubThreads), 0, s, a);
  return hipGetLastError();
}

// grid: workgroups of the large instantiation (one per CU); the small one
// runs four per CU.
hipError_t launch_hub_reduce(bool off64, const HubArgs& a, int grid, hipStream_t s) {
  if (off64) {
    hipLaunchKernelGGL((k_hub_reduce<int64_t, 4095, 256, false>), dim3(4 * grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_hub_reduce<int64_t, kHubSlots, kHubThreads, true>), dim3(grid), dim3(kHubThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_hub_reduce<int32_t, 4095, 256, false>), dim3(4 * grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_hub_reduce<int32_t, kHubSlots, kHubThreads, true>), dim3(grid), dim3(kHubThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_hub_spill(bool off64, const HubArgs& a, int grid, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL((k_hub_spill<int64_t, 256>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_hub_spill<int32_t, 256>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_hub_fin(bool off64, const HubArgs& a, int grid, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL((k_hub_fin<int64_t, 256>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_hub_fin<int32_t, 256>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lpa
