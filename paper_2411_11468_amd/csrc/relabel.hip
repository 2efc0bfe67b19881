// Internal vertex order of a handle: vertices sorted by degree, largest
// first, in 8 steps per octave, ties kept in id order.
//
// Every sweep after the first gathers the current label of each neighbour,
// one 4-byte read at a data-dependent address per CSR entry.  On graphs
// whose ids carry no locality (R-MAT, random orders) almost every such read
// misses in the 4 MB L2 of its XCD and costs a whole cache line.  The number
// of reads that land on a vertex is its degree, so packing the large-degree
// vertices into the lowest ids concentrates the reads on few lines, which
// then stay in L2 and the memory-side cache.
//
// The order changes only where labels live in memory, never their values:
// label values stay the caller's vertex ids, so Eq. 3's tie to the smallest
// label, the Pick-Less comparison and the result are those of the caller's
// order (a deterministic run gives the same labels, an asynchronous run
// differs only in the order in which it sees updates, which the method
// leaves free).
//
//   perm[v]  = internal id of the caller's vertex v
//   inv[v']  = caller's id of internal vertex v'
// The internal CSR keeps each row's entries in the caller's order, with
// targets mapped through perm.
#include <vector>

#include "lpa_device.h"
#include "lpa_internal.h"

namespace lpa {

namespace {

int rl_grid(int64_t n, int per_block, int cap) {
  const int64_t g = (n + per_block - 1) / per_block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

constexpr int kRlThreads = 256;
constexpr int kRlTile = 4096;                  // vertices per tile
constexpr int kRlRounds = kRlTile / kRlThreads;
constexpr int kRlBins = 256;
constexpr int kScanItems = 16;                 // per thread
constexpr int kScanChunk = kRlThreads * kScanItems;

// Sorted bin of a degree, 0 for the largest: degrees below 16 get a bin
// each, larger ones 8 linear steps per octave (the three bits after the
// leading one).
__device__ __forceinline__ uint32_t degree_bin(int64_t d) {
  uint32_t key;
  if (d < 16) {
    key = (uint32_t)d;
  } else {
    const uint64_t u = (uint64_t)d;
    const int e = 63 - __clzll((long long)u);   // floor(log2 d) >= 4
    key = 8u * (uint32_t)(e - 2) + (uint32_t)((u >> (e - 3)) & 7u);
  }
  if (key > (uint32_t)(kRlBins - 1)) key = kRlBins - 1;  // degrees of 2^32 and more
  return (uint32_t)(kRlBins - 1) - key;
}

template <typename OffT>
__device__ __forceinline__ int64_t degree_of(const OffT* off, int64_t v) {
  return (int64_t)off[v + 1] - (int64_t)off[v];
}

}  // namespace

// Per tile: how many of its vertices fall in each bin (bin-major layout, so
// that one exclusive scan gives every (bin, tile) its first position).
template <typename OffT>
__global__ __launch_bounds__(kRlThreads) void k_rl_hist(const OffT* off, int64_t n,
                                                        int64_t ntiles, int64_t* cnt) {
  __shared__ uint32_t hist[kRlBins];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    hist[threadIdx.x] = 0u;
    __syncthreads();
    for (int r = 0; r < kRlRounds; ++r) {
      const int64_t v = t * kRlTile + (int64_t)r * kRlThreads + threadIdx.x;
      if (v < n) atomicAdd(&hist[degree_bin(degree_of(off, v))], 1u);
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * ntiles + t] = hist[threadIdx.x];
    __syncthreads();
  }
}

// Stable scatter: a vertex goes to the first position of its (bin, tile)
// plus the number of same-bin vertices before it in the tile.  Each round
// takes 256 consecutive vertices; lanes of a wave with equal bins find each
// other by one ballot per bin bit.
template <typename OffT>
__global__ __launch_bounds__(kRlThreads) void k_rl_scatter(const OffT* off, int64_t n,
                                                           int64_t ntiles, const int64_t* pos,
                                                           int32_t* inv, int32_t* perm) {
  constexpr int kWaves = kRlThreads / 64;
  __shared__ uint32_t run[kRlBins];
  __shared__ uint32_t wcnt[kWaves][kRlBins];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    run[tid] = 0u;
    for (int r = 0; r < kRlRounds; ++r) {
      const int64_t v = t * kRlTile + (int64_t)r * kRlThreads + tid;
      const bool valid = v < n;
      const uint32_t b = valid ? degree_bin(degree_of(off, v)) : 0u;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) wcnt[q][tid] = 0u;
      __syncthreads();
      unsigned long long peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool set = (b >> bit) & 1u;
        const unsigned long long bal = __ballot(set);
        peers &= set ? bal : ~bal;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lt);
      if (valid && rank == 0) wcnt[wv][b] = (uint32_t)__popcll(peers);
      __syncthreads();
      if (valid) {
        uint32_t before = run[b] + rank;
        for (int q = 0; q < wv; ++q) before += wcnt[q][b];
        const int64_t p = pos[(int64_t)b * ntiles + t] + before;
        inv[p] = (int32_t)v;
        perm[v] = (int32_t)p;
      }
      __syncthreads();
      uint32_t add = 0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) add += wcnt[q][tid];
      run[tid] += add;
      __syncthreads();
    }
  }
}

// Exclusive scan of chunks of kScanChunk items; chunk totals to sums.  In
// place is allowed: every thread reads its own items before writing them.
__global__ __launch_bounds__(kRlThreads) void k_scan_chunks(const int64_t* in, int64_t* out,
                                                            int64_t L, int64_t* sums) {
  constexpr int kWaves = kRlThreads / 64;
  __shared__ int64_t wtot[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)tid * kScanItems;
  int64_t x[kScanItems];
  int64_t tot = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    x[i] = (base + i < L) ? in[base + i] : 0;
    const int64_t y = x[i];
    x[i] = tot;
    tot += y;
  }
  // inclusive scan of the thread totals inside the wave, then across waves
  int64_t inc = tot;
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  int64_t before = inc - tot;
  for (int q = 0; q < wv; ++q) before += wtot[q];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < L) out[base + i] = x[i] + before;
  if (tid == kRlThreads - 1) {
    int64_t s = 0;
    for (int q = 0; q < kWaves; ++q) s += wtot[q];
    sums[blockIdx.x] = s;
  }
}

__global__ void k_scan_add(int64_t* out, int64_t L, const int64_t* sums) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < L;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] += sums[i / kScanChunk];
}

// d[v'] = degree of the caller's vertex inv[v']; d[n] = 0.
template <typename OffT>
__global__ void k_rl_degrees(const OffT* off, const int32_t* inv, int64_t n, int64_t* d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (i < n) ? degree_of(off, inv[i]) : 0;
}

template <typename OffT>
__global__ void k_rl_store_offsets(const int64_t* excl, int64_t n, OffT* noff) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x)
    noff[i] = (OffT)excl[i];
}

// One wave per internal row: the caller's row of inv[v'], entries in the
// same order, targets through perm.
template <typename OffT>
__global__ __launch_bounds__(kRlThreads) void k_rl_rows(const OffT* uoff, const int32_t* utgt,
                                                        const float* uw, const int32_t* inv,
                                                        const int32_t* perm, const int64_t* noff,
                                                        int64_t n, int32_t* ntgt, float* nw) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kRlThreads + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kRlThreads) >> 6;
  for (int64_t vi = wave; vi < n; vi += nwaves) {
    const int32_t v = inv[vi];
    const int64_t src = (int64_t)uoff[v];
    const int64_t d = (int64_t)uoff[v + 1] - src;
    const int64_t dst = noff[vi];
    for (int64_t e = lane; e < d; e += 64) {
      ntgt[dst + e] = perm[utgt[src + e]];
      if (nw) nw[dst + e] = uw[src + e];
    }
  }
}

// Share of CSR entries whose target lies within 2^16 ids of the row's
// vertex, over every stride-th row (at most 1024 entries per row): acc[0]
// near entries, acc[1] all entries.
template <typename OffT>
__global__ void k_rl_locality(const OffT* off, const int32_t* tgt, int64_t n, int64_t stride,
                              unsigned long long* acc) {
  unsigned long long near = 0, all = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i * stride < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i * stride;
    const int64_t o = (int64_t)off[v];
    int64_t d = (int64_t)off[v + 1] - o;
    if (d > 1024) d = 1024;
    for (int64_t e = 0; e < d; ++e) {
      const int64_t j = tgt[o + e];
      near += (j - v < 65536 && v - j < 65536) ? 1u : 0u;
    }
    all += (unsigned long long)d;
  }
  if (near) atomicAdd(&acc[0], near);
  if (all) atomicAdd(&acc[1], all);
}

namespace {

// Device buffers freed when the builder returns.
struct Scratch {
  std::vector<void*> p;
  ~Scratch() { for (void* q : p) (void)hipFree(q); }
  template <typename T>
  hipError_t get(T** out, int64_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, sizeof(T) * (size_t)(count > 0 ? count : 1));
    if (e != hipSuccess) return e;
    p.push_back(q);
    *out = static_cast<T*>(q);
    return hipSuccess;
  }
};

#define RL_TRY(x)                          \
  do {                                     \
    const hipError_t rl_e = (x);           \
    if (rl_e != hipSuccess) return rl_e;   \
  } while (0)

hipError_t scan_exclusive(Scratch& sc, const int64_t* in, int64_t* out, int64_t L,
                          hipStream_t s) {
  if (L <= 0) return hipSuccess;
  const int64_t nch = (L + kScanChunk - 1) / kScanChunk;
  int64_t* sums = nullptr;
  RL_TRY(sc.get(&sums, nch));
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nch), dim3(kRlThreads), 0, s, in, out, L,
                     sums);
  RL_TRY(hipGetLastError());
  if (nch > 1) {
    RL_TRY(scan_exclusive(sc, sums, sums, nch, s));
    hipLaunchKernelGGL(k_scan_add, dim3(rl_grid(L, 256, 8192)), dim3(256), 0, s, out, L,
                       (const int64_t*)sums);
    RL_TRY(hipGetLastError());
  }
  return hipSuccess;
}

template <typename OffT>
hipError_t build_t(const OffT* uoff, const int32_t* utgt, const float* uw, int64_t n,
                   int32_t* perm, int32_t* inv, OffT* noff, int32_t* ntgt, float* nw,
                   hipStream_t s) {
  Scratch sc;
  const int64_t ntiles = (n + kRlTile - 1) / kRlTile;
  const int grid_t = (int)(ntiles < 8192 ? ntiles : 8192);
  int64_t* cnt = nullptr;
  RL_TRY(sc.get(&cnt, (int64_t)kRlBins * ntiles));
  hipLaunchKernelGGL(k_rl_hist<OffT>, dim3(grid_t), dim3(kRlThreads), 0, s, uoff, n, ntiles,
                     cnt);
  RL_TRY(hipGetLastError());
  RL_TRY(scan_exclusive(sc, cnt, cnt, (int64_t)kRlBins * ntiles, s));
  hipLaunchKernelGGL(k_rl_scatter<OffT>, dim3(grid_t), dim3(kRlThreads), 0, s, uoff, n, ntiles,
                     (const int64_t*)cnt, inv, perm);
  RL_TRY(hipGetLastError());
  int64_t* deg = nullptr;
  RL_TRY(sc.get(&deg, n + 1));
  hipLaunchKernelGGL(k_rl_degrees<OffT>, dim3(rl_grid(n + 1, 256, 8192)), dim3(256), 0, s,
                     uoff, (const int32_t*)inv, n, deg);
  RL_TRY(hipGetLastError());
  RL_TRY(scan_exclusive(sc, deg, deg, n + 1, s));
  hipLaunchKernelGGL(k_rl_store_offsets<OffT>, dim3(rl_grid(n + 1, 256, 8192)), dim3(256), 0,
                     s, (const int64_t*)deg, n, noff);
  RL_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_rl_rows<OffT>, dim3(rl_grid(n, kRlThreads / 64, 8192)),
                     dim3(kRlThreads), 0, s, uoff, utgt, uw, (const int32_t*)inv,
                     (const int32_t*)perm, (const int64_t*)deg, n, ntgt, nw);
  RL_TRY(hipGetLastError());
  // the scratch buffers are freed on return: let the kernels finish first
  return hipStreamSynchronize(s);
}

}  // namespace

hipError_t relabel_build(bool off64, const void* uoff, const int32_t* utgt, const float* uw,
                         int64_t n, int32_t* perm, int32_t* inv, void* noff, int32_t* ntgt,
                         float* nw, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (off64)
    return build_t<int64_t>(static_cast<const int64_t*>(uoff), utgt, uw, n, perm, inv,
                            static_cast<int64_t*>(noff), ntgt, nw, s);
  return build_t<int32_t>(static_cast<const int32_t*>(uoff), utgt, uw, n, perm, inv,
                          static_cast<int32_t*>(noff), ntgt, nw, s);
}

hipError_t relabel_locality(bool off64, const void* off, const int32_t* tgt, int64_t n,
                            unsigned long long* acc, hipStream_t s) {
  RL_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 0u, 4, s));
  if (n <= 0) return hipSuccess;
  const int64_t stride = n > 65536 ? n / 65536 : 1;
  if (off64)
    hipLaunchKernelGGL(k_rl_locality<int64_t>, dim3(256), dim3(256), 0, s,
                       static_cast<const int64_t*>(off), tgt, n, stride, acc);
  else
    hipLaunchKernelGGL(k_rl_locality<int32_t>, dim3(256), dim3(256), 0, s,
                       static_cast<const int32_t*>(off), tgt, n, stride, acc);
  return hipGetLastError();
}

// out[i] = in[idx[i]] for 4-, 1- and 8-byte arrays: per-vertex arrays put
// back into the caller's order (idx = perm), or the internal targets mapped
// to the caller's ids (in = inv, idx = the internal targets).
template <typename T>
__global__ void k_unpermute(const T* in, const int32_t* perm, int64_t n, T* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[perm[i]];
}

hipError_t launch_unpermute_i32(const int32_t* in, const int32_t* perm, int64_t n, int32_t* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute<int32_t>, dim3(rl_grid(n, 256, 8192)), dim3(256), 0, s, in,
                     perm, n, out);
  return hipGetLastError();
}
hipError_t launch_unpermute_u8(const uint8_t* in, const int32_t* perm, int64_t n, uint8_t* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute<uint8_t>, dim3(rl_grid(n, 256, 8192)), dim3(256), 0, s, in,
                     perm, n, out);
  return hipGetLastError();
}
hipError_t launch_unpermute_u64(const unsigned long long* in, const int32_t* perm, int64_t n,
                                unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute<unsigned long long>, dim3(rl_grid(n, 256, 8192)), dim3(256),
                     0, s, in, perm, n, out);
  return hipGetLastError();
}

}  // namespace lpa
