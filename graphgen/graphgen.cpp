// graphgen.cpp -- seeded synthetic graph generators (input data only).
//
// This module produces the symmetric CSR inputs that both the GPU library
// and the CPU oracle consume.  It contains no part of the label-propagation
// method.  Every random draw comes from the counter-based generator
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011), keyed by the seed and addressed by a counter
// that names the draw, so the output does not depend on the thread count.
//
// Generators:
//   * planted partition (stochastic block model, Condon & Karp 2001): each
//     unordered pair inside a block is an edge with probability p_in, each
//     pair across blocks with probability p_out; pairs are enumerated with
//     geometric skipping (Batagelj & Brandes 2005), so the cost is linear in
//     the number of edges;
//   * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): 2^scale vertices,
//     edge_factor * 2^scale samples, quadrant probabilities a/b/c/d chosen
//     per bit level, no noise and no vertex permutation;
//   * symmetric integer edge weights from a hash of the unordered pair.
//
// All generators drop self-loops and duplicate edges, add both directions
// and sort every row by target id.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace {

// ---- Philox4x32-10 (Salmon et al. 2011) ------------------------------------
struct P4 { uint32_t v[4]; };

inline void mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

inline P4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo(M0, c0, &hi0, &lo0);
    mulhilo(M1, c2, &hi1, &lo1);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  return P4{{c0, c1, c2, c3}};
}

// Uniform double in [0, 1) from two 32-bit words (53 random bits).
inline double u01(uint32_t hi, uint32_t lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) *
         (1.0 / 9007199254740992.0);
}

// Geometric skip for Bernoulli(p) pair enumeration: number of failures
// before the next success.
inline int64_t geo_skip(double u, double log1mp) {
  if (log1mp == 0.0) return INT64_MAX / 4;   // p == 0: no success ever
  if (std::isinf(log1mp)) return 0;          // p == 1: every pair
  const double s = std::floor(std::log1p(-u) / log1mp);
  return s > 4.0e18 ? (int64_t)4e18 : (int64_t)s;
}

struct Pair { int32_t u, v; };

// Emit the pairs of one SBM region (block a with itself when a == b, else
// block a x block b).  Draw k of the region uses counter (region, k, g, tag).
void sbm_region(int64_t a0, int64_t sa, int64_t b0, int64_t sb, bool same,
                double p, uint32_t region, uint32_t graph, uint32_t k0,
                uint32_t k1, std::vector<Pair>* out) {
  if (p <= 0.0) return;
  const double log1mp = p >= 1.0 ? -INFINITY : std::log1p(-p);
  const int64_t total = same ? sa * (sa - 1) / 2 : sa * sb;
  if (total <= 0) return;
  int64_t idx = -1;
  uint64_t k = 0;
  // For the triangle walk: current row r covers indices [row_lo, row_lo + sa-1-r).
  int64_t r = 0, row_lo = 0;
  for (;;) {
    const P4 x = philox(region, (uint32_t)k, (uint32_t)(k >> 32), graph, k0, k1);
    ++k;
    idx += geo_skip(u01(x.v[0], x.v[1]), log1mp) + 1;
    if (idx >= total) break;
    if (same) {
      while (idx >= row_lo + (sa - 1 - r)) { row_lo += sa - 1 - r; ++r; }
      const int64_t c = r + 1 + (idx - row_lo);
      out->push_back(Pair{(int32_t)(a0 + r), (int32_t)(a0 + c)});
    } else {
      const int64_t r2 = idx / sb, c2 = idx % sb;
      out->push_back(Pair{(int32_t)(a0 + r2), (int32_t)(b0 + c2)});
    }
  }
}

// Build a symmetric CSR (rows sorted, no duplicates, no self-loops) from an
// undirected pair list into caller-visible malloc'd arrays.
struct Csr {
  int64_t n = 0, m = 0;
  int64_t* off = nullptr;
  int32_t* tgt = nullptr;
};

bool csr_from_pairs(int64_t n, const std::vector<Pair>& pairs, Csr* g) {
  std::vector<int64_t> deg(n + 1, 0);
  for (const Pair& p : pairs) {
    if (p.u == p.v) continue;
    ++deg[p.u]; ++deg[p.v];
  }
  g->n = n;
  g->off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  if (!g->off) return false;
  g->off[0] = 0;
  for (int64_t i = 0; i < n; ++i) g->off[i + 1] = g->off[i] + deg[i];
  const int64_t m0 = g->off[n];
  int32_t* t0 = (int32_t*)malloc(sizeof(int32_t) * (m0 > 0 ? m0 : 1));
  if (!t0) return false;
  std::vector<int64_t> cur(g->off, g->off + n);
  for (const Pair& p : pairs) {
    if (p.u == p.v) continue;
    t0[cur[p.u]++] = p.v;
    t0[cur[p.v]++] = p.u;
  }
  // sort + unique each row, then compact
  std::vector<int64_t> nd(n, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b = t0 + g->off[i];
    int32_t* e = t0 + g->off[i + 1];
    std::sort(b, e);
    nd[i] = std::unique(b, e) - b;
  }
  int64_t* noff = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  if (!noff) { free(t0); return false; }
  noff[0] = 0;
  for (int64_t i = 0; i < n; ++i) noff[i + 1] = noff[i] + nd[i];
  g->m = noff[n];
  g->tgt = (int32_t*)malloc(sizeof(int32_t) * (g->m > 0 ? g->m : 1));
  if (!g->tgt) { free(t0); free(noff); return false; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i)
    memcpy(g->tgt + noff[i], t0 + g->off[i], sizeof(int32_t) * nd[i]);
  free(t0);
  free(g->off);
  g->off = noff;
  return true;
}

}  // namespace

extern "C" {

// Raw Philox4x32-10 block (exported for known-answer tests).
void gg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                      uint32_t out[4]) {
  const P4 x = philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
  memcpy(out, x.v, sizeof(x.v));
}

// Handle to a generated CSR held in malloc'd memory until gg_free.
typedef struct gg_graph {
  int64_t n;
  int64_t m;
  int64_t* off;
  int32_t* tgt;
} gg_graph;

void gg_free(gg_graph* g) {
  if (!g) return;
  free(g->off);
  free(g->tgt);
  g->off = nullptr;
  g->tgt = nullptr;
}

// Planted partition on n vertices split into consecutive blocks of the given
// sizes (sum must be n).  Pairs inside block b are edges with probability
// p_in[b]; pairs across blocks with probability p_out.  graph_id separates
// the random streams of graphs generated with one seed.
int gg_sbm(int64_t n, int32_t nblocks, const int64_t* block_sizes,
           const double* p_in, double p_out, uint64_t seed, uint32_t graph_id,
           gg_graph* out) {
  memset(out, 0, sizeof(*out));
  if (n < 0 || nblocks < 0 || n > INT32_MAX) return -1;
  std::vector<int64_t> start(nblocks + 1, 0);
  for (int32_t b = 0; b < nblocks; ++b) start[b + 1] = start[b] + block_sizes[b];
  if (start[nblocks] != n) return -1;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ 0x53424D31u;
  // region id: intra b -> b; inter (a<b) -> nblocks + a*nblocks + b
  const int64_t nreg = (int64_t)nblocks + (int64_t)nblocks * nblocks;
  std::vector<std::vector<Pair>> parts(nblocks);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t a = 0; a < nblocks; ++a) {
    std::vector<Pair>& v = parts[a];
    sbm_region(start[a], block_sizes[a], start[a], block_sizes[a], true,
               p_in[a], (uint32_t)a, graph_id, k0, k1, &v);
    for (int32_t b = a + 1; b < nblocks; ++b) {
      const uint32_t reg = (uint32_t)(nblocks + (int64_t)a * nblocks + b);
      sbm_region(start[a], block_sizes[a], start[b], block_sizes[b], false,
                 p_out, reg, graph_id, k0, k1, &v);
    }
  }
  (void)nreg;
  std::vector<Pair> all;
  size_t tot = 0;
  for (auto& v : parts) tot += v.size();
  all.reserve(tot);
  for (auto& v : parts) all.insert(all.end(), v.begin(), v.end());
  Csr g;
  if (!csr_from_pairs(n, all, &g)) return -2;
  out->n = g.n; out->m = g.m; out->off = g.off; out->tgt = g.tgt;
  return 0;
}

// R-MAT: n = 2^scale, edge_factor * n samples.  At each of the scale bit
// levels (most significant first) the quadrant is chosen with probabilities
// a, b, c, 1-a-b-c from a 16-bit uniform draw; the quadrant (row bit, column
// bit) is (0,0), (0,1), (1,0), (1,1) respectively.  Sample s uses Philox
// counters (s, level group, tag).  Self-loops and duplicates are dropped and
// both directions added.
//
// CSR construction without shared atomics: vertices are split into 2^k
// consecutive bins; pass 1 counts, per thread, the directed entries each bin
// receives; pass 2 regenerates the samples and streams (row, target) pairs
// into per-thread slots of each bin; each bin is then counting-sorted by row
// in cache, rows are sorted and de-duplicated, and the bins are copied into
// the final arrays.
int gg_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c,
            uint64_t seed, gg_graph* out) {
  memset(out, 0, sizeof(*out));
  if (scale < 1 || scale > 30 || edge_factor < 0) return -1;
  const int64_t n = (int64_t)1 << scale;
  const int64_t S = edge_factor * n;
  const uint32_t ta = (uint32_t)std::lround(a * 65536.0);
  const uint32_t tb = (uint32_t)std::lround((a + b) * 65536.0);
  const uint32_t tc = (uint32_t)std::lround((a + b + c) * 65536.0);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ 0x524D4154u;
  auto sample = [&](int64_t s, uint32_t* pu, uint32_t* pv) {
    uint32_t u = 0, v = 0;
    for (int g = 0; g * 8 < scale; ++g) {
      const P4 x = philox((uint32_t)s, (uint32_t)(s >> 32), (uint32_t)g, 0x45444745u, k0, k1);
      for (int q = 0; q < 8 && g * 8 + q < scale; ++q) {
        const uint32_t r = (q & 1) ? (x.v[q >> 1] >> 16) : (x.v[q >> 1] & 0xFFFFu);
        // quadrant a: no bit; b: column bit; c: row bit; d: both
        const int sh = scale - 1 - (g * 8 + q);
        const uint32_t ub = (uint32_t)(r >= tb);
        const uint32_t vb = (uint32_t)(r >= ta) ^ (uint32_t)(r >= tb) ^ (uint32_t)(r >= tc);
        u |= ub << sh;
        v |= vb << sh;
      }
    }
    *pu = u; *pv = v;
  };
  const int bin_bits = std::min(scale, 12);
  const int nb = 1 << bin_bits;
  const int shift = scale - bin_bits;
  const int T = omp_get_max_threads();
  // contiguous sample range per thread, so pass 2 sees the same samples
  std::vector<int64_t> lo(T + 1);
  for (int t = 0; t <= T; ++t) lo[t] = S * t / T;
  std::vector<int64_t> cnt((size_t)T * nb, 0);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    int64_t* my = &cnt[(size_t)t * nb];
    for (int64_t s = lo[t]; s < lo[t + 1]; ++s) {
      uint32_t u, v;
      sample(s, &u, &v);
      if (u == v) continue;
      ++my[u >> shift];
      ++my[v >> shift];
    }
  }
  // bin b, thread t writes at pos[t][b]
  std::vector<int64_t> bin_lo(nb + 1, 0), pos((size_t)T * nb);
  for (int bb = 0; bb < nb; ++bb) {
    int64_t acc = bin_lo[bb];
    for (int t = 0; t < T; ++t) { pos[(size_t)t * nb + bb] = acc; acc += cnt[(size_t)t * nb + bb]; }
    bin_lo[bb + 1] = acc;
  }
  const int64_t m0 = bin_lo[nb];
  uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m0 > 0 ? m0 : 1));
  if (!pairs) return -2;
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    int64_t* my = &pos[(size_t)t * nb];
    for (int64_t s = lo[t]; s < lo[t + 1]; ++s) {
      uint32_t u, v;
      sample(s, &u, &v);
      if (u == v) continue;
      pairs[my[u >> shift]++] = ((uint64_t)u << 32) | v;
      pairs[my[v >> shift]++] = ((uint64_t)v << 32) | u;
    }
  }
  // per bin: counting sort by row, sort + unique rows, targets written back
  // as int32 at the start of the bin's region; deduplicated degrees kept
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!off) { free(pairs); return -2; }
  const int64_t vpb = (int64_t)1 << shift;  // vertices per bin
  std::vector<int> order(nb);
  for (int bb = 0; bb < nb; ++bb) order[bb] = bb;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    return bin_lo[x + 1] - bin_lo[x] > bin_lo[y + 1] - bin_lo[y];
  });
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 1) num_threads(T)
  for (int oi = 0; oi < nb; ++oi) {
    const int bb = order[oi];
    const int64_t e0 = bin_lo[bb], ne = bin_lo[bb + 1] - e0;
    const int64_t v0 = (int64_t)bb << shift;
    std::vector<int64_t> rs(vpb + 1, 0);
    for (int64_t e = 0; e < ne; ++e) ++rs[(pairs[e0 + e] >> 32) - v0 + 1];
    for (int64_t i = 0; i < vpb; ++i) rs[i + 1] += rs[i];
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    if (!tmp) { ok = false; continue; }
    {
      std::vector<int64_t> cur(rs.begin(), rs.end() - 1);
      for (int64_t e = 0; e < ne; ++e) {
        const uint64_t p = pairs[e0 + e];
        tmp[cur[(p >> 32) - v0]++] = (int32_t)(uint32_t)p;
      }
    }
    int32_t* dst = reinterpret_cast<int32_t*>(pairs + e0);
    int64_t w = 0;
    for (int64_t i = 0; i < vpb; ++i) {
      int32_t* rb = tmp + rs[i];
      int32_t* re = tmp + rs[i + 1];
      std::sort(rb, re);
      int32_t* ue = std::unique(rb, re);
      const int64_t k = ue - rb;
      memcpy(dst + w, rb, sizeof(int32_t) * (size_t)k);
      w += k;
      off[v0 + i + 1] = k;  // degree for now
    }
    free(tmp);
  }
  if (!ok) { free(pairs); free(off); return -2; }
  off[0] = 0;
  std::vector<int64_t> bin_out(nb + 1, 0);
  for (int bb = 0; bb < nb; ++bb) {
    int64_t acc = 0;
    for (int64_t i = 0; i < vpb; ++i) acc += off[((int64_t)bb << shift) + i + 1];
    bin_out[bb + 1] = bin_out[bb] + acc;
  }
  for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
  const int64_t m = off[n];
  int32_t* tgt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!tgt) { free(pairs); free(off); return -2; }
#pragma omp parallel for schedule(dynamic, 1) num_threads(T)
  for (int bb = 0; bb < nb; ++bb)
    memcpy(tgt + bin_out[bb], reinterpret_cast<int32_t*>(pairs + bin_lo[bb]),
           sizeof(int32_t) * (size_t)(bin_out[bb + 1] - bin_out[bb]));
  free(pairs);
  out->n = n; out->m = m; out->off = off; out->tgt = tgt;
  return 0;
}

// Many independent planted-partition graphs packed into one CSR.  Graph q
// draws (Philox counter (q, k, 0, tag)) its vertex count n log-uniformly in
// [nmin, nmax], its expected degree d uniformly in [dmin, dmax], its mixing
// mu uniformly in [mumin, mumax], and block sizes uniformly in [bmin, bmax]
// until they cover n (the last block takes the remainder).  Pairs inside a
// block of size b are edges with probability (1 - mu) d / (b - 1), pairs
// across blocks with probability mu d / (n - n/blocks).  Graph q occupies
// global vertices v_off[q] .. v_off[q+1]-1; targets are global ids.
int gg_sbm_batch(int32_t G, uint64_t seed, double nmin, double nmax, double dmin,
                 double dmax, double mumin, double mumax, int32_t bmin, int32_t bmax,
                 int64_t* v_off, gg_graph* out) {
  memset(out, 0, sizeof(*out));
  if (G <= 0 || nmin < 1 || nmax < nmin || bmin < 1 || bmax < bmin) return -1;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ 0x42544348u;
  std::vector<int64_t> n(G);
  std::vector<double> d(G), mu(G);
  std::vector<std::vector<int64_t>> blocks(G);
  for (int32_t q = 0; q < G; ++q) {
    const P4 x = philox((uint32_t)q, 0u, 0u, 0x50415241u, k0, k1);
    const P4 y = philox((uint32_t)q, 1u, 0u, 0x50415241u, k0, k1);
    const double ln = std::log(nmin) + u01(x.v[0], x.v[1]) * (std::log(nmax) - std::log(nmin));
    n[q] = std::min<int64_t>((int64_t)nmax, std::max<int64_t>((int64_t)nmin, (int64_t)std::floor(std::exp(ln))));
    d[q] = dmin + u01(x.v[2], x.v[3]) * (dmax - dmin);
    mu[q] = mumin + u01(y.v[0], y.v[1]) * (mumax - mumin);
    int64_t cov = 0;
    for (uint32_t k = 2; cov < n[q]; ++k) {
      const P4 z = philox((uint32_t)q, k, 0u, 0x424C4B53u, k0, k1);
      int64_t b = bmin + (int64_t)(u01(z.v[0], z.v[1]) * (double)(bmax - bmin + 1));
      if (b > bmax) b = bmax;
      if (cov + b > n[q]) b = n[q] - cov;
      blocks[q].push_back(b);
      cov += b;
    }
  }
  v_off[0] = 0;
  for (int32_t q = 0; q < G; ++q) v_off[q + 1] = v_off[q] + n[q];
  if (v_off[G] > INT32_MAX) return -1;
  std::vector<Csr> part(G);
  std::vector<int32_t> order(G);
  for (int32_t q = 0; q < G; ++q) order[q] = q;
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t oi = 0; oi < G; ++oi) {
    const int32_t q = order[oi];
    const std::vector<int64_t>& bs = blocks[q];
    const int32_t nb = (int32_t)bs.size();
    std::vector<int64_t> start(nb + 1, 0);
    for (int32_t b = 0; b < nb; ++b) start[b + 1] = start[b] + bs[b];
    const double mean_b = (double)n[q] / nb;
    const double p_out = (n[q] - mean_b > 0.0) ? std::min(1.0, mu[q] * d[q] / ((double)n[q] - mean_b)) : 0.0;
    std::vector<Pair> pairs;
    for (int32_t a = 0; a < nb; ++a) {
      const double p_in = bs[a] > 1 ? std::min(1.0, (1.0 - mu[q]) * d[q] / (double)(bs[a] - 1)) : 0.0;
      sbm_region(start[a], bs[a], start[a], bs[a], true, p_in, (uint32_t)a, (uint32_t)q, k0, k1,
                 &pairs);
      for (int32_t b = a + 1; b < nb; ++b)
        sbm_region(start[a], bs[a], start[b], bs[b], false, p_out,
                   (uint32_t)(nb + (int64_t)a * nb + b), (uint32_t)q, k0, k1, &pairs);
    }
    if (!csr_from_pairs(n[q], pairs, &part[q])) ok = false;
  }
  if (!ok) {
    for (Csr& c : part) { free(c.off); free(c.tgt); }
    return -2;
  }
  const int64_t N = v_off[G];
  std::vector<int64_t> e_off(G + 1, 0);
  for (int32_t q = 0; q < G; ++q) e_off[q + 1] = e_off[q] + part[q].m;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N + 1));
  int32_t* tgt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(e_off[G] > 0 ? e_off[G] : 1));
  if (!off || !tgt) {
    free(off); free(tgt);
    for (Csr& c : part) { free(c.off); free(c.tgt); }
    return -2;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t q = 0; q < G; ++q) {
    const Csr& c = part[q];
    for (int64_t i = 0; i < c.n; ++i) off[v_off[q] + i] = e_off[q] + c.off[i];
    const int32_t base = (int32_t)v_off[q];
    for (int64_t e = 0; e < c.m; ++e) tgt[e_off[q] + e] = c.tgt[e] + base;
  }
  off[N] = e_off[G];
  for (Csr& c : part) { free(c.off); free(c.tgt); }
  out->n = N; out->m = e_off[G]; out->off = off; out->tgt = tgt;
  return 0;
}

// LFR-like benchmark graph (after Lancichinetti, Fortunato & Radicchi 2008,
// simplified): degrees from a power law of exponent tau1 on [kmin, kmax] with
// kmin chosen for the requested mean degree; community sizes from a power law
// of exponent tau2 on [cmin, cmax] until they cover n; vertices placed, in
// order of decreasing degree, into a random community large enough for their
// (1 - mu) k intra-community stubs; intra stubs paired uniformly inside each
// community, the remaining mu k stubs paired uniformly across the graph
// (configuration model); self-loops, duplicate pairs and cross stubs that
// land in one community are dropped.  comm_out (n entries, may be NULL)
// receives the planted community of each vertex.
namespace {
double pl_sample(double u, double lo, double hi, double tau) {
  const double a = std::pow(lo, 1.0 - tau), b = std::pow(hi, 1.0 - tau);
  return std::pow(a + u * (b - a), 1.0 / (1.0 - tau));
}
double pl_mean(double lo, double hi, double tau) {
  // mean of the continuous power law on [lo, hi]
  const double z = (std::pow(hi, 1.0 - tau) - std::pow(lo, 1.0 - tau)) / (1.0 - tau);
  const double m = (std::pow(hi, 2.0 - tau) - std::pow(lo, 2.0 - tau)) / (2.0 - tau);
  return m / z;
}
// Fisher-Yates shuffle driven by Philox counters (stream, i).
void shuffle32(std::vector<int32_t>& a, uint32_t stream, uint32_t k0, uint32_t k1) {
  for (int64_t i = (int64_t)a.size() - 1; i > 0; --i) {
    const P4 x = philox(stream, (uint32_t)i, (uint32_t)(i >> 32), 0x53484655u, k0, k1);
    const uint64_t r = ((uint64_t)x.v[0] << 32 | x.v[1]) % (uint64_t)(i + 1);
    std::swap(a[i], a[(int64_t)r]);
  }
}
}  // namespace

int gg_lfr(int64_t n, uint64_t seed, double tau1, double mean_deg, double kmax, double tau2,
           double cmin, double cmax, double mu, int32_t* comm_out, gg_graph* out) {
  memset(out, 0, sizeof(*out));
  if (n < 2 || n > INT32_MAX || mean_deg <= 1.0 || kmax <= mean_deg || mu < 0.0 || mu > 1.0)
    return -1;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ 0x4C465231u;
  // kmin for the requested mean (bisection on the continuous mean)
  double lo = 1.0, hi = mean_deg;
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (pl_mean(mid, kmax, tau1) < mean_deg) lo = mid; else hi = mid;
  }
  const double kmin = 0.5 * (lo + hi);
  std::vector<int32_t> deg(n);
  for (int64_t i = 0; i < n; ++i) {
    const P4 x = philox((uint32_t)i, (uint32_t)(i >> 32), 1u, 0x44454721u, k0, k1);
    deg[i] = (int32_t)std::lround(pl_sample(u01(x.v[0], x.v[1]), kmin, kmax, tau1));
  }
  // community sizes
  std::vector<int64_t> csize;
  int64_t cov = 0;
  for (uint32_t k = 0; cov < n; ++k) {
    const P4 x = philox(k, 0u, 2u, 0x434F4D4Du, k0, k1);
    int64_t c = (int64_t)std::lround(pl_sample(u01(x.v[0], x.v[1]), cmin, cmax, tau2));
    if (cov + c > n) c = n - cov;
    csize.push_back(c);
    cov += c;
  }
  const int32_t nc = (int32_t)csize.size();
  // place vertices by decreasing intra degree into communities with room
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return deg[a] != deg[b] ? deg[a] > deg[b] : a < b;
  });
  std::vector<int64_t> room(csize);
  std::vector<int32_t> comm(n, -1);
  std::vector<int32_t> by_size(nc);
  for (int32_t c = 0; c < nc; ++c) by_size[c] = c;
  std::sort(by_size.begin(), by_size.end(), [&](int32_t a, int32_t b) {
    return csize[a] != csize[b] ? csize[a] > csize[b] : a < b;
  });
  int32_t nfit = 0;  // communities big enough: a prefix of by_size that only grows
  for (int64_t t = 0; t < n; ++t) {
    const int32_t v = order[t];
    const int64_t kin = (int64_t)std::lround((1.0 - mu) * deg[v]);
    while (nfit < nc && csize[by_size[nfit]] - 1 >= kin) ++nfit;
    const int32_t nbig = nfit > 0 ? nfit : 1;
    int32_t pick = -1;
    for (uint32_t tries = 0; tries < 16 && pick < 0; ++tries) {
      const P4 x = philox((uint32_t)v, tries, 3u, 0x504C4143u, k0, k1);
      const int32_t c = by_size[x.v[0] % (uint32_t)nbig];
      if (room[c] > 0) pick = c;
    }
    if (pick < 0) {  // fall back to the community with the most room
      int32_t best = 0;
      for (int32_t c = 1; c < nc; ++c) if (room[c] > room[best]) best = c;
      pick = best;
    }
    comm[v] = pick;
    --room[pick];
  }
  // stubs
  std::vector<std::vector<int32_t>> intra(nc);
  std::vector<int32_t> inter;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t kin = (int32_t)std::lround((1.0 - mu) * deg[v]);
    for (int32_t q = 0; q < kin; ++q) intra[comm[v]].push_back((int32_t)v);
    for (int32_t q = kin; q < deg[v]; ++q) inter.push_back((int32_t)v);
  }
  std::vector<std::vector<Pair>> parts(nc + 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t c = 0; c < nc; ++c) {
    shuffle32(intra[c], (uint32_t)c, k0, k1);
    for (size_t q = 0; q + 1 < intra[c].size(); q += 2)
      if (intra[c][q] != intra[c][q + 1]) parts[c].push_back(Pair{intra[c][q], intra[c][q + 1]});
  }
  shuffle32(inter, 0xFFFFFFFFu, k0, k1);
  for (size_t q = 0; q + 1 < inter.size(); q += 2)
    if (comm[inter[q]] != comm[inter[q + 1]]) parts[nc].push_back(Pair{inter[q], inter[q + 1]});
  std::vector<Pair> all;
  for (auto& p : parts) all.insert(all.end(), p.begin(), p.end());
  Csr g;
  if (!csr_from_pairs(n, all, &g)) return -2;
  if (comm_out) for (int64_t v = 0; v < n; ++v) comm_out[v] = comm[v];
  out->n = g.n; out->m = g.m; out->off = g.off; out->tgt = g.tgt;
  return 0;
}

// Symmetric integer weights: w(u,v) = 1 + (h(min(u,v), max(u,v)) mod wmax)
// where h is the first Philox word of counter (min, max) under the seed.
// Road-like lattice: vertex (r, c) of a rows x cols grid has id r*cols + c;
// each lattice edge -- right (r, c)-(r, c+1) and down (r, c)-(r+1, c) --
// exists with probability keep, drawn from the edge's own counter.  Rows
// come out sorted (up, left, right, down neighbours in id order).
static inline bool gg_lattice_edge(uint64_t u, uint32_t dir, double keep, uint32_t k0,
                                   uint32_t k1) {
  const P4 x = philox((uint32_t)u, (uint32_t)(u >> 32), dir, 0x524F4144u, k0, k1);
  return u01(x.v[0], x.v[1]) < keep;
}

int gg_lattice(int64_t rows, int64_t cols, double keep, uint64_t seed, gg_graph* out) {
  if (rows <= 0 || cols <= 0 || !(keep >= 0.0 && keep <= 1.0)) return -1;
  const int64_t n = rows * cols;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ 0x4C415454u;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!off) return -2;
  // right(u) and down(u) decide the two edges owned by u
  auto right = [&](int64_t u) {
    return (u % cols) + 1 < cols && gg_lattice_edge((uint64_t)u, 0u, keep, k0, k1);
  };
  auto down = [&](int64_t u) {
    return u / cols + 1 < rows && gg_lattice_edge((uint64_t)u, 1u, keep, k0, k1);
  };
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < n; ++u) {
    int64_t d = 0;
    if (u >= cols && down(u - cols)) ++d;
    if (u % cols > 0 && right(u - 1)) ++d;
    if (right(u)) ++d;
    if (down(u)) ++d;
    off[u + 1] = d;
  }
  off[0] = 0;
  for (int64_t u = 0; u < n; ++u) off[u + 1] += off[u];
  const int64_t m = off[n];
  int32_t* tgt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!tgt) { free(off); return -2; }
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < n; ++u) {
    int64_t p = off[u];
    if (u >= cols && down(u - cols)) tgt[p++] = (int32_t)(u - cols);
    if (u % cols > 0 && right(u - 1)) tgt[p++] = (int32_t)(u - 1);
    if (right(u)) tgt[p++] = (int32_t)(u + 1);
    if (down(u)) tgt[p++] = (int32_t)(u + cols);
  }
  out->n = n;
  out->m = m;
  out->off = off;
  out->tgt = tgt;
  return 0;
}

void gg_pair_weights(int64_t n, const int64_t* off, const int32_t* tgt,
                     uint64_t seed, int32_t wmax, float* w) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ 0x57454947u;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      const uint32_t x = (uint32_t)std::min<int64_t>(i, tgt[e]);
      const uint32_t y = (uint32_t)std::max<int64_t>(i, tgt[e]);
      const P4 r = philox(x, y, 0u, 0x57u, k0, k1);
      w[e] = (float)(1 + (int32_t)(r.v[0] % (uint32_t)wmax));
    }
  }
}

// Parallel fill of a float array (unit weights for large graphs).
void gg_fill_f32(int64_t m, float value, float* w) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) w[e] = value;
}

// Copy a generated CSR into caller buffers (offsets as int64 or int32).
int gg_copy_out(const gg_graph* g, int64_t* off64, int32_t* off32,
                int32_t* tgt) {
  if (off64) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i <= g->n; ++i) off64[i] = g->off[i];
  }
  if (off32) {
    if (g->m > INT32_MAX) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i <= g->n; ++i) off32[i] = (int32_t)g->off[i];
  }
  if (tgt) {
    const int64_t chunk = 1 << 22;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < g->m; s += chunk) {
      const int64_t len = std::min<int64_t>(chunk, g->m - s);
      memcpy(tgt + s, g->tgt + s, sizeof(int32_t) * len);
    }
  }
  return 0;
}

int gg_max_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
