// lpa_record.h -- the per-vertex state record of the learned variant (a
// project addition, not in the paper), written by the sweep kernels and read
// by the frontier that runs the change predictor.
//
// Record (8 bytes, byte i = bits 8i..8i+7), from the label sums of the
// vertex's last evaluation (self-loops skipped; K = total neighbour weight,
// own = weight of the vertex's label, best / second = the two largest label
// weights, distinct = number of labels, D = row length):
//   0 q(own)   1 q(best - second)   2 q(best - own)   with q(x) = floor(255 x / K)
//   3 floor(255 distinct / D)   4 lq(1 + D)   5 lq(fp32 value 1 + K)
//   6 change history: bit k = changed when evaluated k iterations before
//     byte 7's iteration (bits 0..6); bit 7 = predicted unchanged in the
//     current plain iteration (set by the frontier, cleared here)
//   7 iteration of the evaluation (at most 254; 255 = never)
// lq(u) = min(255, 8 floor(log2 u) + the three bits after the leading one).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpa {

__device__ __forceinline__ uint32_t rec_q255(float x, float K) {
  if (!(K > 0.0f)) return 0u;
  const float t = floorf((255.0f * x) / K);
  return t >= 255.0f ? 255u : (t <= 0.0f ? 0u : (uint32_t)t);
}

__device__ __forceinline__ uint32_t rec_lq_int(uint32_t u) {  // u >= 1
  const int e = 31 - __clz(u);
  const uint32_t m = e >= 3 ? (u >> (e - 3)) & 7u : (u << (3 - e)) & 7u;
  const uint32_t q = 8u * (uint32_t)e + m;
  return q > 255u ? 255u : q;
}

__device__ __forceinline__ uint32_t rec_lq_float(float x) {  // x >= 1
  const uint32_t b = __float_as_uint(x);
  const int q = 8 * ((int)(b >> 23) - 127) + (int)((b >> 20) & 7u);
  return q > 255 ? 255u : (q < 0 ? 0u : (uint32_t)q);
}

// Rewrite the record of v after its evaluation in iteration l, given its
// previous value `old` (loaded by the caller when the vertex's evaluation
// starts, so that the read's latency hides behind the row scan); returns 1
// when the vertex had been predicted unchanged in this plain iteration and
// moved.
__device__ __forceinline__ uint32_t rec_write(unsigned long long* rec, int32_t v,
                                              unsigned long long old, int l, float K,
                                              float own, float bw, float second,
                                              uint32_t distinct, uint32_t d, bool moved) {
  const uint32_t hist = (uint32_t)(old >> 48) & 0xFFu;
  const uint32_t lu = (uint32_t)(old >> 56);
  const int shift = lu == 255u ? 8 : l - (int)lu;
  const uint32_t h =
      ((shift >= 8 ? 0u : ((hist & 0x7Fu) << shift)) | (moved ? 1u : 0u)) & 0x7Fu;
  const unsigned long long r =
      (unsigned long long)rec_q255(own, K) |
      ((unsigned long long)rec_q255(bw - second, K) << 8) |
      ((unsigned long long)rec_q255(bw - own, K) << 16) |
      ((unsigned long long)((255u * distinct) / d) << 24) |
      ((unsigned long long)rec_lq_int(d + 1u) << 32) |
      ((unsigned long long)rec_lq_float(1.0f + K) << 40) |
      ((unsigned long long)h << 48) |
      ((unsigned long long)(l < 254 ? l : 254) << 56);
  rec[v] = r;
  return ((hist & 0x80u) && moved) ? 1u : 0u;
}

// Features of a record at the start of iteration l (cap = iteration cap,
// rho = Pick-Less period); feature j for j = 4 g .. 4 g + 3 into f[0..3]
// (zero beyond feature 11).
__device__ __forceinline__ void rec_features(unsigned long long r, int l, int cap, int rho,
                                             int g, float f[4]) {
  const uint32_t b7 = (uint32_t)(r >> 56);
  const uint32_t hist = (uint32_t)(r >> 48) & 0x7Fu;
  const bool never = b7 == 255u;
  const int age = never ? cap : l - (int)b7;
  auto byte = [&](int i) { return (float)((uint32_t)(r >> (8 * i)) & 0xFFu); };
  auto changed = [&](int j) {  // changed in iteration l - j
    const int k = j - age;
    return (!never && k >= 0 && k <= 6) ? (float)((hist >> k) & 1u) : 0.0f;
  };
  if (g == 0) {
    f[0] = byte(4) / 64.0f;
    f[1] = byte(5) / 64.0f;
    f[2] = byte(0) / 255.0f;
    f[3] = byte(1) / 255.0f;
  } else if (g == 1) {
    f[0] = byte(2) / 255.0f;
    f[1] = changed(1);
    f[2] = changed(2);
    f[3] = changed(3);
  } else if (g == 2) {
    f[0] = (float)l / (float)cap;
    f[1] = (rho > 0 && l % rho == 0) ? 1.0f : 0.0f;
    f[2] = (float)(age < cap ? age : cap) / (float)cap;
    f[3] = byte(3) / 255.0f;
  } else {
    f[0] = f[1] = f[2] = f[3] = 0.0f;
  }
}

}  // namespace lpa
