// lpa_mlp.h -- change-predictor network: parameter layout, bfloat16 helpers
// and the one-wave MFMA inference routine shared by mlp.hip and the frontier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpa {

constexpr int kMlpIn = 12;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;  // 5,057

// bfloat16 = the upper 16 bits of an IEEE binary32; round to nearest, ties to
// even (NaN kept quiet).
__host__ __device__ inline uint16_t bf16_bits(float x) {
  union { float f; uint32_t u; } c;
  c.f = x;
  if ((c.u & 0x7F800000u) == 0x7F800000u && (c.u & 0x007FFFFFu))
    return (uint16_t)((c.u >> 16) | 0x0040u);
  c.u += 0x7FFFu + ((c.u >> 16) & 1u);
  return (uint16_t)(c.u >> 16);
}
__host__ __device__ inline float bf16_round(float x) {
  union { float f; uint32_t u; } c;
  c.u = (uint32_t)bf16_bits(x) << 16;
  return c.f;
}

// MFMA operand tiles of the bf16 weights (see k_mlp_pack) and fp32 biases.
struct MlpTiles {
  uint16_t w1t[4][64][4];
  uint16_t w2t[4][4][64][4];
  float b1[kMlpHidden];
  float b2[kMlpHidden];
  float w3[kMlpHidden];
  float b3;
};

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// The operands one lane needs, held in registers across many calls: the
// layer-1 and layer-2 A tiles, and the biases / output weights of the hidden
// units u = 16 m + 4 (lane / 16) + i that the lane's accumulator rows hold.
struct MlpLane {
  bf16x4_t w1[4];
  bf16x4_t w2[4][4];
  float b1[16], b2[16], w3[16];  // index 4 m + i
  float b3;
};

__device__ inline void mlp_load(const MlpTiles& t, MlpLane& r) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    r.w1[m] = *reinterpret_cast<const bf16x4_t*>(t.w1t[m][lane]);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      r.w2[m][kb] = *reinterpret_cast<const bf16x4_t*>(t.w2t[m][kb][lane]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int u = 16 * m + 4 * g + i;
      r.b1[4 * m + i] = t.b1[u];
      r.b2[4 * m + i] = t.b2[u];
      r.w3[4 * m + i] = t.w3[u];
    }
  }
  r.b3 = t.b3;
}

// Operand sources for mlp_logit16: the registers of an MlpLane, or the
// tiles themselves (e.g. a copy in LDS), read at each use so that they hold
// no registers between calls.
struct MlpFromRegs {
  const MlpLane& r;
  __device__ bf16x4_t w1(int m) const { return r.w1[m]; }
  __device__ bf16x4_t w2(int m, int kb) const { return r.w2[m][kb]; }
  __device__ float b1(int m, int i) const { return r.b1[4 * m + i]; }
  __device__ float b2(int m, int i) const { return r.b2[4 * m + i]; }
  __device__ float w3(int m, int i) const { return r.w3[4 * m + i]; }
  __device__ float b3() const { return r.b3; }
};
struct MlpFromTiles {
  const MlpTiles& t;
  int lane, g;
  __device__ bf16x4_t w1(int m) const {
    return *reinterpret_cast<const bf16x4_t*>(t.w1t[m][lane]);
  }
  __device__ bf16x4_t w2(int m, int kb) const {
    return *reinterpret_cast<const bf16x4_t*>(t.w2t[m][kb][lane]);
  }
  __device__ float b1(int m, int i) const { return t.b1[16 * m + 4 * g + i]; }
  __device__ float b2(int m, int i) const { return t.b2[16 * m + 4 * g + i]; }
  __device__ float w3(int m, int i) const { return t.w3[16 * m + 4 * g + i]; }
  __device__ float b3() const { return t.b3; }
};

// Logit for 16 samples, one wave: lane l holds features 4 (l/16) .. 4 (l/16)+3
// of sample l % 16 in f (zero beyond feature 11); every lane returns the logit
// of its sample.  Layer 1 and 2 run on v_mfma_f32_16x16x16_bf16 with the
// weights as the A operand and the 16 samples as the columns, so the output
// tile of layer 1 (after bias, ReLU and bf16 rounding) is the B operand of
// layer 2 as it stands.  Layer 3 is a fp32 dot product.  All 64 lanes must be
// active.  The same operations in the same order whatever the source.
template <typename Src>
__device__ inline float mlp_logit16_src(const Src& r, const float f[4]) {
  bf16x4_t xb;
  for (int j = 0; j < 4; ++j) xb[j] = (short)bf16_bits(f[j]);
  bf16x4_t h1[4];
  const f32x4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const f32x4_t acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r.w1(m), xb, zero, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) h1[m][i] = (short)bf16_bits(fmaxf(acc[i] + r.b1(m, i), 0.0f));
  }
  float part = 0.0f;
#pragma unroll
  for (int mo = 0; mo < 4; ++mo) {
    f32x4_t acc = zero;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r.w2(mo, kb), h1[kb], acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) part += fmaxf(acc[i] + r.b2(mo, i), 0.0f) * r.w3(mo, i);
  }
  part += __shfl_xor(part, 16);
  part += __shfl_xor(part, 32);
  return part + r.b3();
}

__device__ inline float mlp_logit16(const MlpLane& r, const float f[4]) {
  return mlp_logit16_src(MlpFromRegs{r}, f);
}

hipError_t launch_mlp_grad(const float* p, const float* X, const float* y, int64_t B,
                           float pos_weight, float* grad, double* loss, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int t, float lr,
                       double beta1, double beta2, float eps, hipStream_t s);
hipError_t launch_mlp_pack(const float* p, MlpTiles* t, hipStream_t s);
hipError_t launch_mlp_gather(const float* X, const float* y, const int32_t* idx, int64_t n,
                             float* sX, float* sy, hipStream_t s);
hipError_t launch_mlp_infer(const MlpTiles* t, const float* X, int64_t B, float* out,
                            hipStream_t s);

}  // namespace lpa
