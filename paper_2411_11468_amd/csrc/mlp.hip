// mlp.hip -- the change predictor: a 12 -> 64 -> 64 -> 1 perceptron with ReLU
// hidden layers and a sigmoid output, stored as fp32 master parameters with
// bfloat16 copies for inference.  (A project addition, not in the paper.)
//
// Parameter order (flat, fp32): W1 [12][64], b1 [64], W2 [64][64], b2 [64],
// W3 [64], b3 [1]; W[k][j] multiplies input k into unit j.
//
//   k_mlp_grad    forward + backward of a minibatch, fp32 arithmetic on
//                 bf16-rounded weights and inputs, gradients of the mean
//                 binary cross-entropy with a positive-class weight, summed
//                 into a global gradient with atomics (one workgroup per 64
//                 samples, activations in LDS)
//   k_adam        one Adam step (Kingma & Ba 2015) with bias correction
//   k_mlp_pack    fp32 masters -> bf16 MFMA operand tiles
//   mlp_logit16   inference of 16 samples by one wave with
//                 v_mfma_f32_16x16x16_bf16: every layer is computed
//                 transposed (weights as the A operand, samples as the 16
//                 columns), so a layer's output tile, after bias, ReLU and
//                 bf16 rounding, is the next layer's B operand unchanged
#include <cmath>

#include "lpa_mlp.h"

namespace lpa {

namespace {

constexpr int kIn = 12, kH = 64;
constexpr int oW1 = 0, ob1 = oW1 + kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              oW3 = ob2 + kH, ob3 = oW3 + kH;
static_assert(ob3 + 1 == kMlpParams, "parameter count");

constexpr int kGradSamples = 64;  // samples per workgroup in k_mlp_grad
constexpr int kGradThreads = 256;

}  // namespace

// ---- training -------------------------------------------------------------------
__global__ __launch_bounds__(kGradThreads) void k_mlp_grad(const float* __restrict__ p,
                                                           const float* __restrict__ X,
                                                           const float* __restrict__ y,
                                                           int64_t B, float inv_total,
                                                           float pos_weight, float* grad,
                                                           double* loss) {
  __shared__ float W1[kIn * kH], W2[kH * kH], W3[kH], b1[kH], b2[kH];
  __shared__ float x[kGradSamples][kIn];
  __shared__ float a1[kGradSamples][kH], a2[kGradSamples][kH];
  __shared__ float dz[kGradSamples];
  __shared__ float red[kGradThreads / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < kIn * kH; i += kGradThreads) W1[i] = bf16_round(p[oW1 + i]);
  for (int i = tid; i < kH * kH; i += kGradThreads) W2[i] = bf16_round(p[oW2 + i]);
  for (int i = tid; i < kH; i += kGradThreads) {
    W3[i] = bf16_round(p[oW3 + i]);
    b1[i] = p[ob1 + i];
    b2[i] = p[ob2 + i];
  }
  const float b3 = p[ob3];
  const int64_t s0 = (int64_t)blockIdx.x * kGradSamples;
  const int ns = (int)((B - s0) < kGradSamples ? (B - s0) : kGradSamples);
  for (int i = tid; i < kGradSamples * kIn; i += kGradThreads) {
    const int s = i / kIn, k = i % kIn;
    x[s][k] = s < ns ? bf16_round(X[(s0 + s) * kIn + k]) : 0.0f;
  }
  __syncthreads();
  // forward
  for (int i = tid; i < kGradSamples * kH; i += kGradThreads) {
    const int s = i / kH, j = i % kH;
    float acc = b1[j];
    for (int k = 0; k < kIn; ++k) acc += x[s][k] * W1[k * kH + j];
    a1[s][j] = acc;
  }
  __syncthreads();
  for (int i = tid; i < kGradSamples * kH; i += kGradThreads) {
    const int s = i / kH, j = i % kH;
    float acc = b2[j];
    for (int k = 0; k < kH; ++k) acc += fmaxf(a1[s][k], 0.0f) * W2[k * kH + j];
    a2[s][j] = acc;
  }
  __syncthreads();
  float my_loss = 0.0f;
  if (tid < kGradSamples) {
    const int s = tid;
    float z = b3;
    for (int k = 0; k < kH; ++k) z += fmaxf(a2[s][k], 0.0f) * W3[k];
    float d = 0.0f;
    if (s < ns) {
      const float t = y[s0 + s];
      const float sg = 1.0f / (1.0f + __expf(-z));
      // d/dz of -[pw t log s + (1 - t) log(1 - s)]
      d = (pos_weight * t * (sg - 1.0f) + (1.0f - t) * sg) * inv_total;
      // log sigmoid(z) and log(1 - sigmoid(z)), stable
      const float ls = -(fmaxf(-z, 0.0f) + log1pf(__expf(-fabsf(z))));
      const float l1s = -(fmaxf(z, 0.0f) + log1pf(__expf(-fabsf(z))));
      my_loss = -(pos_weight * t * ls + (1.0f - t) * l1s);
    }
    dz[s] = d;
  }
  for (int ofs = 32; ofs > 0; ofs >>= 1) my_loss += __shfl_xor(my_loss, ofs);
  if ((tid & 63) == 0) red[tid >> 6] = my_loss;
  __syncthreads();
  if (tid == 0) {
    float t = 0.0f;
    for (int q = 0; q < kGradThreads / 64; ++q) t += red[q];
    atomicAdd(loss, (double)t);
  }
  // backward: da2 = dz W3 [a2 > 0] (kept in a2), da1 = da2 W2^T [a1 > 0]
  // gradients of layer 3 use h2 = relu(a2), so take them first
  for (int j = tid; j < kH; j += kGradThreads) {
    float g = 0.0f;
    for (int s = 0; s < kGradSamples; ++s) g += fmaxf(a2[s][j], 0.0f) * dz[s];
    atomicAdd(&grad[oW3 + j], g);
  }
  if (tid == 0) {
    float g = 0.0f;
    for (int s = 0; s < kGradSamples; ++s) g += dz[s];
    atomicAdd(&grad[ob3], g);
  }
  __syncthreads();
  for (int i = tid; i < kGradSamples * kH; i += kGradThreads) {
    const int s = i / kH, j = i % kH;
    a2[s][j] = a2[s][j] > 0.0f ? dz[s] * W3[j] : 0.0f;
  }
  __syncthreads();
  // layer 2 gradients: W2[k][j] += sum_s h1[s][k] da2[s][j]
  for (int i = tid; i < kH * kH; i += kGradThreads) {
    const int k = i / kH, j = i % kH;
    float g = 0.0f;
    for (int s = 0; s < kGradSamples; ++s) g += fmaxf(a1[s][k], 0.0f) * a2[s][j];
    atomicAdd(&grad[oW2 + i], g);
  }
  for (int j = tid; j < kH; j += kGradThreads) {
    float g = 0.0f;
    for (int s = 0; s < kGradSamples; ++s) g += a2[s][j];
    atomicAdd(&grad[ob2 + j], g);
  }
  __syncthreads();
  // da1 (overwrites a1 once every reader above is done)
  float tmp[kGradSamples * kH / kGradThreads];
  for (int q = 0, i = tid; i < kGradSamples * kH; i += kGradThreads, ++q) {
    const int s = i / kH, k = i % kH;
    float acc = 0.0f;
    for (int j = 0; j < kH; ++j) acc += a2[s][j] * W2[k * kH + j];
    tmp[q] = a1[s][k] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  for (int q = 0, i = tid; i < kGradSamples * kH; i += kGradThreads, ++q)
    a1[i / kH][i % kH] = tmp[q];
  __syncthreads();
  for (int i = tid; i < kIn * kH; i += kGradThreads) {
    const int k = i / kH, j = i % kH;
    float g = 0.0f;
    for (int s = 0; s < kGradSamples; ++s) g += x[s][k] * a1[s][j];
    atomicAdd(&grad[oW1 + i], g);
  }
  for (int j = tid; j < kH; j += kGradThreads) {
    float g = 0.0f;
    for (int s = 0; s < kGradSamples; ++s) g += a1[s][j];
    atomicAdd(&grad[ob1 + j], g);
  }
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr,
                       float beta1, float omb1, float beta2, float omb2, float eps, float c1,
                       float c2) {
  // omb = 1 - beta, c1 = 1 - beta1^t, c2 = 1 - beta2^t, each rounded once from
  // fp64 on the host (1 - 0.999f in fp32 would be off by 1e-5 relative)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + omb1 * gi;
    const float vi = beta2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---- inference ----------------------------------------------------------------------
// Operand tiles, one 8-byte group of 4 bf16 per lane and tile:
//   w1t[m][lane]     = W1[4 (lane/16) + j][16 m + lane%16], j = 0..3, zero for
//                      input rows >= 12                       (m = 0..3)
//   w2t[mo][kb][lane] = W2[16 kb + 4 (lane/16) + j][16 mo + lane%16]
__global__ void k_mlp_pack(const float* p, MlpTiles* t) {
  for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) {
    const int m = i / 64, lane = i % 64;
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * (lane / 16) + j, col = 16 * m + lane % 16;
      t->w1t[m][lane][j] = k < kIn ? bf16_bits(p[oW1 + k * kH + col]) : (uint16_t)0;
    }
  }
  for (int i = threadIdx.x; i < 16 * 64; i += blockDim.x) {
    const int mo = i / 256, kb = (i / 64) % 4, lane = i % 64;
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * kb + 4 * (lane / 16) + j, col = 16 * mo + lane % 16;
      t->w2t[mo][kb][lane][j] = bf16_bits(p[oW2 + k * kH + col]);
    }
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    t->b1[i] = p[ob1 + i];
    t->b2[i] = p[ob2 + i];
    t->w3[i] = bf16_round(p[oW3 + i]);
  }
  if (threadIdx.x == 0) t->b3 = p[ob3];
}

__global__ __launch_bounds__(256) void k_mlp_infer(const MlpTiles* t, const float* X, int64_t B,
                                                   float* out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  MlpLane r;
  mlp_load(*t, r);
  for (int64_t s0 = wave * 16; s0 < B; s0 += nw * 16) {
    const int64_t s = s0 + (lane & 15);
    float f[4];
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * (lane >> 4) + j;
      f[j] = (s < B && k < kIn) ? X[s * kIn + k] : 0.0f;
    }
    const float z = mlp_logit16(r, f);
    if (lane < 16 && s < B) out[s] = 1.0f / (1.0f + __expf(-z));
  }
}

__global__ void k_mlp_gather(const float* X, const float* y, const int32_t* idx, int64_t n,
                             float* sX, float* sy) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx[i];
    for (int k = 0; k < kIn; ++k) sX[i * kIn + k] = X[j * kIn + k];
    sy[i] = y[j];
  }
}

hipError_t launch_mlp_gather(const float* X, const float* y, const int32_t* idx, int64_t n,
                             float* sX, float* sy, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_mlp_gather, dim3((unsigned)g), dim3(256), 0, s, X, y, idx, n, sX, sy);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* p, const float* X, const float* y, int64_t B,
                           float pos_weight, float* grad, double* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const int64_t g = (B + kGradSamples - 1) / kGradSamples;
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)g), dim3(kGradThreads), 0, s, p, X, y, B,
                     1.0f / (float)B, pos_weight, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int t, float lr,
                       double beta1, double beta2, float eps, hipStream_t s) {
  const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, g, m, v,
                     kMlpParams, lr, (float)beta1, (float)(1.0 - beta1), (float)beta2,
                     (float)(1.0 - beta2), eps, (float)c1, (float)c2);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(const float* p, MlpTiles* t, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(256), 0, s, p, t);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpTiles* t, const float* X, int64_t B, float* out,
                            hipStream_t s) {
  if (B <= 0) return hipSuccess;
  int64_t g = (B + 63) / 64;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)g), dim3(256), 0, s, t, X, B, out);
  return hipGetLastError();
}

}  // namespace lpa
