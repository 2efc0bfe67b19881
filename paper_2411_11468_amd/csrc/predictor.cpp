// predictor.cpp -- host side of the change predictor (lpa_predictor_* calls):
// device parameters, gradient, Adam, minibatch training and prediction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "host_common.h"
#include "lpa_mlp.h"

using namespace lpa;

struct lpa_predictor_s {
  hipStream_t stream = nullptr;
  float* p = nullptr;      // fp32 master parameters
  float* g = nullptr;      // gradient
  float* m = nullptr;      // Adam first moment
  float* v = nullptr;      // Adam second moment
  double* loss = nullptr;  // summed loss of the last gradient
  MlpTiles* tiles = nullptr;
  bool tiles_ok = false;
  int32_t steps = 0;       // Adam steps taken
  std::vector<void*> allocs;

  template <typename T>
  lpa_status alloc(T** out, size_t count) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LPA_ERR_OOM, std::string("hipMalloc failed for the predictor: ") +
                                   hipGetErrorString(e));
    }
    allocs.push_back(q);
    *out = static_cast<T*>(q);
    return LPA_OK;
  }
  ~lpa_predictor_s() {
    for (void* q : allocs) (void)hipFree(q);
  }
};

namespace {

// Copy n elements from host or device memory to a device buffer (staging).
template <typename T>
lpa_status to_device(const T* src, size_t n, T** dev, std::vector<void*>* tmp, hipStream_t s) {
  if (is_device_ptr(src)) {
    *dev = const_cast<T*>(src);
    return LPA_OK;
  }
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LPA_ERR_OOM, "hipMalloc failed staging predictor input");
  }
  tmp->push_back(q);
  LPA_HIP(hipMemcpyAsync(q, src, n * sizeof(T), hipMemcpyHostToDevice, s));
  *dev = static_cast<T*>(q);
  return LPA_OK;
}

struct Staging {
  std::vector<void*> bufs;
  ~Staging() {
    for (void* q : bufs) (void)hipFree(q);
  }
};

lpa_status pack(lpa_predictor p) {
  if (!p->tiles_ok) {
    LPA_HIP(launch_mlp_pack(p->p, p->tiles, p->stream));
    p->tiles_ok = true;
  }
  return LPA_OK;
}

}  // namespace

namespace lpa {
const MlpTiles* predictor_tiles(lpa_predictor p) {
  if (!p) return nullptr;
  if (!p->tiles_ok) {
    if (pack(p) != LPA_OK || hipStreamSynchronize(p->stream) != hipSuccess) return nullptr;
  }
  return p->tiles;
}
}  // namespace lpa

extern "C" {

lpa_status lpa_predictor_create(uint64_t seed, void* stream, lpa_predictor* out) {
  if (!out) return fail(LPA_ERR_INVALID, "out is NULL");
  *out = nullptr;
  lpa_predictor p = new (std::nothrow) lpa_predictor_s();
  if (!p) return fail(LPA_ERR_OOM, "host allocation failed");
  p->stream = (hipStream_t)stream;
  lpa_status e = LPA_OK;
  if ((e = p->alloc(&p->p, kMlpParams)) || (e = p->alloc(&p->g, kMlpParams)) ||
      (e = p->alloc(&p->m, kMlpParams)) || (e = p->alloc(&p->v, kMlpParams)) ||
      (e = p->alloc(&p->loss, 1)) || (e = p->alloc(&p->tiles, 1))) {
    delete p;
    return e;
  }
  // He-uniform weights (limit sqrt(6 / fan_in)), zero biases
  std::vector<float> h(kMlpParams, 0.0f);
  std::mt19937_64 rng(seed);
  auto fill = [&](int off, int fan_in, int count) {
    std::uniform_real_distribution<float> u(-std::sqrt(6.0f / fan_in), std::sqrt(6.0f / fan_in));
    for (int i = 0; i < count; ++i) h[off + i] = u(rng);
  };
  fill(0, kMlpIn, kMlpIn * kMlpHidden);
  const int oW2 = kMlpIn * kMlpHidden + kMlpHidden;
  fill(oW2, kMlpHidden, kMlpHidden * kMlpHidden);
  const int oW3 = oW2 + kMlpHidden * kMlpHidden + kMlpHidden;
  fill(oW3, kMlpHidden, kMlpHidden);
  if (lpa_predictor_set_params(p, h.data()) != LPA_OK) {
    delete p;
    return LPA_ERR_HIP;
  }
  *out = p;
  return LPA_OK;
}

void lpa_predictor_destroy(lpa_predictor p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  delete p;
}

lpa_status lpa_predictor_set_params(lpa_predictor p, const float* params) {
  if (!p || !params) return fail(LPA_ERR_INVALID, "NULL argument");
  LPA_HIP(hipMemcpyAsync(p->p, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                         p->stream));
  std::vector<float> z(kMlpParams, 0.0f);
  LPA_HIP(hipMemcpyAsync(p->m, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                         p->stream));
  LPA_HIP(hipMemcpyAsync(p->v, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                         p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  p->steps = 0;
  p->tiles_ok = false;
  return LPA_OK;
}

lpa_status lpa_predictor_get_params(lpa_predictor p, float* params) {
  if (!p || !params) return fail(LPA_ERR_INVALID, "NULL argument");
  LPA_HIP(hipMemcpyAsync(params, p->p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost,
                         p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  return LPA_OK;
}

// Checkpoint blob: a 32-byte header (magic "LPAPRED1", format version 1,
// the layer sizes 12, 64, 64, 1, the parameter count and the Adam step
// count), then the fp32 master parameters and Adam's first and second
// moments, 5,057 values each, little-endian as in memory.
namespace {
struct BlobHeader {
  char magic[8];
  uint32_t version;
  uint16_t n_in, n_h1, n_h2, n_out;
  uint32_t n_params;
  int32_t steps;
  uint32_t reserved;
};
static_assert(sizeof(BlobHeader) == 32, "blob header layout");
constexpr int64_t kBlobBytes = (int64_t)sizeof(BlobHeader) + 3 * (int64_t)kMlpParams * 4;
}  // namespace

lpa_status lpa_predictor_save(lpa_predictor p, void* blob, int64_t cap, int64_t* size) {
  if (!p || !size) return fail(LPA_ERR_INVALID, "NULL argument");
  *size = kBlobBytes;
  if (!blob) return LPA_OK;
  if (cap < kBlobBytes)
    return fail(LPA_ERR_INVALID, "blob capacity below " + std::to_string(kBlobBytes) + " bytes");
  BlobHeader h{};
  std::memcpy(h.magic, "LPAPRED1", 8);
  h.version = 1;
  h.n_in = (uint16_t)kMlpIn;
  h.n_h1 = (uint16_t)kMlpHidden;
  h.n_h2 = (uint16_t)kMlpHidden;
  h.n_out = 1;
  h.n_params = (uint32_t)kMlpParams;
  h.steps = p->steps;
  uint8_t* out = static_cast<uint8_t*>(blob);
  std::memcpy(out, &h, sizeof(h));
  float* body = reinterpret_cast<float*>(out + sizeof(h));
  LPA_HIP(hipMemcpyAsync(body, p->p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost,
                         p->stream));
  LPA_HIP(hipMemcpyAsync(body + kMlpParams, p->m, sizeof(float) * kMlpParams,
                         hipMemcpyDeviceToHost, p->stream));
  LPA_HIP(hipMemcpyAsync(body + 2 * kMlpParams, p->v, sizeof(float) * kMlpParams,
                         hipMemcpyDeviceToHost, p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  return LPA_OK;
}

lpa_status lpa_predictor_load(lpa_predictor p, const void* blob, int64_t size) {
  if (!p || !blob) return fail(LPA_ERR_INVALID, "NULL argument");
  if (size < (int64_t)sizeof(BlobHeader)) return fail(LPA_ERR_INVALID, "blob too short");
  BlobHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (std::memcmp(h.magic, "LPAPRED1", 8) != 0) return fail(LPA_ERR_INVALID, "not a predictor blob");
  if (h.version != 1) return fail(LPA_ERR_INVALID, "unknown predictor blob version");
  if (h.n_in != kMlpIn || h.n_h1 != kMlpHidden || h.n_h2 != kMlpHidden || h.n_out != 1 ||
      h.n_params != (uint32_t)kMlpParams)
    return fail(LPA_ERR_INVALID, "predictor blob of another network shape");
  if (size < kBlobBytes) return fail(LPA_ERR_INVALID, "blob truncated");
  if (h.steps < 0) return fail(LPA_ERR_INVALID, "negative Adam step count in the blob");
  const float* body =
      reinterpret_cast<const float*>(static_cast<const uint8_t*>(blob) + sizeof(h));
  for (int64_t i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(body[i])) return fail(LPA_ERR_INVALID, "non-finite parameter in the blob");
  LPA_HIP(hipMemcpyAsync(p->p, body, sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                         p->stream));
  LPA_HIP(hipMemcpyAsync(p->m, body + kMlpParams, sizeof(float) * kMlpParams,
                         hipMemcpyHostToDevice, p->stream));
  LPA_HIP(hipMemcpyAsync(p->v, body + 2 * kMlpParams, sizeof(float) * kMlpParams,
                         hipMemcpyHostToDevice, p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  p->steps = h.steps;
  p->tiles_ok = false;
  return LPA_OK;
}

lpa_status lpa_predictor_gradient(lpa_predictor p, const float* X, const float* y, int64_t n,
                                  float pos_weight, float* grad, double* loss) {
  if (!p || n < 0 || (n > 0 && (!X || !y))) return fail(LPA_ERR_INVALID, "bad argument");
  Staging st;
  float *dX = nullptr, *dy = nullptr;
  if (lpa_status e = to_device(X, (size_t)n * kMlpIn, &dX, &st.bufs, p->stream)) return e;
  if (lpa_status e = to_device(y, (size_t)n, &dy, &st.bufs, p->stream)) return e;
  std::vector<float> z(kMlpParams, 0.0f);
  LPA_HIP(hipMemcpyAsync(p->g, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                         p->stream));
  const double zero = 0.0;
  LPA_HIP(hipMemcpyAsync(p->loss, &zero, sizeof(double), hipMemcpyHostToDevice, p->stream));
  LPA_HIP(launch_mlp_grad(p->p, dX, dy, n, pos_weight, p->g, p->loss, p->stream));
  if (grad)
    LPA_HIP(hipMemcpyAsync(grad, p->g, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost,
                           p->stream));
  double l = 0.0;
  LPA_HIP(hipMemcpyAsync(&l, p->loss, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  if (loss) *loss = n > 0 ? l / (double)n : 0.0;
  return LPA_OK;
}

lpa_status lpa_predictor_adam(lpa_predictor p, const float* grad, float lr) {
  if (!p) return fail(LPA_ERR_INVALID, "predictor is NULL");
  if (grad)
    LPA_HIP(hipMemcpyAsync(p->g, grad, sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                           p->stream));
  p->steps += 1;
  LPA_HIP(launch_adam(p->p, p->g, p->m, p->v, p->steps, lr, 0.9, 0.999, 1e-8f, p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  p->tiles_ok = false;
  return LPA_OK;
}

lpa_status lpa_predictor_train(lpa_predictor p, const float* X, const float* y, int64_t n,
                               const lpa_train_options* opt, float* final_loss) {
  if (!p || !opt || n <= 0 || !X || !y) return fail(LPA_ERR_INVALID, "bad argument");
  if (opt->epochs < 0 || opt->batch <= 0 || !(opt->lr > 0.0f))
    return fail(LPA_ERR_INVALID, "epochs >= 0, batch > 0 and lr > 0 required");
  Staging st;
  float *dX = nullptr, *dy = nullptr;
  if (lpa_status e = to_device(X, (size_t)n * kMlpIn, &dX, &st.bufs, p->stream)) return e;
  if (lpa_status e = to_device(y, (size_t)n, &dy, &st.bufs, p->stream)) return e;
  // shuffled copies of the samples, one permutation per epoch (host RNG)
  float *sX = nullptr, *sy = nullptr;
  int32_t* didx = nullptr;
  {
    void* q;
    if (hipMalloc(&q, sizeof(float) * (size_t)n * kMlpIn) != hipSuccess)
      return fail(LPA_ERR_OOM, "hipMalloc failed");
    st.bufs.push_back(q);
    sX = static_cast<float*>(q);
    if (hipMalloc(&q, sizeof(float) * (size_t)n) != hipSuccess)
      return fail(LPA_ERR_OOM, "hipMalloc failed");
    st.bufs.push_back(q);
    sy = static_cast<float*>(q);
    if (hipMalloc(&q, sizeof(int32_t) * (size_t)n) != hipSuccess)
      return fail(LPA_ERR_OOM, "hipMalloc failed");
    st.bufs.push_back(q);
    didx = static_cast<int32_t*>(q);
  }
  std::vector<int32_t> perm((size_t)n);
  std::iota(perm.begin(), perm.end(), 0);
  std::mt19937_64 rng(opt->seed);
  std::vector<float> z(kMlpParams, 0.0f);
  double last = 0.0;
  for (int32_t ep = 0; ep < opt->epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    LPA_HIP(hipMemcpyAsync(didx, perm.data(), sizeof(int32_t) * (size_t)n,
                           hipMemcpyHostToDevice, p->stream));
    LPA_HIP(launch_mlp_gather(dX, dy, didx, n, sX, sy, p->stream));
    double ep_loss = 0.0;
    for (int64_t b0 = 0; b0 < n; b0 += opt->batch) {
      const int64_t nb = std::min<int64_t>(opt->batch, n - b0);
      LPA_HIP(hipMemcpyAsync(p->g, z.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                             p->stream));
      const double zero = 0.0;
      LPA_HIP(hipMemcpyAsync(p->loss, &zero, sizeof(double), hipMemcpyHostToDevice, p->stream));
      LPA_HIP(launch_mlp_grad(p->p, sX + b0 * kMlpIn, sy + b0, nb, opt->pos_weight, p->g,
                              p->loss, p->stream));
      p->steps += 1;
      LPA_HIP(launch_adam(p->p, p->g, p->m, p->v, p->steps, opt->lr, 0.9, 0.999, 1e-8f,
                          p->stream));
      double l = 0.0;
      LPA_HIP(hipMemcpyAsync(&l, p->loss, sizeof(double), hipMemcpyDeviceToHost, p->stream));
      LPA_HIP(hipStreamSynchronize(p->stream));
      ep_loss += l;
    }
    last = ep_loss / (double)n;
  }
  p->tiles_ok = false;
  if (final_loss) *final_loss = (float)last;
  return LPA_OK;
}

lpa_status lpa_predictor_predict(lpa_predictor p, const float* X, int64_t n, float* prob) {
  if (!p || n < 0 || (n > 0 && (!X || !prob))) return fail(LPA_ERR_INVALID, "bad argument");
  if (n == 0) return LPA_OK;
  if (lpa_status e = pack(p)) return e;
  Staging st;
  float* dX = nullptr;
  if (lpa_status e = to_device(X, (size_t)n * kMlpIn, &dX, &st.bufs, p->stream)) return e;
  float* dout = prob;
  const bool host_out = !is_device_ptr(prob);
  if (host_out) {
    void* q;
    if (hipMalloc(&q, sizeof(float) * (size_t)n) != hipSuccess)
      return fail(LPA_ERR_OOM, "hipMalloc failed");
    st.bufs.push_back(q);
    dout = static_cast<float*>(q);
  }
  LPA_HIP(launch_mlp_infer(p->tiles, dX, n, dout, p->stream));
  if (host_out)
    LPA_HIP(hipMemcpyAsync(prob, dout, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost,
                           p->stream));
  LPA_HIP(hipStreamSynchronize(p->stream));
  return LPA_OK;
}

}  // extern "C"
