// rowsort.hip -- sort every row of a handle's internal CSR by target id,
// smallest first (weights moved with their targets), once, when the handle
// is created.
//
// The sweeps read each entry's neighbour label at the target's address.  In
// the internal order (largest degree first) a row sorted by target walks the
// label array upwards: the entries that fall in the dense low-id region of a
// long row then share cache lines, both among the lanes of one load and
// between consecutive loads of a lane, where unsorted entries touch a new
// line almost every time.  (Largest ids first measured slower in the
// workgroup-table sweeps.)  Sums, maxima and every result are unchanged
// (addition order only matters for non-integer weights, where the LDS
// atomics already leave it free).
#include <hipcub/hipcub.hpp>

#include "lpa_internal.h"

namespace lpa {

template <typename OffT>
static hipError_t sort_rows_t(const OffT* off, int32_t* tgt, float* w, int64_t n, int64_t m,
                              hipStream_t s) {
  int32_t* kout = nullptr;
  float* vout = nullptr;
  void* tmp = nullptr;
  size_t bytes = 0;
  hipError_t e = hipMalloc(&kout, sizeof(int32_t) * (size_t)m);
  if (e == hipSuccess && w) e = hipMalloc(&vout, sizeof(float) * (size_t)m);
  if (e == hipSuccess) {
    e = w ? hipcub::DeviceSegmentedSort::SortPairs(nullptr, bytes, tgt, kout, w, vout, (int)m,
                                                   (int)n, off, off + 1, s)
          : hipcub::DeviceSegmentedSort::SortKeys(nullptr, bytes, tgt, kout, (int)m, (int)n, off,
                                                  off + 1, s);
  }
  if (e == hipSuccess) e = hipMalloc(&tmp, bytes > 0 ? bytes : 1);
  if (e == hipSuccess) {
    e = w ? hipcub::DeviceSegmentedSort::SortPairs(tmp, bytes, tgt, kout, w, vout, (int)m,
                                                   (int)n, off, off + 1, s)
          : hipcub::DeviceSegmentedSort::SortKeys(tmp, bytes, tgt, kout, (int)m, (int)n, off,
                                                  off + 1, s);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(tgt, kout, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && w)
    e = hipMemcpyAsync(w, vout, sizeof(float) * (size_t)m, hipMemcpyDeviceToDevice, s);
  const hipError_t sync = hipStreamSynchronize(s);
  if (e == hipSuccess) e = sync;
  if (kout) (void)hipFree(kout);
  if (vout) (void)hipFree(vout);
  if (tmp) (void)hipFree(tmp);
  return e;
}

hipError_t sort_rows(bool off64, const void* off, int32_t* tgt, float* w, int64_t n, int64_t m,
                     hipStream_t s) {
  if (n <= 0 || m <= 1) return hipSuccess;
  if (m > (int64_t)INT32_MAX || n > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  if (off64) return sort_rows_t(static_cast<const int64_t*>(off), tgt, w, n, m, s);
  return sort_rows_t(static_cast<const int32_t*>(off), tgt, w, n, m, s);
}

}  // namespace lpa
