// host_common.h -- error reporting shared by the host-side translation units.
#pragma once

#include <string>

#include "../../include/lpa.h"

namespace lpa {
// Record msg as the calling thread's last error and return s.
lpa_status fail(lpa_status s, const std::string& msg);
// True for device or managed memory of the current device.
bool is_device_ptr(const void* p);
// Packed bf16 operand tiles of a predictor's current parameters (packed on
// first use after a change and synchronised); NULL on error.
struct MlpTiles;
const MlpTiles* predictor_tiles(lpa_predictor p);
}  // namespace lpa

#define LPA_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::lpa::fail(LPA_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
