// Fused register-resident kernel: not written yet.
#include "common.hpp"

namespace stp {
template <>
hipError_t launch_fused_degree<STP_DEGREE>(const PredictArgs&, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace stp
