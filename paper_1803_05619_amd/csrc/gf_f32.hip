// Launchers of the guided filtering kernels for float image I/O.
#include "gf_guide.h"

namespace gf {

hipError_t launch_forward_f32(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_t<float>(p, a, s);
}

hipError_t launch_backward_f32(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_t<float>(p, a, s);
}

hipError_t launch_forward_guided_f32(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_guided_t<float>(p, a, s);
}

hipError_t launch_backward_guided_f32(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_guided_t<float>(p, a, s);
}

hipError_t launch_batched_f32(const BatchLaunch& b, int mode, char* ws, hipStream_t s) {
  return batched_t<float>(b, mode, ws, s);
}

}  // namespace gf
