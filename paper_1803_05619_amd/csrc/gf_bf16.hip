// Launchers of the guided filtering kernels for bf16 image I/O.
#include "gf_guide.h"

namespace gf {

hipError_t launch_forward_bf16(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_t<bf16>(p, a, s);
}

hipError_t launch_backward_bf16(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_t<bf16>(p, a, s);
}

hipError_t launch_forward_guided_bf16(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_guided_t<bf16>(p, a, s);
}

hipError_t launch_backward_guided_bf16(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_guided_t<bf16>(p, a, s);
}

hipError_t launch_batched_bf16(const BatchLaunch& b, int mode, char* ws, hipStream_t s) {
  return batched_t<bf16>(b, mode, ws, s);
}

}  // namespace gf
