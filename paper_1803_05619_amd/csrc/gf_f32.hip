// Launchers of the guided filtering kernels for float image I/O.
#include "gf_kernels.h"

namespace gf {

hipError_t launch_forward_f32(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_t<float>(p, a, s);
}

hipError_t launch_backward_f32(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_t<float>(p, a, s);
}

}  // namespace gf
