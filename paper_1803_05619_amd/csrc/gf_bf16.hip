// Launchers of the guided filtering kernels for bf16 image I/O.
#include "gf_kernels.h"

namespace gf {

hipError_t launch_forward_bf16(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_t<bf16>(p, a, s);
}

hipError_t launch_backward_bf16(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_t<bf16>(p, a, s);
}

}  // namespace gf
