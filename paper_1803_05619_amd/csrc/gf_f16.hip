// Launchers of the guided filtering kernels for _Float16 image I/O.
#include "gf_guide.h"
#include "gf_resample.h"
#include "gf_conv.h"

namespace gf {

hipError_t launch_forward_f16(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_t<_Float16>(p, a, s);
}

hipError_t launch_backward_f16(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_t<_Float16>(p, a, s);
}

hipError_t launch_forward_guided_f16(const Plan& p, const FwdArgs& a, hipStream_t s) {
  return forward_guided_t<_Float16>(p, a, s);
}

hipError_t launch_backward_guided_f16(const Plan& p, const BwdArgs& a, hipStream_t s) {
  return backward_guided_t<_Float16>(p, a, s);
}

hipError_t launch_batched_f16(const BatchLaunch& b, int mode, char* ws, hipStream_t s) {
  return batched_t<_Float16>(b, mode, ws, s);
}

hipError_t launch_downsample_f16(const DownArgs& a, hipStream_t s) {
  return downsample_t<_Float16>(a, s);
}

hipError_t launch_conv_forward_f16(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                   void* q, char* ws, hipStream_t s) {
  return conv_forward_t<_Float16>(cp, a, I_hi, q, ws, s);
}

hipError_t launch_conv_backward_f16(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                    const void* dq, void* dI_hi, char* ws, hipStream_t s) {
  return conv_backward_t<_Float16>(cp, a, I_hi, dq, dI_hi, ws, s);
}

}  // namespace gf
