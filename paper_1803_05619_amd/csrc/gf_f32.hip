// Launchers of the guided filtering kernels for float image I/O.
#include "gf_guide.h"
#include "gf_resample.h"
#include "gf_conv.h"

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

hipError_t launch_downsample_f32(const DownArgs& a, hipStream_t s) {
  return downsample_t<float>(a, s);
}

hipError_t launch_conv_forward_f32(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                   void* q, char* ws, hipStream_t s) {
  return conv_forward_t<float>(cp, a, I_hi, q, ws, s);
}

hipError_t launch_conv_backward_f32(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                    const void* dq, void* dI_hi, char* ws, hipStream_t s) {
  return conv_backward_t<float>(cp, a, I_hi, dq, dI_hi, ws, s);
}

}  // namespace gf
