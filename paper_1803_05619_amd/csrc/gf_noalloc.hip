// gf_forward_backward_static: gf_forward_backward with the library's own
// scratch memory instead of a caller workspace, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The scratch memory is a file-scope device array of GF_STATIC_SCRATCH_BYTES
// that every GPU the library runs on holds until the process ends.  In host
// code the array's name is only a host-side stand-in for the symbol, so its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current, on the first call there) and only that address is
// passed to the kernels.  Every call on one GPU shares that GPU's array:
// calls that overlap on one GPU (on different streams, or from several host
// threads without ordering) race on it.  The kernels write every scratch
// word before they read it, so the contents a previous call left behind do
// not matter and nothing has to be cleared.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "gf_internal.h"

namespace {

constexpr size_t kScratchBytes = GF_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up on
// the first call on that device; nullptr (with the error detail set) if the
// lookup fails.
void* scratch_ptr(int32_t* status) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *status = gf::set_error(GF_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *status = gf::set_error(GF_ERR_UNSUPPORTED, "device index beyond the library's table");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *status = gf::set_error(GF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                              hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int32_t gf_forward_backward_static(const gf_desc_t* desc, const gf_guide_t* guide,
                                              const void* I_lo, const void* p_lo,
                                              const void* I_hi, const float* eps,
                                              int32_t eps_count, const void* dq_hi, void* q_hi,
                                              float* dI_lo, float* dp_lo, void* dI_hi,
                                              float* deps, float* dparams, void* stream) {
  // host-side size check first: an invalid or oversized problem touches no
  // device
  const size_t need = gf_workspace_size(desc, guide, 2);
  if (need == 0)
    return gf_forward_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, q_hi,
                               dI_lo, dp_lo, dI_hi, deps, dparams, nullptr, 0, stream);
  if (need > kScratchBytes)
    return gf::set_error(GF_ERR_WORKSPACE,
                         "problem needs " + std::to_string(need) +
                             " bytes of scratch memory; the static scratch holds " +
                             std::to_string(kScratchBytes) +
                             " (use gf_forward_backward with a caller workspace)");
  int32_t st = GF_OK;
  void* ws = scratch_ptr(&st);
  if (!ws) return st;
  return gf_forward_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, q_hi, dI_lo,
                             dp_lo, dI_hi, deps, dparams, ws, kScratchBytes, stream);
}
