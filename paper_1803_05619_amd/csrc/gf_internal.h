// Internal interface between the C-ABI layer (gf_api.cpp) and the HIP
// kernels (gf_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gf.h"

namespace gf {

// Geometry and launch shapes derived from a gf_desc_t on the host.
struct Plan {
  int n, c, h, w, H, W, r, mean_ab, dtype;
  int S;        // integer upsampling factor (H = S h, W = S w)
  int xcd;      // XCD-aware workgroup order for the high-res kernels
  int VEC;      // high-res elements per thread-load (16 bytes, or 1)
  int planes;   // n * c
  // low-res coefficient kernel: one wave per strip of 64 lanes (columns)
  // x coTR output rows; co_nx strips, co_ny row segments
  int coTR, co_nx, co_ny;
  size_t coLDS;
  // high-res apply: rows per thread
  int RB, nrb, nxv;
  // backward high-res blocks (one wave each): bh low-res rows x tw low-res
  // columns (64 * VEC high-res columns)
  int bh, tw, nby, nbx;
  size_t ublk_floats;  // floats per block (2 * (bh + 2) * (tw + 2))
  // backward low-res kernel: same walker shape
  int loTR, lo_nx, lo_ny;
  size_t loLDS;
  // guidance map: mode (gf_guide_mode_t), input channels, hidden channels
  // (padded to KP = 16 for the transform)
  int gmode, c_in, hidden, KP;
  float bn_eps, slope;
  const float* gparams;
  float* gstats;
  int use_stats;
  // guide reductions: chunks per image of the moments / guide-backward grids
  int g_chunks_lo, g_chunks_hi;
  // workspace layout (bytes)
  size_t off_abar, off_bbar, off_u, off_eps, ws_fwd, ws_bwd;
  // guided path: G_l, G_h (float planes), dG_l, dG_h, moments partials,
  // folded transform parameters (2 calls), accumulator partials/totals
  size_t off_gl, off_gh, off_dgl, off_dgh, off_mom, off_fold, off_accp, off_acct;
};

// Per-call folded transform parameters (floats), see gf_guide.h.
constexpr int kFoldFloats = 1024;
constexpr int kMomFloats = 12;    // 3 shifted sums + 6 second moments (+ pad)
constexpr int kAccFloats = 256;   // 3 + 7 KP accumulators (KP = 16) + pad

// Rows of the low-res walkers' LDS ring buffers for radius R: a block writes
// `block` rows before reading 2R + 1, so at least 2R + block rows; rounded
// up to a power of two (index by mask) when the LDS footprint stays within
// 64 KB, i.e. up to `pow2_max` rows.
constexpr int walker_ring_rows(int R, int block, int pow2_max) {
  int need = 2 * R + block, p2 = 1;
  while (p2 < need) p2 <<= 1;
  return p2 <= pow2_max ? p2 : need;
}
constexpr int kWalkBlock = 4;        // rows per block of the low-res walkers
constexpr int kCoefRingPow2Max = 32;  // coef: 64 * (16 KR + 24 * 4) bytes
constexpr int kBwdLoRingPow2Max = 16;  // bwd_lo: 64 * (32 KR + 40 * 4) bytes

// Returns GF_OK and fills `p`, or an error code with a message in `why`.
int make_plan(const gf_desc_t* d, const gf_guide_t* g, Plan* p, const char** why);

struct FwdArgs {
  const void *I_lo, *p_lo, *I_hi;
  const float* eps;
  int eps_count;
  void* q;
  char* ws;
};

struct BwdArgs {
  const void *I_lo, *p_lo, *I_hi, *dq;
  const float* eps;
  int eps_count;
  float *dI_lo, *dp_lo, *deps, *dparams;
  void* dI_hi;
  char* ws;
};

// One pair of launchers per image I/O type (gf_f32.hip, gf_f16.hip,
// gf_bf16.hip); gf_api.cpp picks by desc->io_dtype.
hipError_t launch_forward_f32(const Plan& p, const FwdArgs& a, hipStream_t s);
// Guided path (grey or transform guide), same per-type split.
hipError_t launch_forward_guided_f32(const Plan& p, const FwdArgs& a, hipStream_t s);
hipError_t launch_backward_guided_f32(const Plan& p, const BwdArgs& a, hipStream_t s);
hipError_t launch_forward_guided_f16(const Plan& p, const FwdArgs& a, hipStream_t s);
hipError_t launch_backward_guided_f16(const Plan& p, const BwdArgs& a, hipStream_t s);
hipError_t launch_forward_guided_bf16(const Plan& p, const FwdArgs& a, hipStream_t s);
hipError_t launch_backward_guided_bf16(const Plan& p, const BwdArgs& a, hipStream_t s);
hipError_t launch_backward_f32(const Plan& p, const BwdArgs& a, hipStream_t s);
hipError_t launch_forward_f16(const Plan& p, const FwdArgs& a, hipStream_t s);
hipError_t launch_backward_f16(const Plan& p, const BwdArgs& a, hipStream_t s);
hipError_t launch_forward_bf16(const Plan& p, const FwdArgs& a, hipStream_t s);
hipError_t launch_backward_bf16(const Plan& p, const BwdArgs& a, hipStream_t s);

// Profiling hooks (gf_api.cpp): wrap one kernel launch.
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);

}  // namespace gf
