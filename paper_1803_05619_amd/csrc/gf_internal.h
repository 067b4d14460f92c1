// Internal interface between the C-ABI layer (gf_api.cpp) and the HIP
// kernels (gf_kernels.h, gf_guide.h, instantiated per I/O type in
// gf_f32.hip, gf_f16.hip, gf_bf16.hip) and the batched planner
// (gf_batch.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gf.h"

namespace gf {

// Geometry and launch shapes derived from a gf_desc_t on the host.
struct Plan {
  int n, c, h, w, H, W, r, mean_ab, dtype;
  int ac;       // corner-aligned bilinear (align_corners)
  int S;        // integer upsampling factor (H = S h, W = S w); 0 for any other ratio
  int gen;      // 1: any size ratio (the general high-res kernels), S = 0
  int xcd;      // XCD-aware workgroup order for the high-res kernels (0: off; see xcd_order)
  int lo_xcd;   // the same for the single-problem low-res walkers
  int wide_co, wide_lo;  // coefficients / low-res backward through the wide (FP64) walkers
  int VEC;      // high-res elements per thread-load (16 bytes, or 1)
  int planes;   // n * c
  // low-res coefficient kernel: one wave per strip of 64 lanes (columns)
  // x coTR output rows; co_nx strips, co_ny row segments
  int coTR, co_nx, co_ny;
  size_t coLDS;
  // high-res apply: rows per thread
  int RB, nrb, nxv;
  // backward high-res blocks: a workgroup of hw waves (1 .. kHiWaves), each
  // wave bh low-res rows (stacked) x tw low-res columns (64 * VEC high-res
  // columns); the workgroup writes one merged partial block of ubh = hw * bh
  // rows (nby x nbx blocks per plane)
  int bh, hw, ubh, tw, nby, nbx;
  size_t ublk_floats;  // floats per partial block (2 * (ubh + 2) * (tw + 2))
  size_t hiLDS;        // the workgroup's LDS for merging its waves' partial rows
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
  // any size ratio: the vertical adjoint's low-res rows x high-res columns
  // (dA_bar and db_bar parts)
  size_t off_v;
  // wide low-res passes: their plane (wide_x_floats floats per pixel)
  size_t off_x;
  // guided path: G_l, G_h (float planes), dG_l, dG_h, moments partials,
  // folded transform parameters (2 calls), accumulator partials/totals
  size_t off_gl, off_gh, off_dgl, off_dgh, off_mom, off_fold, off_accp, off_acct;
  // transform: leaky-ReLU branch of every hidden channel per pixel (bit k
  // of a 16-bit word), written by the map and read by the backward kernels
  size_t off_mlo, off_mhi;
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
// Waves per workgroup of the high-res backward (at most): vertically
// stacked row bands whose overlapping partial rows are summed in LDS, so one
// partial block of hw * bh + 2 rows is written per workgroup (rather than
// bh + 2 rows per wave), and the bands' shared low-res coefficient rows are
// read by one CU.
constexpr int kHiWaves = 4;
// Stacking pays for its barrier where the partial planes and coefficient
// halos are a large share of the traffic: FP32 gradients at S >= 4
// (measured slower for the half types and for S <= 2 on MI355X).  The same
// rule, on the gradient element type, selects the kernel variant.
constexpr bool hi_merge(bool f32_grad, int S) { return f32_grad && S >= 4; }
// LDS of that merge: two buffers (waves of even / odd index, whose row
// ranges do not overlap within a buffer) x two quantities x (ubh + 2) rows
// x (tw + 2) columns.
constexpr size_t bwd_hi_lds_bytes(int ubh, int tw) {
  return (size_t)2 * 2 * (ubh + 2) * (tw + 2) * sizeof(float);
}
constexpr size_t kHiLdsMax = 65536;
constexpr int kCoefRingPow2Max = 32;  // coef: 64 * (16 KR + 24 * 4) bytes
// Wide low-res walkers (gf_wide.h), from radius wide_bwd_min_r(): 256
// threads (input columns) per strip, blocks of kWideB rows, LDS rows of
// 256 + 256 / 4 padded columns holding the block's FP64 column sums (6
// quantities in the first pass, 48 bytes per padded column and row; 4 in the
// second).  The environment variable GF_WIDE_BWD_R overrides the default
// radius (at least kWideMinR), for measurements; a precise descriptor takes
// them at every radius.
constexpr int kWideMinR = 1, kWideBwdR = 5, kWideCoefR = 5;
constexpr int kWideB = 4;
constexpr int kWideBThreads = 256;
constexpr size_t wide_row(int nt) { return (size_t)nt + nt / 4; }
constexpr size_t bwd_wide_lds_bytes() { return (size_t)kWideB * wide_row(kWideBThreads) * 48; }
// LDS of one wide pass holding nq FP64 quantities per padded column and row
// (coefficients: 4 in the statistics pass, 2 in the mean; backward: 6, 4).
constexpr size_t wide_lds_bytes(int nq) { return (size_t)kWideB * wide_row(kWideBThreads) * 8 * nq; }
constexpr size_t kLdsPerCU = 160 * 1024;  // MI355X
int wide_bwd_min_r();
inline bool wide_bwd(int r) { return r >= wide_bwd_min_r(); }

// Floats per low-res pixel of the wide passes' plane: the backward's X
// quantities in FP64 for FP32 I/O (8), else in FP32 (4, which also holds the
// coefficients' (A, b)).
inline size_t wide_x_floats(const Plan& p) {
  return p.wide_lo && p.dtype == GF_F32 ? 8 : 4;
}

// The coefficients the same way (two passes: (A, b) per pixel, then their
// window mean); GF_WIDE_COEF_R overrides the radius.
int wide_coef_min_r();
inline bool wide_coef(int r) { return r >= wide_coef_min_r(); }
constexpr int kBwdLoRingPow2Max = 16;  // bwd_lo: 64 * (32 KR + 40 * 4) bytes

// Radii up to 8 keep each lane's vertical windows (2R + block rows) in
// registers instead of LDS rings: the LDS footprint per wave then shrinks to
// the row buffers of the horizontal windows, which lifts occupancy.  The
// coefficient walker holds 2 x 2 floats per window row (at r = 8: 188
// VGPRs, two waves per SIMD, against four waves per CU with 39 KB of
// rings), the backward walker 2 x 4 (at r = 8 one wave per SIMD, against
// three waves per CU with 51 KB of rings).
constexpr bool coef_reg_window(int R) { return 4 * (2 * R + kWalkBlock) <= 80; }
constexpr bool bwd_lo_reg_window(int R) { return 8 * (2 * R + kWalkBlock) <= 160; }
// Radii whose horizontal windows are formed by whole-wave DPP lane shifts
// (R shifts each way) rather than through LDS row buffers: with vertical
// windows in registers as well, such walkers use no LDS at all.  Measured
// on the uneven batch's r = 4 class: the backward 1,054 -> 966 us with DPP,
// the coefficients 373 -> 468 us (their horizontal work is mostly the
// statistics' deviations, which need every neighbour value), so the
// coefficient walker keeps LDS rows above r = 2.
constexpr bool coef_lane_dpp(int R) { return R <= 2; }
constexpr bool bwd_lo_lane_dpp(int R) { return R <= 4; }
constexpr size_t coef_lds_bytes(int R) {
  return 64 * ((coef_lane_dpp(R) ? 0 : 24 * kWalkBlock) +
               (coef_reg_window(R) ? 0 : 16 * walker_ring_rows(R, kWalkBlock, kCoefRingPow2Max)));
}
constexpr size_t bwd_lo_lds_bytes(int R) {
  return 64 * ((bwd_lo_lane_dpp(R) ? 0 : 40 * kWalkBlock) +
               (bwd_lo_reg_window(R) ? 0
                                     : 32 * walker_ring_rows(R, kWalkBlock, kBwdLoRingPow2Max)));
}

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
  void* q;  // non-null: forward and backward in one pass (q written too)
};

// Kernel arguments of the four filter kernels (one problem each).
struct CoefArgs {
  const void* I_lo;
  const void* p_lo;
  const float* eps;
  int eps_count, c, h, w, TR;
  float* abar;  // [planes, h, w]
  float* bbar;  // [planes, h, w] or null
  int xcd;      // XCD-aware strip order (see xcd_order)
  float* X;     // wide coefficient passes with the window mean: the (A, b) plane
};

struct ApplyArgs {
  const void* I_hi;
  void* q;
  const float* abar;
  const float* bbar;
  int h, w, H, W, RB, nrb, nxv;
  long long total;
  int xcd;  // XCD-aware workgroup order (0: off; see xcd_order)
};

struct BwdHiArgs {
  const void* I_hi;
  const void* dq;
  void* dI_hi;  // may be null
  const float* abar;
  float* U;     // per-block partial planes
  int h, w, H, W, bh, tw, nby, nbx;  // bh: rows per wave; nby: partial blocks (hw * bh rows)
  int hw;                            // waves per workgroup
  int xcd;  // XCD-aware workgroup order (0: off; see xcd_order)
  // forward in the same pass (fused kernel only): q = A_h G_h + b_h
  const float* bbar;
  void* q;
};

// The high-res kernels of problems of any size ratio (one problem each).
struct GenArgs {
  const void* G_hi;
  const void* dq;
  void* dI_hi;        // may be null
  void* q;            // forward output (apply; the fused backward pass)
  const float* abar;
  const float* bbar;
  float* V;           // [planes][2][h][W] vertical adjoint
  float* U;           // [planes][2][h + 2][w + 2] partial planes, one block
  int planes, h, w, H, W, RB, nrb, nxv;
  long long total;    // threads of the launch
};

// Area downsampling (the DGF framework's I_h -> I_l): one workgroup per
// (low-res column chunk of jc pixels, low-res row, plane); span = the most
// high-res columns a chunk covers (its LDS floats).
struct DownArgs {
  const void* x;
  void* y;
  int planes, H, W, h, w, jc, span;
};
constexpr int kDownMaxSpan = 8192;

struct BwdLoArgs {
  const void* I_lo;
  const void* p_lo;
  const float* eps;
  int eps_count, c;
  const float* U;
  int bh, tw, nby, nbx;
  int h, w, TR;
  float* dI_lo;     // may be null
  float* dp_lo;     // may be null
  float* eps_part;  // [planes][pny][pnx]: one partial per strip segment
  int pnx, pny;     // strips and row segments per plane
  float* X;         // wide walkers: [planes][h][w][4] adjoint quantities
  int xcd;          // XCD-aware strip order (see xcd_order)
};

// ------------------------------------------------------------ convolutional layer
// The convolutional guided filtering layer (Sec. III-E): 3x3 depthwise
// dilated convolutions (normalised by their response to ones) in place of
// the box filter, a bias-free pointwise block 2c -> K -> K -> c on (cov,
// var) in place of A = cov / (var + eps).  Parameters (device, float):
// D [c][9] | W1 [K][2c] | W2 [K][K] | W3 [c][K].
constexpr int kConvMaxC = 4, kConvMaxK = 16;
constexpr int kConvTile = 256;   // pixels per workgroup tile of the parameter-gradient sums
constexpr int kConvBlocks = 1024;  // most workgroups of those sums
// most workgroups per plane of the window-mean adjoint (each thread walks
// its plane's pixels with a stride of 256 x this; enough workgroups that the
// gathers' latency is hidden)
constexpr int kConvAbGrid = 512;
constexpr int conv_param_count(int c, int K) { return 9 * c + 2 * c * K + K * K + c * K; }

struct ConvPlan {
  Plan p;        // the high-res kernels' plan (and the identity workspace layout)
  int r, K;      // dilation, hidden width
  float slope;
  const float* params;
  int nparam;
  int blk_grid;  // workgroups of the parameter-gradient sums over pixels
  int ab_grid;   // workgroups per plane of the window-mean adjoint
  // workspace (bytes): per-pixel statistics, coefficients and adjoints, all
  // low-res float planes [n][c][h][w]; partial parameter gradients
  size_t off_mI, off_mP, off_cov, off_var, off_A, off_B, off_dAb, off_dBb;
  size_t off_gmI, off_gmP, off_gcov, off_gvar, off_dA, off_dB, off_part, off_partab;
  size_t ws_fwd, ws_bwd;
};

struct ConvArgs {
  const void* I_lo;
  const void* p_lo;
  const float* params;
  int n, c, h, w, r, K, nparam, mean_ab;
  float slope;
  float *mI, *mP, *cov, *var, *A, *B, *abar, *bbar;
  float *dAb, *dBb, *dA, *dB, *gmI, *gmP, *gcov, *gvar;
  float *dI_lo, *dp_lo, *dparams;
  float *part, *partab;
  int blk_grid, ab_grid;
  // the high-res backward's partial planes
  const float* U;
  int bh, tw, nby, nbx;
};

hipError_t launch_conv_forward_f32(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                   void* q, char* ws, hipStream_t s);
hipError_t launch_conv_forward_f16(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                   void* q, char* ws, hipStream_t s);
hipError_t launch_conv_forward_bf16(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                    void* q, char* ws, hipStream_t s);
hipError_t launch_conv_backward_f32(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                    const void* dq, void* dI_hi, char* ws, hipStream_t s);
hipError_t launch_conv_backward_f16(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                    const void* dq, void* dI_hi, char* ws, hipStream_t s);
hipError_t launch_conv_backward_bf16(const ConvPlan& cp, const ConvArgs& a, const void* I_hi,
                                     const void* dq, void* dI_hi, char* ws, hipStream_t s);

// ------------------------------------------------------------ batched launches
// One launch per phase and launch class covers the tiles of many problems:
// the items of a class are laid out in device memory as
//   base[count] (first tile of each item, ascending, base[0] = 0)
//   MultiItem<Args>[count]
// and workgroup t (grid-stride when the grid is smaller than the tile count)
// finds its item by a wave ballot over base[].  Workspace pointers inside
// the item arguments are stored as (offset + 1) and rebased on the device
// against the workspace passed at launch (0 stays null).
template <typename Args>
struct MultiItem {
  Args a;
  int nx, ny;  // tiles along x and y; the rest of the tile index is the plane
  long long base;
};

struct EpsItem {
  const float* part;  // workspace-relative (offset + 1)
  long long count;
  float* deps;
};

struct MultiLaunch {
  const long long* base;
  const void* items;
  int count;
  long long total;  // tiles
  char* ws;         // set per launch
  int grid;         // workgroups launched (<= total)
};

enum { kClassCoef = 0, kClassApply = 1, kClassBwdHi = 2, kClassBwdLo = 3 };

struct BatchClass {
  int kind;
  int S, VEC, AC; // high-res classes (AC: corner alignment)
  int R, MAB;     // low-res classes
  int wide;       // low-res classes: the wide (FP64) walkers
  size_t lds;     // dynamic LDS bytes
  int hw;         // high-res backward: waves per workgroup
  MultiLaunch m;
};

struct BatchLaunch {
  std::vector<BatchClass> coef, apply, bwd_hi, bwd_lo;
  const EpsItem* eps_items;  // device
  int eps_count;             // items with a deps output
};

hipError_t launch_batched_f32(const BatchLaunch& b, int mode, char* ws, hipStream_t s);
hipError_t launch_batched_f16(const BatchLaunch& b, int mode, char* ws, hipStream_t s);
hipError_t launch_batched_bf16(const BatchLaunch& b, int mode, char* ws, hipStream_t s);

// ------------------------------------------------------------ tile-shape table
// Launch shapes per (io dtype, factor S, radius, guide mode, mean_ab),
// filled by the autotuner (or imported); make_plan uses an entry when one
// exists, else its defaults.
struct TuneKey {
  int dtype, S, r, gmode, mean_ab;
};
struct TuneVal {
  int coTR, loTR, RB, bh;
};
bool tune_lookup(const TuneKey& k, TuneVal* v);
void tune_store(const TuneKey& k, const TuneVal& v);

// Shared by the C-ABI files: sets the thread's error detail, returns code.
int set_error(int code, const std::string& why);
// Profiling hooks are muted while a stream is being captured into a graph.
void prof_mute(bool on);

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

hipError_t launch_downsample_f32(const DownArgs& a, hipStream_t s);
hipError_t launch_downsample_f16(const DownArgs& a, hipStream_t s);
hipError_t launch_downsample_bf16(const DownArgs& a, hipStream_t s);

// Profiling hooks (gf_api.cpp): wrap one kernel launch.
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);

}  // namespace gf
