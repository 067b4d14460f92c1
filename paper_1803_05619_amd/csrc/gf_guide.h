// Guidance-map kernels of the guided filtering layer (paper Sec. III-D):
// the grey guide (channel mean) and the trainable transform
//   h = W1 x, y = lam h + mu BN(h), z = leaky_relu(y), G = W2 z + b2,
// with BN using the batch statistics of each call (I_lo and I_hi).
//
// The guided path maps both guides to float planes G_l, G_h in the
// workspace, runs the filter kernels on them, and maps the guide gradients
// dG_l, dG_h back through the transform:
//   moments_kernel       per-chunk shifted sums of x and x x^T (batch stats)
//   guide_fold_kernel    batch mean/covariance -> BN statistics of h = W1 x
//                        (mean W1 m, variance W1 C W1^T) -> per-call folded
//                        constants y_k = w1f_k . x + bf_k
//   guide_map_*_kernel   G = F(x) per pixel
//   guide_bwd_kernel     grey: dx directly; transform: per-chunk sums of
//                        dG, dG z^T, dy, dy x^T (the only pixel sums the
//                        parameter gradients need)
//   guide_acc_reduce_kernel, guide_grad_kernel
//                        fixed-order totals -> parameter gradients and the
//                        two batch means that the BN input gradient needs
//   guide_dx_kernel      transform: dx = W1^T dh per pixel
// Every reduction runs in a fixed order (deterministic).
#pragma once

#include "gf_kernels.h"

namespace gf {
namespace {

// Offsets (floats) of the per-call folded block; arrays over the hidden
// channels have stride kKP.
constexpr int kKP = 16;
constexpr int FO_W1F = 0;          // [kKP][3] lam-mu folded first layer
constexpr int FO_BF = 48;          // [kKP]    folded bias
constexpr int FO_W2 = 64;          // [3][kKP] second layer
constexpr int FO_B2 = 112;         // [3]
constexpr int FO_W1 = 116;         // [kKP][3] first layer as given
constexpr int FO_M = 164;          // [kKP] batch mean of h
constexpr int FO_RSTD = 180;       // [kKP] 1 / sqrt(batch var of h + bn_eps)
constexpr int FO_CDH = 196;        // [kKP] mu gamma rstd
constexpr int FO_SCAL = 212;       // lam, mu, slope, pixel count
constexpr int FO_MDY = 216;        // [kKP] batch mean of dy (after the gradient pass)
constexpr int FO_MDYHN = 232;      // [kKP] batch mean of dy * hn
constexpr int FO_MEAN = 248;       // [3] batch mean of x
constexpr int FO_COV = 252;        // [9] batch covariance of x
constexpr int FO_GAM = 264;        // [kKP] BN scale
constexpr int FO_BET = 280;        // [kKP] BN shift
static_assert(FO_BET + kKP <= kFoldFloats, "fold block");

// Accumulator layout of the transform's gradient pass.
constexpr int AC_DG = 0;                   // [3]       sum dG_c
constexpr int AC_DGZ = 3;                  // [3][kKP]  sum dG_c z_k
constexpr int AC_DY = 3 + 3 * kKP;         // [kKP]     sum dy_k
constexpr int AC_DYX = 3 + 4 * kKP;        // [kKP][3]  sum dy_k (x_i - mean x_i)
constexpr int AC_N = 3 + 7 * kKP;
static_assert(AC_N <= kAccFloats, "accumulators");

// ------------------------------------------------------------ batch moments

struct MomArgs {
  const void* x;   // [n][3][P]
  long long P;     // pixels per image plane
  float* part;     // [n * chunks][kMomFloats]
};

// Shifted sums (shift = the first pixel of the call, so that the second
// moments do not cancel) of x and x x^T over this chunk's pixels.
template <typename TX>
__global__ __launch_bounds__(256) void moments_kernel(MomArgs a) {
  __shared__ float red[9][256];
  const TX* X = reinterpret_cast<const TX*>(a.x);
  const int b = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const float s0 = to_f(X[0]), s1 = to_f(X[a.P]), s2 = to_f(X[2 * a.P]);
  const TX* xb = X + (size_t)b * 3 * a.P;
  float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  auto add = [&](float x0, float x1, float x2) __attribute__((always_inline)) {
    const float d0 = x0 - s0, d1 = x1 - s1, d2 = x2 - s2;
    acc[0] += d0;
    acc[1] += d1;
    acc[2] += d2;
    acc[3] += d0 * d0;
    acc[4] += d0 * d1;
    acc[5] += d0 * d2;
    acc[6] += d1 * d1;
    acc[7] += d1 * d2;
    acc[8] += d2 * d2;
  };
  const long long stride = (long long)gridDim.x * 256;
  long long p0 = 0;
  // four pixels per thread and step (one 4-element vector load per plane)
  // when the planes are whole vectors and aligned; any other pixels one by one
  constexpr int kV = 4;
  if (a.P % kV == 0 && reinterpret_cast<uintptr_t>(X) % (kV * sizeof(TX)) == 0) {
    typedef typename Carrier<sizeof(TX) * kV>::type C;
    for (long long v = (long long)chunk * 256 + tid; v < a.P / kV; v += stride) {
      TX t[3][kV];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const C c = *reinterpret_cast<const C*>(xb + k * a.P + kV * v);
        __builtin_memcpy(t[k], &c, sizeof(C));
      }
#pragma unroll
      for (int e = 0; e < kV; ++e) add(to_f(t[0][e]), to_f(t[1][e]), to_f(t[2][e]));
    }
    p0 = a.P;
  }
  for (long long p = p0 + (long long)chunk * 256 + tid; p < a.P; p += stride)
    add(to_f(xb[p]), to_f(xb[a.P + p]), to_f(xb[2 * a.P + p]));
#pragma unroll
  for (int k = 0; k < 9; ++k) red[k][tid] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st)
#pragma unroll
      for (int k = 0; k < 9; ++k) red[k][tid] += red[k][tid + st];
    __syncthreads();
  }
  if (tid < 9) a.part[((size_t)b * gridDim.x + chunk) * kMomFloats + tid] = red[tid][0];
}

// ------------------------------------------------------------ folding

struct FoldArgs {
  const float* part;     // moments partials, npart entries (null when stats_in given)
  int npart;
  const void* x;         // the call's input (for the shift), element type by `dtype`
  int dtype;
  long long P;           // plane pixels
  float count;           // pixels of the call (n * P)
  const float* params;   // user parameters
  int hidden;
  float bn_eps, slope;
  const float* stats_in; // optional: mean[3], cov[9] of the call
  float* stats_out;      // optional
  float* fold;           // kFoldFloats
};

__device__ __forceinline__ float load_any(const void* x, int dtype, long long i) {
  if (dtype == GF_F32) return reinterpret_cast<const float*>(x)[i];
  if (dtype == GF_F16) return (float)reinterpret_cast<const _Float16*>(x)[i];
  return to_f(reinterpret_cast<const bf16*>(x)[i]);
}

// One workgroup: the partials are summed by all 256 threads in a fixed
// order (strided, then a tree), the tiny fold arithmetic runs on thread 0.
__global__ __launch_bounds__(256) void guide_fold_kernel(FoldArgs a) {
  __shared__ float red[9][256];
  const int tid = threadIdx.x;
  if (!a.stats_in) {
    float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int q = tid; q < a.npart; q += 256)
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[k] += a.part[(size_t)q * kMomFloats + k];
#pragma unroll
    for (int k = 0; k < 9; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st)
#pragma unroll
        for (int k = 0; k < 9; ++k) red[k][tid] += red[k][tid + st];
      __syncthreads();
    }
  }
  __shared__ float st[12];  // batch mean (3) and covariance (9) of x
  if (tid == 0) {
    float mean[3], cov[9];
    if (a.stats_in) {
      for (int i = 0; i < 3; ++i) mean[i] = a.stats_in[i];
      for (int i = 0; i < 9; ++i) cov[i] = a.stats_in[3 + i];
    } else {
      float S[9];
      for (int k = 0; k < 9; ++k) S[k] = red[k][0];
      const float inv = 1.f / a.count;
      const float sh[3] = {load_any(a.x, a.dtype, 0), load_any(a.x, a.dtype, a.P),
                           load_any(a.x, a.dtype, 2 * a.P)};
      float d[3];
      for (int i = 0; i < 3; ++i) {
        d[i] = S[i] * inv;  // mean of the shifted values
        mean[i] = sh[i] + d[i];
      }
      const int idx[3][3] = {{3, 4, 5}, {4, 6, 7}, {5, 7, 8}};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) cov[i * 3 + j] = S[idx[i][j]] * inv - d[i] * d[j];
    }
    for (int i = 0; i < 3; ++i) st[i] = mean[i];
    for (int i = 0; i < 9; ++i) st[3 + i] = cov[i];
    if (a.stats_out)
      for (int i = 0; i < 12; ++i) a.stats_out[i] = st[i];
  }
  __syncthreads();
  const int K = a.hidden;
  const float* W1 = a.params;
  const float* W2 = W1 + 3 * K;
  const float* b2 = W2 + 3 * K;
  const float lam = b2[3], mu = b2[4];
  const float* gamma = b2 + 5;
  const float* beta = gamma + K;
  float* f = a.fold;
  // one thread per (padded) hidden channel; padding channels get zeros
  if (tid < kKP) {
    const int k = tid;
    float m = 0.f, v = 0.f, w[3] = {0.f, 0.f, 0.f}, g = 0.f, be = 0.f, rstd = 0.f;
    if (k < K) {
      for (int i = 0; i < 3; ++i) w[i] = W1[k * 3 + i];
      for (int i = 0; i < 3; ++i) {
        m += w[i] * st[i];
        for (int j = 0; j < 3; ++j) v += w[i] * w[j] * st[3 + i * 3 + j];
      }
      rstd = 1.f / sqrtf(fmaxf(v, 0.f) + a.bn_eps);
      g = gamma[k];
      be = beta[k];
    }
    const float ak = k < K ? lam + mu * g * rstd : 0.f;
    for (int i = 0; i < 3; ++i) {
      f[FO_W1F + k * 3 + i] = ak * w[i];
      f[FO_W1 + k * 3 + i] = w[i];
    }
    f[FO_BF + k] = k < K ? mu * (be - g * m * rstd) : 0.f;
    for (int c = 0; c < 3; ++c) f[FO_W2 + c * kKP + k] = k < K ? W2[c * K + k] : 0.f;
    f[FO_M + k] = m;
    f[FO_RSTD + k] = rstd;
    f[FO_CDH + k] = mu * g * rstd;
    f[FO_GAM + k] = g;
    f[FO_BET + k] = be;
    f[FO_MDY + k] = 0.f;
    f[FO_MDYHN + k] = 0.f;
  } else if (tid == kKP) {
    for (int c = 0; c < 3; ++c) f[FO_B2 + c] = b2[c];
    f[FO_SCAL + 0] = lam;
    f[FO_SCAL + 1] = mu;
    f[FO_SCAL + 2] = a.slope;
    f[FO_SCAL + 3] = a.count;
    for (int i = 0; i < 3; ++i) f[FO_MEAN + i] = st[i];
    for (int i = 0; i < 9; ++i) f[FO_COV + i] = st[3 + i];
  }
}

// ------------------------------------------------------------ per-pixel map

// The folded constants one pixel of the transform needs, copied into
// registers before the pixel loop (uniform: the compiler keeps them in
// scalar registers where it can).
struct FoldRegs {
  float w1f[kKP][3], bf[kKP], w2[3][kKP], b2[3], slope;
};

__device__ __forceinline__ void load_fold(const float* __restrict__ f, FoldRegs& c) {
#pragma unroll
  for (int k = 0; k < kKP; ++k) {
    c.w1f[k][0] = f[FO_W1F + 3 * k];
    c.w1f[k][1] = f[FO_W1F + 3 * k + 1];
    c.w1f[k][2] = f[FO_W1F + 3 * k + 2];
    c.bf[k] = f[FO_BF + k];
    c.w2[0][k] = f[FO_W2 + k];
    c.w2[1][k] = f[FO_W2 + kKP + k];
    c.w2[2][k] = f[FO_W2 + 2 * kKP + k];
  }
  c.b2[0] = f[FO_B2];
  c.b2[1] = f[FO_B2 + 1];
  c.b2[2] = f[FO_B2 + 2];
  c.slope = f[FO_SCAL + 2];
}

// G of PX pixels in FP64 (one rounding at the store): the filter amplifies
// per-pixel noise in G by the inverse local spread of G, so G carries only
// its own half-ulp rounding (the folded constants are FP32; their rounding
// perturbs G smoothly across pixels, which the filter does not amplify).
// The constants sit in LDS as FP64 (row k: w1f[k][0..2], bf[k], w2[0..2][k]);
// PX pixels share each read.
struct FoldF64 {
  double k[kKP][8];
  double b2[3], slope;
};

__device__ __forceinline__ void stage_fold_f64(const float* __restrict__ f, FoldF64& c) {
  const int t = threadIdx.x;
  if (t < kKP) {
    c.k[t][0] = f[FO_W1F + 3 * t];
    c.k[t][1] = f[FO_W1F + 3 * t + 1];
    c.k[t][2] = f[FO_W1F + 3 * t + 2];
    c.k[t][3] = f[FO_BF + t];
    c.k[t][4] = f[FO_W2 + t];
    c.k[t][5] = f[FO_W2 + kKP + t];
    c.k[t][6] = f[FO_W2 + 2 * kKP + t];
    c.k[t][7] = 0.0;
  } else if (t == kKP) {
    c.b2[0] = f[FO_B2];
    c.b2[1] = f[FO_B2 + 1];
    c.b2[2] = f[FO_B2 + 2];
    c.slope = f[FO_SCAL + 2];
  }
  __syncthreads();
}

// The branch taken by each hidden channel is returned in bits (bit k set
// when y_k > 0): the backward uses the same branches, so the gradient is
// that of the G this map produced (a pixel whose y_k is within rounding of 0
// could otherwise take the other branch in single precision).
template <int PX>
__device__ __forceinline__ void transform_px(const FoldF64& c, const float (&x)[3][PX],
                                             float (&g)[3][PX], unsigned (&bits)[PX]) {
  double acc[3][PX], xd[3][PX];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int e = 0; e < PX; ++e) {
      acc[i][e] = c.b2[i];
      xd[i][e] = x[i][e];
    }
  const double slope = c.slope;
#pragma unroll
  for (int e = 0; e < PX; ++e) bits[e] = 0u;
#pragma unroll 2
  for (int k = 0; k < kKP; ++k) {
    const double a0 = c.k[k][0], a1 = c.k[k][1], a2 = c.k[k][2], bb = c.k[k][3];
    const double v0 = c.k[k][4], v1 = c.k[k][5], v2 = c.k[k][6];
#pragma unroll
    for (int e = 0; e < PX; ++e) {
      const double y = bb + a0 * xd[0][e] + a1 * xd[1][e] + a2 * xd[2][e];
      const bool pos = y > 0.0;
      const double z = pos ? y : slope * y;
      bits[e] |= (pos ? 1u : 0u) << k;
      acc[0][e] += v0 * z;
      acc[1][e] += v1 * z;
      acc[2][e] += v2 * z;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int e = 0; e < PX; ++e) g[i][e] = (float)acc[i][e];
}

struct MapArgs {
  const void* x;   // [n][c_in][P]
  float* G;        // [n][c][P]
  long long P;
  int c_in, c;
  const float* fold;
  uint16_t* mask;  // transform: [n][P] leaky-ReLU branches (bit k: y_k > 0)
};

// Grey map: every output channel is the mean of the c_in input channels.
template <typename TX>
__global__ __launch_bounds__(256) void guide_map_grey_kernel(MapArgs a) {
  const TX* X = reinterpret_cast<const TX*>(a.x) + (size_t)blockIdx.y * a.c_in * a.P;
  float* G = a.G + (size_t)blockIdx.y * a.c * a.P;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < a.P;
       p += (long long)gridDim.x * 256) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < a.c_in) s += to_f(X[i * a.P + p]);
    s *= 1.f / (float)a.c_in;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < a.c) G[c * a.P + p] = s;
  }
}

// Transform map: 4 adjacent pixels per thread (vector loads and stores)
// when the plane size allows, else one.
template <typename TX>
__global__ __launch_bounds__(256) void guide_map_transform_kernel(MapArgs a) {
  const TX* __restrict__ X = reinterpret_cast<const TX*>(a.x) + (size_t)blockIdx.y * 3 * a.P;
  float* __restrict__ G = a.G + (size_t)blockIdx.y * 3 * a.P;
  uint16_t* __restrict__ M = a.mask + (size_t)blockIdx.y * a.P;
  __shared__ FoldF64 c;
  stage_fold_f64(a.fold, c);
  const long long stride = (long long)gridDim.x * 256;
  if ((a.P & 3) == 0) {
    const long long P4 = a.P >> 2;
    for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < P4; v += stride) {
      float x[3][4], g[3][4];
      unsigned bits[4];
#pragma unroll
      for (int i = 0; i < 3; ++i) load_vec_nt<TX, 4>(X + i * a.P + 4 * v, x[i]);
      transform_px<4>(c, x, g, bits);
      *reinterpret_cast<uint2*>(M + 4 * v) =
          make_uint2(bits[0] | (bits[1] << 16), bits[2] | (bits[3] << 16));
#pragma unroll
      for (int i = 0; i < 3; ++i)
        *reinterpret_cast<float4*>(G + i * a.P + 4 * v) = make_float4(g[i][0], g[i][1], g[i][2],
                                                                      g[i][3]);
    }
  } else {
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < a.P; p += stride) {
      float x[3][1], g[3][1];
      unsigned bits[1];
#pragma unroll
      for (int i = 0; i < 3; ++i) x[i][0] = to_f(X[i * a.P + p]);
      transform_px<1>(c, x, g, bits);
      M[p] = (uint16_t)bits[0];
#pragma unroll
      for (int i = 0; i < 3; ++i) G[i * a.P + p] = g[i][0];
    }
  }
}

// ------------------------------------------------------------ guide backward

struct GBwdArgs {
  const void* x;     // [n][c_in][P]
  const float* dG;   // [n][c][P]
  void* dx;          // grey: [n][c_in][P] of type TDX (may be null)
  float* part;       // transform: [n * chunks][kAccFloats]
  long long P;
  int c_in, c;
  const float* fold;
  const uint16_t* mask;  // transform: the map's leaky-ReLU branches
  int hidden;            // transform: hidden channels (the rest of kKP are zero)
};

template <typename TX, typename TDX, int MODE>
__global__ __launch_bounds__(256) void guide_bwd_kernel(GBwdArgs a) {
  const int b = blockIdx.y, tid = threadIdx.x;
  const TX* X = reinterpret_cast<const TX*>(a.x) + (size_t)b * a.c_in * a.P;
  const float* dG = a.dG + (size_t)b * a.c * a.P;
  if (MODE == GF_GUIDE_GREY) {
    TDX* dX = reinterpret_cast<TDX*>(a.dx) + (size_t)b * a.c_in * a.P;
    for (long long p = (long long)blockIdx.x * 256 + tid; p < a.P; p += (long long)gridDim.x * 256) {
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < a.c) s += dG[c * a.P + p];
      s *= 1.f / (float)a.c_in;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < a.c_in) dX[i * a.P + p] = from_f<TDX>(s);
    }
    return;
  }
  const float* __restrict__ f = a.fold;
  const float slope = f[FO_SCAL + 2];
  const float mx0 = f[FO_MEAN], mx1 = f[FO_MEAN + 1], mx2 = f[FO_MEAN + 2];
  // The 112 folded constants are read from LDS inside the pixel loop
  // (broadcast reads): held across the loop they exceed the scalar
  // registers and were spilled to vector-register lanes, costing about 90
  // lane reads per pixel.  Unit k: (w1f[k][0..2], bf[k]), (w2[0..2][k], 0).
  __shared__ float4 cst[2 * kKP];
  if (tid < kKP)
    cst[2 * tid] = make_float4(f[FO_W1F + 3 * tid], f[FO_W1F + 3 * tid + 1],
                               f[FO_W1F + 3 * tid + 2], f[FO_BF + tid]);
  else if (tid < 2 * kKP)
    cst[2 * (tid - kKP) + 1] = make_float4(f[FO_W2 + tid - kKP], f[FO_W2 + tid],
                                           f[FO_W2 + kKP + tid], 0.f);
  __syncthreads();
  float acc[AC_N];
#pragma unroll
  for (int k = 0; k < AC_N; ++k) acc[k] = 0.f;
  const uint16_t* Mk = a.mask + (size_t)b * a.P;
  // two pixels per iteration (p and p + T), so that each constant read
  // serves both; a missing second pixel contributes zero (dG := 0)
  const long long T = (long long)gridDim.x * 256;
  for (long long p = (long long)blockIdx.x * 256 + tid; p < a.P; p += 2 * T) {
    const bool two = p + T < a.P;
    const long long q = two ? p + T : p;
    float x[2][3], d[2][3];
    unsigned mb[2];
    x[0][0] = to_f(X[p]);
    x[0][1] = to_f(X[a.P + p]);
    x[0][2] = to_f(X[2 * a.P + p]);
    x[1][0] = to_f(X[q]);
    x[1][1] = to_f(X[a.P + q]);
    x[1][2] = to_f(X[2 * a.P + q]);
    d[0][0] = dG[p];
    d[0][1] = dG[a.P + p];
    d[0][2] = dG[2 * a.P + p];
    d[1][0] = two ? dG[q] : 0.f;
    d[1][1] = two ? dG[a.P + q] : 0.f;
    d[1][2] = two ? dG[2 * a.P + q] : 0.f;
    mb[0] = Mk[p];
    mb[1] = Mk[q];
    // an offset the compiler cannot see through keeps the constant reads in
    // the loop (hoisted, they would be held in registers again)
    int coff = 0;
    asm volatile("" : "+v"(coff));
    const float4* cc = cst + coff;
    float xc[2][3];  // the inputs less their batch means, once per pixel
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[AC_DG] += d[j][0];
      acc[AC_DG + 1] += d[j][1];
      acc[AC_DG + 2] += d[j][2];
      xc[j][0] = x[j][0] - mx0;
      xc[j][1] = x[j][1] - mx1;
      xc[j][2] = x[j][2] - mx2;
    }
#pragma unroll
    for (int k = 0; k < kKP; ++k) {
      // the padding channels have zero weights and add nothing: skipped
      // behind a uniform (scalar) branch, the loop staying fully unrolled so
      // that every accumulator index is a constant
      if (k < a.hidden) {
      const float4 u = cc[2 * k], v = cc[2 * k + 1];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float y = u.w + u.x * x[j][0] + u.y * x[j][1] + u.z * x[j][2];
        // the branch's factor, selected once for z and dy (x 1 is exact)
        const float sl = (mb[j] >> k) & 1u ? 1.f : slope;
        const float z = y * sl;
        acc[AC_DGZ + k] += d[j][0] * z;
        acc[AC_DGZ + kKP + k] += d[j][1] * z;
        acc[AC_DGZ + 2 * kKP + k] += d[j][2] * z;
        const float dz = v.x * d[j][0] + v.y * d[j][1] + v.z * d[j][2];
        const float dy = dz * sl;
        acc[AC_DY + k] += dy;
        acc[AC_DYX + 3 * k] += dy * xc[j][0];
        acc[AC_DYX + 3 * k + 1] += dy * xc[j][1];
        acc[AC_DYX + 3 * k + 2] += dy * xc[j][2];
      }
      }
    }
  }
  // fixed-order reduction: within each wave by shuffles, then across the
  // four waves through LDS
  __shared__ float red[4][AC_N];
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int k = 0; k < AC_N; ++k) {
    float v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  for (int k = tid; k < AC_N; k += 256)
    a.part[((size_t)b * gridDim.x + blockIdx.x) * kAccFloats + k] =
        ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// One workgroup per accumulator; fixed-order sum (strided, then a tree).
__global__ __launch_bounds__(256) void guide_acc_reduce_kernel(const float* part, int npart,
                                                                float* tot) {
  __shared__ float red[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  float s = 0.f;
  for (int q = tid; q < npart; q += 256) s += part[(size_t)q * kAccFloats + k];
  red[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) tot[k] = red[0];
}

// Parameter gradients from the two calls' totals (I_lo call first, then
// I_hi), and the batch means of dy and dy * hn each call's input gradient
// needs.  One thread; the data is tiny.
struct GradArgs {
  const float* tot[2];
  float* fold[2];
  int hidden;
  float* dparams;  // may be null
};

__global__ __launch_bounds__(64) void guide_grad_kernel(GradArgs a) {
  // one thread per hidden channel; lam and mu sum the channels' shares in
  // channel order afterwards
  __shared__ float slam[kKP], smu[kKP];
  const int K = a.hidden, k = threadIdx.x;
  float* d = a.dparams;
  if (k < kKP) {
    slam[k] = 0.f;
    smu[k] = 0.f;
  }
  if (k < K) {
    float dw1[3] = {0.f, 0.f, 0.f}, dw2[3] = {0.f, 0.f, 0.f};
    float dl = 0.f, dm = 0.f, dg = 0.f, db = 0.f;
    for (int call = 0; call < 2; ++call) {
      const float* T = a.tot[call];
      float* f = a.fold[call];
      const float lam = f[FO_SCAL], mu = f[FO_SCAL + 1], P = f[FO_SCAL + 3];
      const float* mean = f + FO_MEAN;
      const float* cov = f + FO_COV;
      // With e = x - mean(x) (the accumulators hold sums of dy e):
      //   sum dy_k h_k        = W1_k . sum dy_k e + m_k sum dy_k
      //   sum dy_k hn_k       = rstd_k W1_k . sum dy_k e
      //   sum hn_k x_i        = rstd_k P (W1_k C)_i          (C: covariance of x)
      //   sum dy_k x_i - mean(dy_k) sum x_i = sum dy_k e_i
      const float* W1 = f + FO_W1 + 3 * k;
      const float* Se = T + AC_DYX + 3 * k;
      const float m = f[FO_M + k], rstd = f[FO_RSTD + k], cdh = f[FO_CDH + k];
      const float sdy = T[AC_DY + k];
      const float sdye = W1[0] * Se[0] + W1[1] * Se[1] + W1[2] * Se[2];
      const float sdyhn = rstd * sdye;
      f[FO_MDY + k] = sdy / P;
      f[FO_MDYHN + k] = sdyhn / P;
      for (int i = 0; i < 3; ++i) {
        const float wc = W1[0] * cov[i] + W1[1] * cov[3 + i] + W1[2] * cov[6 + i];
        const float shnx = rstd * P * wc;
        dw1[i] += lam * (Se[i] + mean[i] * sdy) + cdh * (Se[i] - (sdyhn / P) * shnx);
      }
      const float gamma = f[FO_GAM + k], beta = f[FO_BET + k];
      dl += sdye + m * sdy;
      dm += gamma * sdyhn + beta * sdy;
      dg += mu * sdyhn;
      db += mu * sdy;
      for (int c = 0; c < 3; ++c) dw2[c] += T[AC_DGZ + c * kKP + k];
    }
    if (d) {
      for (int i = 0; i < 3; ++i) d[3 * k + i] = dw1[i];
      for (int c = 0; c < 3; ++c) d[3 * K + c * K + k] = dw2[c];
      d[6 * K + 5 + k] = dg;
      d[7 * K + 5 + k] = db;
    }
    slam[k] = dl;
    smu[k] = dm;
  }
  __syncthreads();
  if (k == 0 && d) {
    float dl = 0.f, dm = 0.f;
    for (int j = 0; j < K; ++j) {
      dl += slam[j];
      dm += smu[j];
    }
    for (int c = 0; c < 3; ++c) d[6 * K + c] = a.tot[0][AC_DG + c] + a.tot[1][AC_DG + c];
    d[6 * K + 3] = dl;
    d[6 * K + 4] = dm;
  }
}

// Input gradient of the transform: dh_k = lam dy_k + mu gamma_k rstd_k
// (dy_k - mean(dy_k) - hn_k mean(dy_k hn_k)), dx = W1^T dh.
template <typename TX, typename TDX>
__global__ __launch_bounds__(256) void guide_dx_kernel(GBwdArgs a) {
  const int b = blockIdx.y;
  const TX* __restrict__ X = reinterpret_cast<const TX*>(a.x) + (size_t)b * 3 * a.P;
  const float* __restrict__ dG = a.dG + (size_t)b * 3 * a.P;
  TDX* __restrict__ dX = reinterpret_cast<TDX*>(a.dx) + (size_t)b * 3 * a.P;
  const float* __restrict__ f = a.fold;
  FoldRegs c;
  load_fold(f, c);
  float w1[kKP][3], m[kKP], rstd[kKP], cdh[kKP], mdy[kKP], mdyhn[kKP];
#pragma unroll
  for (int k = 0; k < kKP; ++k) {
    w1[k][0] = f[FO_W1 + 3 * k];
    w1[k][1] = f[FO_W1 + 3 * k + 1];
    w1[k][2] = f[FO_W1 + 3 * k + 2];
    m[k] = f[FO_M + k];
    rstd[k] = f[FO_RSTD + k];
    cdh[k] = f[FO_CDH + k];
    mdy[k] = f[FO_MDY + k];
    mdyhn[k] = f[FO_MDYHN + k];
  }
  const float lam = f[FO_SCAL], slope = c.slope;
  const uint16_t* __restrict__ Mk = a.mask + (size_t)b * a.P;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < a.P;
       p += (long long)gridDim.x * 256) {
    const float x0 = to_f(X[p]), x1 = to_f(X[a.P + p]), x2 = to_f(X[2 * a.P + p]);
    const float d0 = dG[p], d1 = dG[a.P + p], d2 = dG[2 * a.P + p];
    const unsigned mbits = Mk[p];
    float o0 = 0.f, o1 = 0.f, o2 = 0.f;
#pragma unroll
    for (int k = 0; k < kKP; ++k) {
      const float dz = c.w2[0][k] * d0 + c.w2[1][k] * d1 + c.w2[2][k] * d2;
      const float dy = ((mbits >> k) & 1u) ? dz : slope * dz;
      const float h = w1[k][0] * x0 + w1[k][1] * x1 + w1[k][2] * x2;
      const float hn = (h - m[k]) * rstd[k];
      const float dh = lam * dy + cdh[k] * (dy - mdy[k] - hn * mdyhn[k]);
      o0 += w1[k][0] * dh;
      o1 += w1[k][1] * dh;
      o2 += w1[k][2] * dh;
    }
    dX[p] = from_f<TDX>(o0);
    dX[a.P + p] = from_f<TDX>(o1);
    dX[2 * a.P + p] = from_f<TDX>(o2);
  }
}

// ------------------------------------------------------------ guided pipelines

template <typename T>
hipError_t guided_fold(const Plan& p, const void* x, long long P, int chunks, float* part,
                       const float* stats_in, float* stats_out, float* fold, hipStream_t s) {
  if (!stats_in) {
    MomArgs m{x, P, part};
    prof_begin("gf_guide_moments", s);
    hipLaunchKernelGGL(moments_kernel<T>, dim3(chunks, p.n), dim3(256), 0, s, m);
    prof_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  FoldArgs f{part, chunks * p.n, x, p.dtype, P, (float)((double)P * p.n), p.gparams,
             p.hidden, p.bn_eps, p.slope, stats_in, stats_out, fold};
  prof_begin("gf_guide_fold", s);
  hipLaunchKernelGGL(guide_fold_kernel, dim3(1), dim3(256), 0, s, f);
  prof_end(s);
  return hipGetLastError();
}

template <typename T>
hipError_t guided_map(const Plan& p, const void* x, float* G, long long P, int chunks,
                      const float* fold, uint16_t* mask, hipStream_t s) {
  MapArgs m{x, G, P, p.c_in, p.c, fold, mask};
  prof_begin("gf_guide_map", s);
  if (p.gmode == GF_GUIDE_GREY)
    hipLaunchKernelGGL((guide_map_grey_kernel<T>), dim3(chunks * 4, p.n), dim3(256), 0,
                       s, m);
  else
    hipLaunchKernelGGL((guide_map_transform_kernel<T>), dim3(chunks * 4, p.n),
                       dim3(256), 0, s, m);
  prof_end(s);
  return hipGetLastError();
}

// Statistics and folded constants of both calls (transform only).
template <typename T>
hipError_t guided_prepare(const Plan& p, const void* I_lo, const void* I_hi, char* ws,
                          bool backward, hipStream_t s) {
  if (p.gmode != GF_GUIDE_TRANSFORM) return hipSuccess;
  float* part = reinterpret_cast<float*>(ws + p.off_mom);
  float* fold = reinterpret_cast<float*>(ws + p.off_fold);
  const int sc = (int)gf_guide_stats_count(3) / 2;
  const bool saved = backward && p.use_stats;
  float* st_out = (!backward && p.gstats) ? p.gstats : nullptr;
  hipError_t e = guided_fold<T>(p, I_lo, (long long)p.h * p.w, p.g_chunks_lo, part,
                                saved ? p.gstats : nullptr, st_out, fold, s);
  if (e != hipSuccess) return e;
  return guided_fold<T>(p, I_hi, (long long)p.H * p.W, p.g_chunks_hi,
                        part + (size_t)kMomFloats * p.n * p.g_chunks_lo,
                        saved ? p.gstats + sc : nullptr, st_out ? st_out + sc : nullptr,
                        fold + kFoldFloats, s);
}

template <typename T>
hipError_t forward_guided_t(const Plan& p, const FwdArgs& f, hipStream_t s) {
  hipError_t e = guided_prepare<T>(p, f.I_lo, f.I_hi, f.ws, false, s);
  if (e != hipSuccess) return e;
  const float* fold = reinterpret_cast<const float*>(f.ws + p.off_fold);
  float* Gl = reinterpret_cast<float*>(f.ws + p.off_gl);
  float* Gh = reinterpret_cast<float*>(f.ws + p.off_gh);
  uint16_t* Ml = reinterpret_cast<uint16_t*>(f.ws + p.off_mlo);
  uint16_t* Mh = reinterpret_cast<uint16_t*>(f.ws + p.off_mhi);
  e = guided_map<T>(p, f.I_lo, Gl, (long long)p.h * p.w, p.g_chunks_lo, fold, Ml, s);
  if (e != hipSuccess) return e;
  e = guided_map<T>(p, f.I_hi, Gh, (long long)p.H * p.W, p.g_chunks_hi, fold + kFoldFloats, Mh,
                    s);
  if (e != hipSuccess) return e;
  float* abar = reinterpret_cast<float*>(f.ws + p.off_abar);
  float* bbar = reinterpret_cast<float*>(f.ws + p.off_bbar);
  e = launch_coef<float, T>(p, Gl, f.p_lo, f.eps, f.eps_count, abar, bbar,
                            reinterpret_cast<float*>(f.ws + p.off_x), s);
  if (e != hipSuccess) return e;
  return launch_apply<float, T>(p, Gh, f.q, abar, bbar, s);
}

template <typename T>
hipError_t guided_input_grad(const Plan& p, const void* x, const float* dG, void* dx, bool lo,
                             float* part, const float* fold, const uint16_t* mask,
                             hipStream_t s) {
  const long long P = lo ? (long long)p.h * p.w : (long long)p.H * p.W;
  const int chunks = lo ? p.g_chunks_lo : p.g_chunks_hi;
  GBwdArgs g{x, dG, dx, part, P, p.c_in, p.c, fold, mask, p.hidden};
  prof_begin(lo ? "gf_guide_dx_lo" : "gf_guide_dx_hi", s);
  if (p.gmode == GF_GUIDE_GREY) {
    if (lo)
      hipLaunchKernelGGL((guide_bwd_kernel<T, float, GF_GUIDE_GREY>), dim3(chunks * 4, p.n),
                         dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((guide_bwd_kernel<T, T, GF_GUIDE_GREY>), dim3(chunks * 4, p.n),
                         dim3(256), 0, s, g);
  } else {
    if (lo)
      hipLaunchKernelGGL((guide_dx_kernel<T, float>), dim3(chunks * 4, p.n), dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((guide_dx_kernel<T, T>), dim3(chunks * 4, p.n), dim3(256), 0, s, g);
  }
  prof_end(s);
  return hipGetLastError();
}

// With b.q set, the forward runs first on the same guide maps and
// coefficients (batch statistics computed, and saved if asked, as by the
// forward).
template <typename T>
hipError_t backward_guided_t(const Plan& p, const BwdArgs& b, hipStream_t s) {
  hipError_t e = guided_prepare<T>(p, b.I_lo, b.I_hi, b.ws, b.q == nullptr, s);
  if (e != hipSuccess) return e;
  float* fold = reinterpret_cast<float*>(b.ws + p.off_fold);
  float* Gl = reinterpret_cast<float*>(b.ws + p.off_gl);
  float* Gh = reinterpret_cast<float*>(b.ws + p.off_gh);
  float* dGl = reinterpret_cast<float*>(b.ws + p.off_dgl);
  float* dGh = reinterpret_cast<float*>(b.ws + p.off_dgh);
  uint16_t* Ml = reinterpret_cast<uint16_t*>(b.ws + p.off_mlo);
  uint16_t* Mh = reinterpret_cast<uint16_t*>(b.ws + p.off_mhi);
  e = guided_map<T>(p, b.I_lo, Gl, (long long)p.h * p.w, p.g_chunks_lo, fold, Ml, s);
  if (e != hipSuccess) return e;
  e = guided_map<T>(p, b.I_hi, Gh, (long long)p.H * p.W, p.g_chunks_hi, fold + kFoldFloats, Mh,
                    s);
  if (e != hipSuccess) return e;
  float* abar = reinterpret_cast<float*>(b.ws + p.off_abar);
  float* U = reinterpret_cast<float*>(b.ws + p.off_u);
  float* bbar = b.q ? reinterpret_cast<float*>(b.ws + p.off_bbar) : nullptr;
  e = launch_coef<float, T>(p, Gl, b.p_lo, b.eps, b.eps_count, abar, bbar,
                            reinterpret_cast<float*>(b.ws + p.off_x), s);
  if (e != hipSuccess) return e;
  // dG_h = dq * A_h (the guide gradient at high resolution) and the
  // transposed-bilinear partial planes (and q, in the same pass, with the
  // forward)
  float* V = reinterpret_cast<float*>(b.ws + p.off_v);
  e = launch_bwd_hi<float, T, float, T>(p, Gh, b.dq, dGh, abar, U, V, s, bbar, b.q);
  if (e != hipSuccess) return e;
  float* epart = reinterpret_cast<float*>(b.ws + p.off_eps);
  e = launch_bwd_lo<float, T>(p, Gl, b.p_lo, b.eps, b.eps_count, U, dGl, b.dp_lo, epart,
                              reinterpret_cast<float*>(b.ws + p.off_x), s);
  if (e != hipSuccess) return e;
  if (b.deps) {
    e = launch_eps_reduce(p, epart, b.eps_count, b.deps, s);
    if (e != hipSuccess) return e;
  }
  if (p.gmode == GF_GUIDE_TRANSFORM) {
    // parameter gradients: per-chunk sums, fixed-order totals, finalisation
    float* part = reinterpret_cast<float*>(b.ws + p.off_accp);
    float* tot = reinterpret_cast<float*>(b.ws + p.off_acct);
    const size_t half = (size_t)kAccFloats * p.n * p.g_chunks_lo;
    for (int call = 0; call < 2; ++call) {
      const bool lo = call == 0;
      const long long P = lo ? (long long)p.h * p.w : (long long)p.H * p.W;
      const int chunks = lo ? p.g_chunks_lo : p.g_chunks_hi;
      GBwdArgs g{lo ? b.I_lo : b.I_hi, lo ? dGl : dGh, nullptr, part + (lo ? 0 : half), P,
                 p.c_in, p.c, fold + call * kFoldFloats,
                 reinterpret_cast<const uint16_t*>(b.ws + (lo ? p.off_mlo : p.off_mhi)),
                 p.hidden};
      prof_begin("gf_guide_bwd", s);
      hipLaunchKernelGGL((guide_bwd_kernel<T, float, GF_GUIDE_TRANSFORM>), dim3(chunks, p.n),
                         dim3(256), 0, s, g);
      prof_end(s);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      prof_begin("gf_guide_acc_reduce", s);
      hipLaunchKernelGGL(guide_acc_reduce_kernel, dim3(AC_N), dim3(256), 0, s,
                         part + (lo ? 0 : half), chunks * p.n, tot + call * kAccFloats);
      prof_end(s);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    GradArgs ga{{tot, tot + kAccFloats}, {fold, fold + kFoldFloats}, p.hidden, b.dparams};
    prof_begin("gf_guide_grad", s);
    hipLaunchKernelGGL(guide_grad_kernel, dim3(1), dim3(64), 0, s, ga);
    prof_end(s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.dI_lo) {
    e = guided_input_grad<T>(p, b.I_lo, dGl, b.dI_lo, true, nullptr, fold, Ml, s);
    if (e != hipSuccess) return e;
  }
  if (b.dI_hi) {
    e = guided_input_grad<T>(p, b.I_hi, dGh, b.dI_hi, false, nullptr, fold + kFoldFloats, Mh,
                             s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace gf
