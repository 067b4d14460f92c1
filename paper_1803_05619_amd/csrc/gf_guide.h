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
//   guide_map_kernel     G = F(x) per pixel
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
  for (long long p = (long long)chunk * 256 + tid; p < a.P; p += (long long)gridDim.x * 256) {
    const float d0 = to_f(xb[p]) - s0, d1 = to_f(xb[a.P + p]) - s1, d2 = to_f(xb[2 * a.P + p]) - s2;
    acc[0] += d0;
    acc[1] += d1;
    acc[2] += d2;
    acc[3] += d0 * d0;
    acc[4] += d0 * d1;
    acc[5] += d0 * d2;
    acc[6] += d1 * d1;
    acc[7] += d1 * d2;
    acc[8] += d2 * d2;
  }
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

// One workgroup (thread 0 does the arithmetic; the data is tiny).
__global__ __launch_bounds__(64) void guide_fold_kernel(FoldArgs a) {
  if (threadIdx.x != 0) return;
  float mean[3], cov[9];
  if (a.stats_in) {
    for (int i = 0; i < 3; ++i) mean[i] = a.stats_in[i];
    for (int i = 0; i < 9; ++i) cov[i] = a.stats_in[3 + i];
  } else {
    float S[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < a.npart; ++q)
      for (int k = 0; k < 9; ++k) S[k] += a.part[(size_t)q * kMomFloats + k];
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
  if (a.stats_out) {
    for (int i = 0; i < 3; ++i) a.stats_out[i] = mean[i];
    for (int i = 0; i < 9; ++i) a.stats_out[3 + i] = cov[i];
  }
  const int K = a.hidden;
  const float* W1 = a.params;
  const float* W2 = W1 + 3 * K;
  const float* b2 = W2 + 3 * K;
  const float lam = b2[3], mu = b2[4];
  const float* gamma = b2 + 5;
  const float* beta = gamma + K;
  float* f = a.fold;
  for (int i = 0; i < kFoldFloats; ++i) f[i] = 0.f;
  for (int k = 0; k < K; ++k) {
    float m = 0.f, v = 0.f;
    for (int i = 0; i < 3; ++i) {
      m += W1[k * 3 + i] * mean[i];
      for (int j = 0; j < 3; ++j) v += W1[k * 3 + i] * W1[k * 3 + j] * cov[i * 3 + j];
    }
    const float rstd = 1.f / sqrtf(fmaxf(v, 0.f) + a.bn_eps);
    const float ak = lam + mu * gamma[k] * rstd;
    for (int i = 0; i < 3; ++i) {
      f[FO_W1F + k * 3 + i] = ak * W1[k * 3 + i];
      f[FO_W1 + k * 3 + i] = W1[k * 3 + i];
    }
    f[FO_BF + k] = mu * (beta[k] - gamma[k] * m * rstd);
    for (int c = 0; c < 3; ++c) f[FO_W2 + c * kKP + k] = W2[c * K + k];
    f[FO_M + k] = m;
    f[FO_RSTD + k] = rstd;
    f[FO_CDH + k] = mu * gamma[k] * rstd;
    f[FO_GAM + k] = gamma[k];
    f[FO_BET + k] = beta[k];
  }
  for (int c = 0; c < 3; ++c) f[FO_B2 + c] = b2[c];
  f[FO_SCAL + 0] = lam;
  f[FO_SCAL + 1] = mu;
  f[FO_SCAL + 2] = a.slope;
  f[FO_SCAL + 3] = a.count;
  for (int i = 0; i < 3; ++i) f[FO_MEAN + i] = mean[i];
  for (int i = 0; i < 9; ++i) f[FO_COV + i] = cov[i];
}

// ------------------------------------------------------------ per-pixel map

struct MapArgs {
  const void* x;   // [n][c_in][P]
  float* G;        // [n][c][P]
  long long P;
  int c_in, c;
  const float* fold;
};

// MODE: GF_GUIDE_GREY or GF_GUIDE_TRANSFORM.
template <typename TX, int MODE>
__global__ __launch_bounds__(256) void guide_map_kernel(MapArgs a) {
  const TX* X = reinterpret_cast<const TX*>(a.x) + (size_t)blockIdx.y * a.c_in * a.P;
  float* G = a.G + (size_t)blockIdx.y * a.c * a.P;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < a.P;
       p += (long long)gridDim.x * 256) {
    if (MODE == GF_GUIDE_GREY) {
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < a.c_in) s += to_f(X[i * a.P + p]);
      s *= 1.f / (float)a.c_in;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < a.c) G[c * a.P + p] = s;
    } else {
      // FP64 arithmetic, one rounding at the store: the filter amplifies
      // per-pixel noise in G by the inverse local spread of G, so G carries
      // only its own half-ulp rounding (the folded constants are FP32; their
      // rounding perturbs G smoothly across pixels, which the filter does
      // not amplify).
      const float* f = a.fold;
      const double x0 = to_f(X[p]), x1 = to_f(X[a.P + p]), x2 = to_f(X[2 * a.P + p]);
      double g0 = f[FO_B2], g1 = f[FO_B2 + 1], g2 = f[FO_B2 + 2];
      const double slope = f[FO_SCAL + 2];
#pragma unroll
      for (int k = 0; k < kKP; ++k) {
        const double y = (double)f[FO_BF + k] + (double)f[FO_W1F + 3 * k] * x0 +
                         (double)f[FO_W1F + 3 * k + 1] * x1 + (double)f[FO_W1F + 3 * k + 2] * x2;
        const double z = y > 0.0 ? y : slope * y;
        g0 += (double)f[FO_W2 + k] * z;
        g1 += (double)f[FO_W2 + kKP + k] * z;
        g2 += (double)f[FO_W2 + 2 * kKP + k] * z;
      }
      G[p] = (float)g0;
      G[a.P + p] = (float)g1;
      G[2 * a.P + p] = (float)g2;
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
  const float* f = a.fold;
  const float slope = f[FO_SCAL + 2];
  const float mx0 = f[FO_MEAN], mx1 = f[FO_MEAN + 1], mx2 = f[FO_MEAN + 2];
  float acc[AC_N];
#pragma unroll
  for (int k = 0; k < AC_N; ++k) acc[k] = 0.f;
  for (long long p = (long long)blockIdx.x * 256 + tid; p < a.P; p += (long long)gridDim.x * 256) {
    const float x0 = to_f(X[p]), x1 = to_f(X[a.P + p]), x2 = to_f(X[2 * a.P + p]);
    const float d0 = dG[p], d1 = dG[a.P + p], d2 = dG[2 * a.P + p];
    acc[AC_DG] += d0;
    acc[AC_DG + 1] += d1;
    acc[AC_DG + 2] += d2;
#pragma unroll
    for (int k = 0; k < kKP; ++k) {
      const float y = f[FO_BF + k] + f[FO_W1F + 3 * k] * x0 + f[FO_W1F + 3 * k + 1] * x1 +
                      f[FO_W1F + 3 * k + 2] * x2;
      const bool pos = y > 0.f;
      const float z = pos ? y : slope * y;
      acc[AC_DGZ + k] += d0 * z;
      acc[AC_DGZ + kKP + k] += d1 * z;
      acc[AC_DGZ + 2 * kKP + k] += d2 * z;
      const float dz = f[FO_W2 + k] * d0 + f[FO_W2 + kKP + k] * d1 + f[FO_W2 + 2 * kKP + k] * d2;
      const float dy = pos ? dz : slope * dz;
      acc[AC_DY + k] += dy;
      acc[AC_DYX + 3 * k] += dy * (x0 - mx0);
      acc[AC_DYX + 3 * k + 1] += dy * (x1 - mx1);
      acc[AC_DYX + 3 * k + 2] += dy * (x2 - mx2);
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

__global__ __launch_bounds__(256) void guide_acc_reduce_kernel(const float* part, int npart,
                                                                float* tot) {
  for (int k = threadIdx.x; k < AC_N; k += 256) {
    float s = 0.f;
    for (int q = 0; q < npart; ++q) s += part[(size_t)q * kAccFloats + k];
    tot[k] = s;
  }
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
  if (threadIdx.x != 0) return;
  const int K = a.hidden;
  float* d = a.dparams;
  float* dW1 = d;
  float* dW2 = d ? d + 3 * K : nullptr;
  float* db2 = d ? dW2 + 3 * K : nullptr;
  float* dlam = d ? db2 + 3 : nullptr;
  float* dmu = d ? dlam + 1 : nullptr;
  float* dgam = d ? dmu + 1 : nullptr;
  float* dbet = d ? dgam + K : nullptr;
  if (d)
    for (int i = 0; i < 3 * K + 3 * K + 3 + 2 + 2 * K; ++i) d[i] = 0.f;
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
    for (int k = 0; k < K; ++k) {
      const float* W1 = f + FO_W1 + 3 * k;
      const float* Se = T + AC_DYX + 3 * k;
      const float m = f[FO_M + k], rstd = f[FO_RSTD + k], cdh = f[FO_CDH + k];
      const float sdy = T[AC_DY + k];
      const float sdye = W1[0] * Se[0] + W1[1] * Se[1] + W1[2] * Se[2];
      const float sdyhn = rstd * sdye;
      f[FO_MDY + k] = sdy / P;
      f[FO_MDYHN + k] = sdyhn / P;
      if (!d) continue;
      for (int i = 0; i < 3; ++i) {
        const float wc = W1[0] * cov[i] + W1[1] * cov[3 + i] + W1[2] * cov[6 + i];
        const float shnx = rstd * P * wc;
        dW1[3 * k + i] += lam * (Se[i] + mean[i] * sdy) + cdh * (Se[i] - (sdyhn / P) * shnx);
      }
      const float gamma = f[FO_GAM + k], beta = f[FO_BET + k];
      *dlam += sdye + m * sdy;
      *dmu += gamma * sdyhn + beta * sdy;
      dgam[k] += mu * sdyhn;
      dbet[k] += mu * sdy;
      for (int c = 0; c < 3; ++c) dW2[c * K + k] += T[AC_DGZ + c * kKP + k];
    }
    if (d)
      for (int c = 0; c < 3; ++c) db2[c] += T[AC_DG + c];
  }
}

// Input gradient of the transform: dh_k = lam dy_k + mu gamma_k rstd_k
// (dy_k - mean(dy_k) - hn_k mean(dy_k hn_k)), dx = W1^T dh.
template <typename TX, typename TDX>
__global__ __launch_bounds__(256) void guide_dx_kernel(GBwdArgs a) {
  const int b = blockIdx.y;
  const TX* X = reinterpret_cast<const TX*>(a.x) + (size_t)b * 3 * a.P;
  const float* dG = a.dG + (size_t)b * 3 * a.P;
  TDX* dX = reinterpret_cast<TDX*>(a.dx) + (size_t)b * 3 * a.P;
  const float* f = a.fold;
  const float lam = f[FO_SCAL], slope = f[FO_SCAL + 2];
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < a.P;
       p += (long long)gridDim.x * 256) {
    const float x0 = to_f(X[p]), x1 = to_f(X[a.P + p]), x2 = to_f(X[2 * a.P + p]);
    const float d0 = dG[p], d1 = dG[a.P + p], d2 = dG[2 * a.P + p];
    float o0 = 0.f, o1 = 0.f, o2 = 0.f;
#pragma unroll
    for (int k = 0; k < kKP; ++k) {
      const float y = f[FO_BF + k] + f[FO_W1F + 3 * k] * x0 + f[FO_W1F + 3 * k + 1] * x1 +
                      f[FO_W1F + 3 * k + 2] * x2;
      const float dz = f[FO_W2 + k] * d0 + f[FO_W2 + kKP + k] * d1 + f[FO_W2 + 2 * kKP + k] * d2;
      const float dy = y > 0.f ? dz : slope * dz;
      const float h = f[FO_W1 + 3 * k] * x0 + f[FO_W1 + 3 * k + 1] * x1 + f[FO_W1 + 3 * k + 2] * x2;
      const float hn = (h - f[FO_M + k]) * f[FO_RSTD + k];
      const float dh =
          lam * dy + f[FO_CDH + k] * (dy - f[FO_MDY + k] - hn * f[FO_MDYHN + k]);
      o0 += f[FO_W1 + 3 * k] * dh;
      o1 += f[FO_W1 + 3 * k + 1] * dh;
      o2 += f[FO_W1 + 3 * k + 2] * dh;
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
  hipLaunchKernelGGL(guide_fold_kernel, dim3(1), dim3(64), 0, s, f);
  prof_end(s);
  return hipGetLastError();
}

template <typename T>
hipError_t guided_map(const Plan& p, const void* x, float* G, long long P, int chunks,
                      const float* fold, hipStream_t s) {
  MapArgs m{x, G, P, p.c_in, p.c, fold};
  prof_begin("gf_guide_map", s);
  if (p.gmode == GF_GUIDE_GREY)
    hipLaunchKernelGGL((guide_map_kernel<T, GF_GUIDE_GREY>), dim3(chunks * 4, p.n), dim3(256), 0,
                       s, m);
  else
    hipLaunchKernelGGL((guide_map_kernel<T, GF_GUIDE_TRANSFORM>), dim3(chunks * 4, p.n),
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
  e = guided_map<T>(p, f.I_lo, Gl, (long long)p.h * p.w, p.g_chunks_lo, fold, s);
  if (e != hipSuccess) return e;
  e = guided_map<T>(p, f.I_hi, Gh, (long long)p.H * p.W, p.g_chunks_hi, fold + kFoldFloats, s);
  if (e != hipSuccess) return e;
  float* abar = reinterpret_cast<float*>(f.ws + p.off_abar);
  float* bbar = reinterpret_cast<float*>(f.ws + p.off_bbar);
  e = launch_coef<float, T>(p, Gl, f.p_lo, f.eps, f.eps_count, abar, bbar, s);
  if (e != hipSuccess) return e;
  return launch_apply<float, T>(p, Gh, f.q, abar, bbar, s);
}

template <typename T>
hipError_t guided_input_grad(const Plan& p, const void* x, const float* dG, void* dx, bool lo,
                             float* part, const float* fold, hipStream_t s) {
  const long long P = lo ? (long long)p.h * p.w : (long long)p.H * p.W;
  const int chunks = lo ? p.g_chunks_lo : p.g_chunks_hi;
  GBwdArgs g{x, dG, dx, part, P, p.c_in, p.c, fold};
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

template <typename T>
hipError_t backward_guided_t(const Plan& p, const BwdArgs& b, hipStream_t s) {
  hipError_t e = guided_prepare<T>(p, b.I_lo, b.I_hi, b.ws, true, s);
  if (e != hipSuccess) return e;
  float* fold = reinterpret_cast<float*>(b.ws + p.off_fold);
  float* Gl = reinterpret_cast<float*>(b.ws + p.off_gl);
  float* Gh = reinterpret_cast<float*>(b.ws + p.off_gh);
  float* dGl = reinterpret_cast<float*>(b.ws + p.off_dgl);
  float* dGh = reinterpret_cast<float*>(b.ws + p.off_dgh);
  e = guided_map<T>(p, b.I_lo, Gl, (long long)p.h * p.w, p.g_chunks_lo, fold, s);
  if (e != hipSuccess) return e;
  e = guided_map<T>(p, b.I_hi, Gh, (long long)p.H * p.W, p.g_chunks_hi, fold + kFoldFloats, s);
  if (e != hipSuccess) return e;
  float* abar = reinterpret_cast<float*>(b.ws + p.off_abar);
  float* U = reinterpret_cast<float*>(b.ws + p.off_u);
  e = launch_coef<float, T>(p, Gl, b.p_lo, b.eps, b.eps_count, abar, nullptr, s);
  if (e != hipSuccess) return e;
  // dG_h = dq * A_h (the guide gradient at high resolution) and the
  // transposed-bilinear partial planes
  e = launch_bwd_hi<float, T, float>(p, Gh, b.dq, dGh, abar, U, s);
  if (e != hipSuccess) return e;
  float* epart = reinterpret_cast<float*>(b.ws + p.off_eps);
  e = launch_bwd_lo<float, T>(p, Gl, b.p_lo, b.eps, b.eps_count, U, dGl, b.dp_lo, epart, s);
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
                 p.c_in, p.c, fold + call * kFoldFloats};
      prof_begin("gf_guide_bwd", s);
      hipLaunchKernelGGL((guide_bwd_kernel<T, float, GF_GUIDE_TRANSFORM>), dim3(chunks, p.n),
                         dim3(256), 0, s, g);
      prof_end(s);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      prof_begin("gf_guide_acc_reduce", s);
      hipLaunchKernelGGL(guide_acc_reduce_kernel, dim3(1), dim3(256), 0, s,
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
    e = guided_input_grad<T>(p, b.I_lo, dGl, b.dI_lo, true, nullptr, fold, s);
    if (e != hipSuccess) return e;
  }
  if (b.dI_hi) {
    e = guided_input_grad<T>(p, b.I_hi, dGh, b.dI_hi, false, nullptr, fold + kFoldFloats, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace gf
