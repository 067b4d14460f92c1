#pragma once
// The convolutional guided filtering layer (Sec. III-E; the layer of the
// DGF_b^c variant, Sec. IV-B).  The box filter f_mu becomes a learned 3x3
// depthwise convolution with dilation r, normalised by its response to the
// ones image (f_d), and the local linear model A = cov / (var + eps) a
// bias-free pointwise block 2c -> K -> K -> c with leaky ReLU applied to the
// per-pixel (cov, var) of all channels; eps is gone.  Everything else is
// the layer of Sec. III-B/C: b = mean_p - A mean_I, the window means of A and
// b (f_d again), bilinear upsampling and q = A_h I_h + b_h, so the high-res
// passes are the library's existing kernels (Abar, bbar planes in, partial
// planes of dAbar, dbbar out).
//
// Low resolution, one thread per pixel (the block couples the channels, so
// a thread holds every channel of its pixel); the 9 taps of every f_d come
// from L1/L2, the parameters from LDS:
//   conv_stats_kernel       mean_I, mean_p, cov, var (two-pass over the 9
//                           weighted taps), the block, A and b
//   conv_fd_ab_kernel       Abar = f_d(A), bbar = f_d(b)
//   conv_collapse_kernel    dense dAbar, dbbar from the partial planes
//   conv_fdT_ab_kernel      dA, db through the window means (transposed f_d
//                           as a 9-tap gather) and those uses' weight terms
//   conv_bwd_block_kernel   b's adjoint, the block's backward, the adjoint
//                           inputs of the statistics, and the pixel sums of
//                           the parameter gradients (the weight products on
//                           the matrix cores, 4 pixels per instruction)
//   conv_inputs_grad_kernel dI_l, dp_l: transposed statistics as a gather
//   conv_param_reduce_kernel  fixed-order totals of the partial sums
// No atomics; every sum runs in a fixed order (bitwise reproducible).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_internal.h"

namespace gf {
namespace {

constexpr int kConvParamMax = conv_param_count(kConvMaxC, kConvMaxK);

__device__ __forceinline__ float lrelu_f(float y, float s) { return y > 0.f ? y : s * y; }
__device__ __forceinline__ float lrelu_df(float y, float s) { return y > 0.f ? 1.f : s; }

// Tap t (0..8, row-major over (dy, dx) in {-1, 0, 1}^2) of pixel (i, j) at
// dilation r: its flat index in `o`, and whether it lies in the image.
__device__ __forceinline__ bool conv_tap(int i, int j, int t, int r, int h, int w, int& o) {
  const int u = i + (t / 3 - 1) * r, v = j + (t % 3 - 1) * r;
  o = u * w + v;
  return (unsigned)u < (unsigned)h && (unsigned)v < (unsigned)w;
}

// f_d's normaliser at (i, j): the in-image taps' weights summed.
__device__ __forceinline__ float conv_norm(const float* Dk, int i, int j, int r, int h, int w) {
  float N = 0.f;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    int o;
    N += conv_tap(i, j, t, r, h, w, o) ? Dk[t] : 0.f;
  }
  return N;
}

__device__ __forceinline__ void load_params(const ConvArgs& a, float* prm) {
  for (int e = threadIdx.x; e < a.nparam; e += blockDim.x) prm[e] = a.params[e];
  __syncthreads();
}

// The pointwise block at one pixel.
__device__ __forceinline__ void conv_block(const float* W1, const float* W2, const float* W3,
                                           int c, int K, float slope, const float* u,
                                           float* y1, float* z1, float* y2, float* z2,
                                           float* A) {
#pragma unroll
  for (int q = 0; q < kConvMaxK; ++q) {
    float s = 0.f;
    if (q < K) {
#pragma unroll
      for (int e = 0; e < 2 * kConvMaxC; ++e)
        if (e < 2 * c) s += W1[q * 2 * c + e] * u[e];
    }
    y1[q] = s;
    z1[q] = lrelu_f(s, slope);
  }
#pragma unroll
  for (int q = 0; q < kConvMaxK; ++q) {
    float s = 0.f;
    if (q < K) {
#pragma unroll
      for (int e = 0; e < kConvMaxK; ++e)
        if (e < K) s += W2[q * K + e] * z1[e];
    }
    y2[q] = s;
    z2[q] = lrelu_f(s, slope);
  }
#pragma unroll
  for (int k = 0; k < kConvMaxC; ++k) {
    float s = 0.f;
    if (k < c) {
#pragma unroll
      for (int e = 0; e < kConvMaxK; ++e)
        if (e < K) s += W3[k * K + e] * z2[e];
    }
    A[k] = s;
  }
}

// Statistics, block, A and b of every low-res pixel (all channels).  With
// a.mI set (backward) the statistics are kept for the adjoint.
template <typename T>
__global__ __launch_bounds__(256) void conv_stats_kernel(ConvArgs a) {
  __shared__ float prm[kConvParamMax];
  load_params(a, prm);
  const int h = a.h, w = a.w, c = a.c, r = a.r;
  // pixel indices in 32 bits (the planner keeps n h w below 2^31)
  const unsigned P = (unsigned)h * (unsigned)w;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (unsigned)a.n * P) return;
  const int b = (int)(t / P);
  const int m = (int)(t - (unsigned)b * P);
  const int i = m / w, j = m - (m / w) * w;
  const float* W1 = prm + 9 * c;
  const float* W2 = W1 + 2 * c * a.K;
  const float* W3 = W2 + a.K * a.K;
  // u = (cov_0 .. cov_{c-1}, var_0 .. var_{c-1}): cleared before the
  // channel loop writes it
  float u[2 * kConvMaxC], mi[kConvMaxC], mp[kConvMaxC];
#pragma unroll
  for (int e = 0; e < 2 * kConvMaxC; ++e) u[e] = 0.f;
#pragma unroll
  for (int k = 0; k < kConvMaxC; ++k) {
    mi[k] = mp[k] = 0.f;
    if (k >= c) continue;
    const size_t pofs = (size_t)(b * c + k) * P;
    const T* Ik = reinterpret_cast<const T*>(a.I_lo) + pofs;
    const T* pk = reinterpret_cast<const T*>(a.p_lo) + pofs;
    const float* Dk = prm + 9 * k;
    float xi[9], xp[9], wt[9], N = 0.f, si = 0.f, sp = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      int o;
      const bool in = conv_tap(i, j, q, r, h, w, o);
      wt[q] = in ? Dk[q] : 0.f;
      xi[q] = in ? to_f(Ik[o]) : 0.f;
      xp[q] = in ? to_f(pk[o]) : 0.f;
      N += wt[q];
      si += wt[q] * xi[q];
      sp += wt[q] * xp[q];
    }
    const float mI = si / N, mP = sp / N;
    float sv = 0.f, sc = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float di = xi[q] - mI;
      sv += wt[q] * di * di;
      sc += wt[q] * di * (xp[q] - mP);
    }
    mi[k] = mI;
    mp[k] = mP;
    u[k] = sc / N;
    u[c + k] = sv / N;
    if (a.mI) {
      a.mI[pofs + m] = mI;
      a.mP[pofs + m] = mP;
      a.cov[pofs + m] = sc / N;
      a.var[pofs + m] = sv / N;
    }
  }
  float y1[kConvMaxK], z1[kConvMaxK], y2[kConvMaxK], z2[kConvMaxK], Av[kConvMaxC];
  conv_block(W1, W2, W3, c, a.K, a.slope, u, y1, z1, y2, z2, Av);
#pragma unroll
  for (int k = 0; k < kConvMaxC; ++k) {
    if (k >= c) continue;
    const size_t o = (size_t)(b * c + k) * P + m;
    a.A[o] = Av[k];
    a.B[o] = mp[k] - Av[k] * mi[k];
  }
}

// Abar = f_d(A), bbar = f_d(b): one thread per plane pixel.
__global__ __launch_bounds__(256) void conv_fd_ab_kernel(ConvArgs a) {
  const int h = a.h, w = a.w, c = a.c, r = a.r;
  const unsigned P = (unsigned)h * (unsigned)w;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (unsigned)(a.n * c) * P) return;
  const int plane = (int)(t / P);
  const int m = (int)(t - (unsigned)plane * P);
  const int i = m / w, j = m - (m / w) * w;
  float Dk[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) Dk[q] = a.params[9 * (plane % c) + q];
  const float* A = a.A + (size_t)plane * P;
  const float* B = a.B + (size_t)plane * P;
  float N = 0.f, sa = 0.f, sb = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int o;
    if (conv_tap(i, j, q, r, h, w, o)) {
      N += Dk[q];
      sa += Dk[q] * A[o];
      sb += Dk[q] * B[o];
    }
  }
  a.abar[(size_t)plane * P + m] = sa / N;
  a.bbar[(size_t)plane * P + m] = sb / N;
}

// Dense dAbar, dbbar of each low-res pixel from the high-res backward's
// partial planes: blocks of (bh + 2) x (tw + 2) rows and columns per
// quantity whose border rows and columns overlap the neighbouring blocks'.
__global__ __launch_bounds__(256) void conv_collapse_kernel(ConvArgs a) {
  const int h = a.h, w = a.w;
  const unsigned P = (unsigned)h * (unsigned)w;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (unsigned)(a.n * a.c) * P) return;
  const int plane = (int)(t / P);
  const int m = (int)(t - (unsigned)plane * P);
  const int i = m / w, j = m - (m / w) * w;
  const int bh = a.bh, tw = a.tw, UW = tw + 2;
  const size_t UP = (size_t)(bh + 2) * UW;
  const float* U = a.U + (size_t)plane * a.nby * a.nbx * 2 * UP;
  const int b0 = i / bh, c0 = j / tw;
  int rows[2] = {b0, b0}, cols[2] = {c0, c0};
  int nr = 1, nc = 1;
  if (i - b0 * bh == 0 && b0 > 0) rows[nr++] = b0 - 1;
  else if (i - b0 * bh == bh - 1 && b0 + 1 < a.nby) rows[nr++] = b0 + 1;
  if (j - c0 * tw == 0 && c0 > 0) cols[nc++] = c0 - 1;
  else if (j - c0 * tw == tw - 1 && c0 + 1 < a.nbx) cols[nc++] = c0 + 1;
  float sA = 0.f, sB = 0.f;
  for (int x = 0; x < nr; ++x)
    for (int y = 0; y < nc; ++y) {
      const int br = rows[x], bc = cols[y];
      const size_t o = (size_t)(br * a.nbx + bc) * 2 * UP +
                       (size_t)(i - (br * bh - 1)) * UW + (j - (bc * tw - 1));
      sA += U[o];
      sB += U[o + UP];
    }
  a.dAb[(size_t)plane * P + m] = sA;
  a.dBb[(size_t)plane * P + m] = sB;
}

// Fixed-order sum of 256 threads' values per slot (shuffle tree per wave,
// then the four waves in order); thread 0 gets the totals.
__device__ __forceinline__ void block_sum9(float (&v)[9], float (*red)[4]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    float s = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
  }
}

// Through the window means: dA(m) = sum over the pixels o whose tap q lands
// on m of D[q] / N(o) dAbar(o) (likewise db), and, at each pixel o, the
// weight terms dAbar(o) (A at tap q - Abar(o)) / N(o) (and b's) of those two
// f_d uses, summed per tap over the workgroup's pixels.  Grid: (ab_grid,
// planes), each workgroup strided over its plane.
__global__ __launch_bounds__(256) void conv_fdT_ab_kernel(ConvArgs a) {
  __shared__ float red[9][4];
  const int h = a.h, w = a.w, r = a.r;
  const int plane = blockIdx.y;
  const int P = h * w;
  float Dk[9], Dsum = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    Dk[q] = a.params[9 * (plane % a.c) + q];
    Dsum += Dk[q];
  }
  const size_t pofs = (size_t)plane * P;
  const float *A = a.A + pofs, *B = a.B + pofs, *Ab = a.abar + pofs, *Bb = a.bbar + pofs;
  const float *gA = a.dAb + pofs, *gB = a.dBb + pofs;
  float acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.f;
  for (int m = blockIdx.x * 256 + threadIdx.x; m < P; m += 256 * gridDim.x) {
    const int i = m / w, j = m - (m / w) * w;
    // pixels at least 2r from every border: all windows that touch them are
    // whole, so every normaliser is the sum of the weights
    const bool inner = i >= 2 * r && i < h - 2 * r && j >= 2 * r && j < w - 2 * r;
    float dA = 0.f, dB = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      // the pixel o whose tap q is m
      const int oi = i - (q / 3 - 1) * r, oj = j - (q % 3 - 1) * r;
      if ((unsigned)oi < (unsigned)h && (unsigned)oj < (unsigned)w) {
        const int o = oi * w + oj;
        const float wq = Dk[q] / (inner ? Dsum : conv_norm(Dk, oi, oj, r, h, w));
        dA += wq * gA[o];
        dB += wq * gB[o];
      }
    }
    a.dA[pofs + m] = dA;
    a.dB[pofs + m] = dB;
    const float rN = 1.f / (inner ? Dsum : conv_norm(Dk, i, j, r, h, w));
    const float ga = gA[m] * rN, gb = gB[m] * rN;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      int o;
      if (conv_tap(i, j, q, r, h, w, o)) acc[q] += ga * (A[o] - Ab[m]) + gb * (B[o] - Bb[m]);
    }
  }
  block_sum9(acc, red);
  if (threadIdx.x == 0) {
    float* out = a.partab + ((size_t)plane * a.ab_grid + blockIdx.x) * 9;
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = acc[q];
  }
}

// Per pixel: b = mean_p - A mean_I and the block backward (dA through W3,
// W2, W1 to (dcov, dvar)); the statistics' adjoint inputs (gmI, gmP, gcov,
// gvar: the direct gradients of mean_I, mean_p and of cov, var as whole
// functions of the taps) are stored for conv_inputs_grad_kernel.
//
// The pixel sums of the block's weight gradients are matrix products with
// the pixels as the contraction: dW2 = sum_p dy2_p z1_p^T, dW1 = sum_p dy1_p
// u_p^T, dW3 = sum_p dA_p z2_p^T (16 x 16 at most).  Each wave (one pixel
// per lane) stages a pair of per-pixel vectors in its LDS block (pixel-major,
// 16 floats per pixel) and accumulates them on the matrix cores,
// v_mfma_f32_16x16x4f32 taking 4 pixels per instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], the two operands read from the
// same 64 consecutive floats (no bank conflicts).  The accumulators stay in
// registers across the wave's tiles (lane l, register g holds row
// 4 (l / 16) + g, column l % 16); the 27 weight terms of D are summed per
// lane in registers.  At the end each wave's sums go to an LDS row and the
// workgroup writes the waves' rows summed in wave order.  The hardware's
// accumulation order is fixed, so results are reproducible.
constexpr int kConvWaves = 4;
typedef float conv_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Adds sum over the wave's 64 pixels of a_p b_p^T (16-vectors staged in
// S[0] and S[1], pixel-major) to C.
__device__ __forceinline__ conv_f4 mfma_pixels(const float* S0, const float* S1, int lane,
                                               conv_f4 C) {
#pragma unroll
  for (int g = 0; g < 16; ++g)
    C = __builtin_amdgcn_mfma_f32_16x16x4f32(S0[64 * g + lane], S1[64 * g + lane], C, 0, 0, 0);
  return C;
}

template <typename T>
__global__ __launch_bounds__(64 * kConvWaves) void conv_bwd_block_kernel(ConvArgs a) {
  __shared__ float prm[kConvParamMax];
  __shared__ float stage[kConvWaves][2][64 * 16];
  __shared__ float wacc[kConvWaves][kConvParamMax];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  load_params(a, prm);
  const int h = a.h, w = a.w, c = a.c, r = a.r, K = a.K;
  const long long P = (long long)h * w, total = (long long)a.n * P;
  const float* W1 = prm + 9 * c;
  const float* W2 = W1 + 2 * c * K;
  const float* W3 = W2 + K * K;
  float* S0 = stage[wave][0];
  float* S1 = stage[wave][1];
  conv_f4 C1 = {0.f, 0.f, 0.f, 0.f}, C2 = C1, C3 = C1;
  float dacc[kConvMaxC][9];
#pragma unroll
  for (int k = 0; k < kConvMaxC; ++k)
#pragma unroll
    for (int q = 0; q < 9; ++q) dacc[k][q] = 0.f;
  constexpr int kTile = 64 * kConvWaves;
  const long long tiles = (total + kTile - 1) / kTile;
  for (long long tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const long long t = tile * kTile + threadIdx.x;
    float u[2 * kConvMaxC], dAt[kConvMaxC];
    float y1[kConvMaxK], z1[kConvMaxK], y2[kConvMaxK], z2[kConvMaxK];
    float dy2[kConvMaxK], dy1[kConvMaxK];
#pragma unroll
    for (int e = 0; e < 2 * kConvMaxC; ++e) u[e] = 0.f;
#pragma unroll
    for (int k = 0; k < kConvMaxC; ++k) dAt[k] = 0.f;
#pragma unroll
    for (int e = 0; e < kConvMaxK; ++e) y1[e] = z1[e] = y2[e] = z2[e] = dy1[e] = dy2[e] = 0.f;
    if (t < total) {
      const int b = (int)((unsigned)t / (unsigned)P);
      const int m = (int)((unsigned)t - (unsigned)b * (unsigned)P);
      const int i = m / w, j = m - (m / w) * w;
      float mi[kConvMaxC], mp[kConvMaxC], Ak[kConvMaxC], dBk[kConvMaxC];
#pragma unroll
      for (int k = 0; k < kConvMaxC; ++k) {
        mi[k] = mp[k] = Ak[k] = dBk[k] = 0.f;
        if (k >= c) continue;
        const size_t o = (size_t)(b * c + k) * P + m;
        mi[k] = a.mI[o];
        mp[k] = a.mP[o];
        u[k] = a.cov[o];
        u[c + k] = a.var[o];
        Ak[k] = a.A[o];
        dBk[k] = a.dB[o];
        dAt[k] = a.dA[o] - dBk[k] * mi[k];
        a.gmP[o] = dBk[k];
        a.gmI[o] = -dBk[k] * Ak[k];
      }
      float Ar[kConvMaxC];
      conv_block(W1, W2, W3, c, K, a.slope, u, y1, z1, y2, z2, Ar);
#pragma unroll
      for (int e = 0; e < kConvMaxK; ++e) {
        float sacc = 0.f;
#pragma unroll
        for (int k = 0; k < kConvMaxC; ++k)
          if (k < c && e < K) sacc += W3[k * K + e] * dAt[k];
        dy2[e] = sacc * lrelu_df(y2[e], a.slope);
      }
#pragma unroll
      for (int e = 0; e < kConvMaxK; ++e) {
        float sacc = 0.f;
#pragma unroll
        for (int q = 0; q < kConvMaxK; ++q)
          if (q < K && e < K) sacc += W2[q * K + e] * dy2[q];
        dy1[e] = sacc * lrelu_df(y1[e], a.slope);
      }
      float du[2 * kConvMaxC];
#pragma unroll
      for (int e = 0; e < 2 * kConvMaxC; ++e) {
        float sacc = 0.f;
#pragma unroll
        for (int q = 0; q < kConvMaxK; ++q)
          if (q < K && e < 2 * c) sacc += W1[q * 2 * c + e] * dy1[q];
        du[e] = sacc;
      }
      // the statistics' weight terms at this pixel, per channel and tap
#pragma unroll
      for (int k = 0; k < kConvMaxC; ++k) {
        if (k >= c) continue;
        const size_t pofs = (size_t)(b * c + k) * P;
        const float dcov = du[k], dvar = du[c + k];
        a.gcov[pofs + m] = dcov;
        a.gvar[pofs + m] = dvar;
        const T* Ik = reinterpret_cast<const T*>(a.I_lo) + pofs;
        const T* pk = reinterpret_cast<const T*>(a.p_lo) + pofs;
        const float* Dk = prm + 9 * k;
        const float rN = 1.f / conv_norm(Dk, i, j, r, h, w);
        const float gmI = -dBk[k] * Ak[k], gmP = dBk[k];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          int o;
          if (conv_tap(i, j, q, r, h, w, o)) {
            const float di = to_f(Ik[o]) - mi[k], dp = to_f(pk[o]) - mp[k];
            dacc[k][q] += (gmI * di + gmP * dp + dcov * (di * dp - u[k]) +
                           dvar * (di * di - u[c + k])) * rN;
          }
        }
      }
    }
    // the three weight products of the wave's 64 pixels on the matrix
    // cores (pixels past the end contribute zero vectors)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      S0[lane * 16 + e] = dy2[e];
      S1[lane * 16 + e] = z1[e];
    }
    wave_sync();
    C2 = mfma_pixels(S0, S1, lane, C2);
    wave_sync();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      S0[lane * 16 + e] = dy1[e];
      S1[lane * 16 + e] = e < 2 * kConvMaxC ? u[e < 2 * kConvMaxC ? e : 0] : 0.f;
    }
    wave_sync();
    C1 = mfma_pixels(S0, S1, lane, C1);
    wave_sync();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      S0[lane * 16 + e] = e < kConvMaxC ? dAt[e < kConvMaxC ? e : 0] : 0.f;
      S1[lane * 16 + e] = z2[e];
    }
    wave_sync();
    C3 = mfma_pixels(S0, S1, lane, C3);
    wave_sync();
  }
  // this wave's sums into its LDS row: C[4 (lane / 16) + g][lane % 16]
  float* acc = wacc[wave];
  const int oW1 = 9 * c, oW2 = oW1 + 2 * c * K, oW3 = oW2 + K * K;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int row = 4 * (lane >> 4) + g, col = lane & 15;
    if (row < K && col < K) acc[oW2 + row * K + col] = C2[g];
    if (row < K && col < 2 * c) acc[oW1 + row * 2 * c + col] = C1[g];
    if (row < c && col < K) acc[oW3 + row * K + col] = C3[g];
  }
#pragma unroll
  for (int k = 0; k < kConvMaxC; ++k)
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float v = wave_sum(dacc[k][q]);
      if (k < c && lane == 0) acc[9 * k + q] = v;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < a.nparam; e += 64 * kConvWaves) {
    float v = wacc[0][e];
#pragma unroll
    for (int q = 1; q < kConvWaves; ++q) v += wacc[q][e];
    a.part[(size_t)blockIdx.x * a.nparam + e] = v;
  }
}

// dI_l, dp_l: each input pixel m gathers, from the pixels o whose tap q is m,
// a_q(o) = D[q] / N(o) times the derivatives of mean_I, mean_p, cov and var
// of o with respect to that tap.
template <typename T>
__global__ __launch_bounds__(256) void conv_inputs_grad_kernel(ConvArgs a) {
  const int h = a.h, w = a.w, c = a.c, r = a.r;
  const unsigned P = (unsigned)h * (unsigned)w;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (unsigned)(a.n * c) * P) return;
  const int plane = (int)(t / P);
  const int m = (int)(t - (unsigned)plane * P);
  const int i = m / w, j = m - (m / w) * w;
  const size_t pofs = (size_t)plane * P;
  float Dk[9], Dsum = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    Dk[q] = a.params[9 * (plane % c) + q];
    Dsum += Dk[q];
  }
  const bool inner = i >= 2 * r && i < h - 2 * r && j >= 2 * r && j < w - 2 * r;
  const float Im = to_f(reinterpret_cast<const T*>(a.I_lo)[pofs + m]);
  const float pm = to_f(reinterpret_cast<const T*>(a.p_lo)[pofs + m]);
  float dI = 0.f, dp = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int oi = i - (q / 3 - 1) * r, oj = j - (q % 3 - 1) * r;
    if ((unsigned)oi < (unsigned)h && (unsigned)oj < (unsigned)w) {
      const size_t o = pofs + (size_t)oi * w + oj;
      const float aq = Dk[q] / (inner ? Dsum : conv_norm(Dk, oi, oj, r, h, w));
      const float di = Im - a.mI[o], dpp = pm - a.mP[o];
      dI += aq * (a.gmI[o] + a.gcov[o] * dpp + 2.f * a.gvar[o] * di);
      dp += aq * (a.gmP[o] + a.gcov[o] * di);
    }
  }
  if (a.dI_lo) a.dI_lo[pofs + m] = dI;
  if (a.dp_lo) a.dp_lo[pofs + m] = dp;
}

// Totals of the parameter gradients: entry e sums the workgroups' partials
// in order, then (D entries, with the window means) the window-mean
// adjoint's partials image by image.
__global__ __launch_bounds__(256) void conv_param_reduce_kernel(ConvArgs a) {
  __shared__ float red[4];
  const int e = blockIdx.x, tid = threadIdx.x;
  float s = 0.f;
  for (int g = tid; g < a.blk_grid; g += 256) s += a.part[(size_t)g * a.nparam + e];
  if (a.mean_ab && e < 9 * a.c) {
    const int k = e / 9, q = e - (e / 9) * 9;
    const int nab = a.n * a.ab_grid;
    for (int g = tid; g < nab; g += 256) {
      const int b = g / a.ab_grid, gg = g - b * a.ab_grid;
      s += a.partab[(((size_t)b * a.c + k) * a.ab_grid + gg) * 9 + q];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) a.dparams[e] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

template <typename T>
hipError_t conv_forward_t(const ConvPlan& cp, const ConvArgs& a0, const void* I_hi, void* q,
                          char* ws, hipStream_t s) {
  ConvArgs a = a0;
  const long long npix = (long long)a.n * a.h * a.w, nplane = npix * a.c;
  prof_begin("gf_conv_stats", s);
  hipLaunchKernelGGL((conv_stats_kernel<T>), dim3((unsigned)((npix + 255) / 256)), dim3(256), 0,
                     s, a);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.mean_ab) {
    prof_begin("gf_conv_fd_ab", s);
    hipLaunchKernelGGL(conv_fd_ab_kernel, dim3((unsigned)((nplane + 255) / 256)), dim3(256), 0,
                       s, a);
    prof_end(s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  (void)ws;
  return launch_apply<T, T>(cp.p, I_hi, q, a.abar, a.bbar, s);
}

template <typename T>
hipError_t conv_backward_t(const ConvPlan& cp, const ConvArgs& a0, const void* I_hi,
                           const void* dq, void* dI_hi, char* ws, hipStream_t s) {
  ConvArgs a = a0;
  const Plan& p = cp.p;
  const long long npix = (long long)a.n * a.h * a.w, nplane = npix * a.c;
  const unsigned gplane = (unsigned)((nplane + 255) / 256);
  prof_begin("gf_conv_stats", s);
  hipLaunchKernelGGL((conv_stats_kernel<T>), dim3((unsigned)((npix + 255) / 256)), dim3(256), 0,
                     s, a);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.mean_ab) {
    prof_begin("gf_conv_fd_ab", s);
    hipLaunchKernelGGL(conv_fd_ab_kernel, dim3(gplane), dim3(256), 0, s, a);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  float* U = reinterpret_cast<float*>(ws + p.off_u);
  float* V = reinterpret_cast<float*>(ws + p.off_v);
  e = launch_bwd_hi<T, T, T, T>(p, I_hi, dq, dI_hi, a.abar, U, V, s);
  if (e != hipSuccess) return e;
  a.U = U;
  a.bh = p.ubh;
  a.tw = p.tw;
  a.nby = p.nby;
  a.nbx = p.nbx;
  prof_begin("gf_conv_collapse", s);
  hipLaunchKernelGGL(conv_collapse_kernel, dim3(gplane), dim3(256), 0, s, a);
  prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.mean_ab) {
    prof_begin("gf_conv_fdT_ab", s);
    hipLaunchKernelGGL(conv_fdT_ab_kernel, dim3(a.ab_grid, a.n * a.c), dim3(256), 0, s, a);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  prof_begin("gf_conv_bwd_block", s);
  hipLaunchKernelGGL((conv_bwd_block_kernel<T>), dim3(a.blk_grid), dim3(64 * kConvWaves), 0, s,
                     a);
  prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.dI_lo || a.dp_lo) {
    prof_begin("gf_conv_inputs_grad", s);
    hipLaunchKernelGGL((conv_inputs_grad_kernel<T>), dim3(gplane), dim3(256), 0, s, a);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (a.dparams) {
    prof_begin("gf_conv_param_reduce", s);
    hipLaunchKernelGGL(conv_param_reduce_kernel, dim3(a.nparam), dim3(256), 0, s, a);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gf
