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

// The same with the tap's row and column clamped into the image, so that
// `o` is always a valid index (loads need no branch; the caller masks).
__device__ __forceinline__ bool conv_tap_clamped(int i, int j, int t, int r, int h, int w,
                                                 int& o) {
  const int u = i + (t / 3 - 1) * r, v = j + (t % 3 - 1) * r;
  o = min(max(u, 0), h - 1) * w + min(max(v, 0), w - 1);
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

// The block's weights and the taps' weights in LDS, zero-padded to fixed
// shapes so that every loop over them has compile-time bounds and offsets
// (a padded weight multiplies a zero input or yields an unused zero):
// W1 [16][8] (inputs cov_0..c-1, var_0..c-1, then zeros), W2 [16][16],
// W3 [4][16], D [4][9].
struct ConvW {
  float w1[kConvMaxK][2 * kConvMaxC];
  float w2[kConvMaxK][kConvMaxK];
  float w3[kConvMaxC][kConvMaxK];
  float d[kConvMaxC][9];
};
constexpr int kConvWFloats = (int)(sizeof(ConvW) / sizeof(float));

__device__ __forceinline__ void load_conv_w(const ConvArgs& a, ConvW& W) {
  const int c = a.c, K = a.K;
  const float* W1 = a.params + 9 * c;
  const float* W2 = W1 + 2 * c * K;
  const float* W3 = W2 + K * K;
  float* f = reinterpret_cast<float*>(&W);
  constexpr int n1 = kConvMaxK * 2 * kConvMaxC, n2 = n1 + kConvMaxK * kConvMaxK,
                n3 = n2 + kConvMaxC * kConvMaxK;
  for (int e = threadIdx.x; e < kConvWFloats; e += blockDim.x) {
    float v = 0.f;
    if (e < n1) {
      const int q = e / (2 * kConvMaxC), x = e % (2 * kConvMaxC);
      if (q < K && x < 2 * c) v = W1[q * 2 * c + x];
    } else if (e < n2) {
      const int q = (e - n1) / kConvMaxK, x = (e - n1) % kConvMaxK;
      if (q < K && x < K) v = W2[q * K + x];
    } else if (e < n3) {
      const int k = (e - n2) / kConvMaxK, x = (e - n2) % kConvMaxK;
      if (k < c && x < K) v = W3[k * K + x];
    } else {
      const int k = (e - n3) / 9, t = (e - n3) % 9;
      if (k < c) v = a.params[9 * k + t];
    }
    f[e] = v;
  }
  __syncthreads();
}

// The pointwise block at one pixel of C channels from u = (cov_0..C-1,
// var_0..C-1): the hidden activations z1, z2, the leaky-ReLU branches (bit q
// of m1, m2 set where the pre-activation is positive) and A.
template <int C>
__device__ __forceinline__ void conv_block(const ConvW& W, float slope, const float (&u)[2 * C],
                                           float (&z1)[kConvMaxK], float (&z2)[kConvMaxK],
                                           unsigned& m1, unsigned& m2, float (&A)[C]) {
  m1 = m2 = 0u;
#pragma unroll
  for (int q = 0; q < kConvMaxK; ++q) {
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < 2 * C; ++e) s += W.w1[q][e] * u[e];
    z1[q] = lrelu_f(s, slope);
    m1 |= (s > 0.f ? 1u : 0u) << q;
  }
#pragma unroll
  for (int q = 0; q < kConvMaxK; ++q) {
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < kConvMaxK; ++e) s += W.w2[q][e] * z1[e];
    z2[q] = lrelu_f(s, slope);
    m2 |= (s > 0.f ? 1u : 0u) << q;
  }
#pragma unroll
  for (int k = 0; k < C; ++k) {
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < kConvMaxK; ++e) s += W.w3[k][e] * z2[e];
    A[k] = s;
  }
}

// Statistics, block, A and b of every low-res pixel (all channels).  With
// a.mI set (backward) the statistics are kept for the adjoint.
template <typename T, int C>
__global__ __launch_bounds__(256) void conv_stats_kernel(ConvArgs a) {
  __shared__ ConvW W;
  load_conv_w(a, W);
  const int h = a.h, w = a.w, r = a.r;
  // pixel indices in 32 bits (the planner keeps n h w below 2^31)
  const unsigned P = (unsigned)h * (unsigned)w;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (unsigned)a.n * P) return;
  const int b = (int)(t / P);
  const int m = (int)(t - (unsigned)b * P);
  const int i = m / w, j = m - (m / w) * w;
  // u = (cov_0 .. cov_C-1, var_0 .. var_C-1)
  float u[2 * C], mi[C], mp[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const unsigned pofs = (unsigned)(b * C + k) * P;
    const T* Ik = reinterpret_cast<const T*>(a.I_lo) + pofs;
    const T* pk = reinterpret_cast<const T*>(a.p_lo) + pofs;
    float xi[9], xp[9], wt[9], N = 0.f, si = 0.f, sp = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      int o;
      const bool in = conv_tap_clamped(i, j, q, r, h, w, o);
      wt[q] = in ? W.d[k][q] : 0.f;
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
    u[C + k] = sv / N;
    if (a.mI) {
      a.mI[pofs + m] = mI;
      a.mP[pofs + m] = mP;
      a.cov[pofs + m] = u[k];
      a.var[pofs + m] = u[C + k];
    }
  }
  float z1[kConvMaxK], z2[kConvMaxK], Av[C];
  unsigned m1, m2;
  conv_block<C>(W, a.slope, u, z1, z2, m1, m2, Av);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const unsigned o = (unsigned)(b * C + k) * P + m;
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
  float Dk[9], Dsum = 0.f, wi[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    Dk[q] = a.params[9 * (plane % a.c) + q];
    Dsum += Dk[q];
  }
  // interior pixels' tap weights D[q] / N (N the sum of the weights)
  const float rDsum = 1.f / Dsum;
#pragma unroll
  for (int q = 0; q < 9; ++q) wi[q] = Dk[q] / Dsum;
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
    if (inner) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        // the pixel o whose tap q is m
        const int o = m - (q / 3 - 1) * r * w - (q % 3 - 1) * r;
        dA += wi[q] * gA[o];
        dB += wi[q] * gB[o];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int oi = i - (q / 3 - 1) * r, oj = j - (q % 3 - 1) * r;
        if ((unsigned)oi < (unsigned)h && (unsigned)oj < (unsigned)w) {
          const int o = oi * w + oj;
          const float wq = Dk[q] / conv_norm(Dk, oi, oj, r, h, w);
          dA += wq * gA[o];
          dB += wq * gB[o];
        }
      }
    }
    a.dA[pofs + m] = dA;
    a.dB[pofs + m] = dB;
    const float rN = inner ? rDsum : 1.f / conv_norm(Dk, i, j, r, h, w);
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

// Stages this lane's pixel vectors x, y (16 each) pixel-major in the wave's
// LDS block and adds the wave's sum of x y^T to C.
__device__ __forceinline__ conv_f4 stage_mfma(float* S0, float* S1, int lane,
                                              const float (&x)[16], const float (&y)[16],
                                              conv_f4 C) {
#pragma unroll
  for (int e = 0; e < 16; e += 4) {
    *reinterpret_cast<float4*>(S0 + lane * 16 + e) = make_float4(x[e], x[e + 1], x[e + 2], x[e + 3]);
    *reinterpret_cast<float4*>(S1 + lane * 16 + e) = make_float4(y[e], y[e + 1], y[e + 2], y[e + 3]);
  }
  wave_sync();
  C = mfma_pixels(S0, S1, lane, C);
  wave_sync();
  return C;
}

template <typename T, int C>
__global__ __launch_bounds__(64 * kConvWaves, 2) void conv_bwd_block_kernel(ConvArgs a) {
  __shared__ ConvW W;
  __shared__ __align__(16) float stage[kConvWaves][2][64 * 16];
  static_assert(kConvParamMax <= 2 * 64 * 16, "a wave's sums fit its staging block");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  load_conv_w(a, W);
  const int h = a.h, w = a.w, r = a.r, K = a.K;
  const unsigned P = (unsigned)h * (unsigned)w, total = (unsigned)a.n * P;
  float* S0 = stage[wave][0];
  float* S1 = stage[wave][1];
  const float slope = a.slope;
  conv_f4 C1 = {0.f, 0.f, 0.f, 0.f}, C2 = C1, C3 = C1;
  float dacc[C][9];
#pragma unroll
  for (int k = 0; k < C; ++k)
#pragma unroll
    for (int q = 0; q < 9; ++q) dacc[k][q] = 0.f;
  constexpr unsigned kTile = 64 * kConvWaves;
  const unsigned tiles = (total + kTile - 1) / kTile;
  for (unsigned tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const unsigned t = tile * kTile + threadIdx.x;
    const bool live = t < total;
    // pixels past the end run on zero vectors and contribute nothing
    const unsigned tt = live ? t : 0u;
    const int b = (int)(tt / P);
    const int m = (int)(tt - (unsigned)b * P);
    const int i = m / w, j = m - (m / w) * w;
    float u[2 * C], dAt[C], mi[C], mp[C], Ak[C], dBk[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const unsigned o = (unsigned)(b * C + k) * P + m;
      mi[k] = live ? a.mI[o] : 0.f;
      mp[k] = live ? a.mP[o] : 0.f;
      u[k] = live ? a.cov[o] : 0.f;
      u[C + k] = live ? a.var[o] : 0.f;
      Ak[k] = live ? a.A[o] : 0.f;
      dBk[k] = live ? a.dB[o] : 0.f;
      dAt[k] = live ? a.dA[o] - dBk[k] * mi[k] : 0.f;
      if (live) {
        a.gmP[o] = dBk[k];
        a.gmI[o] = -dBk[k] * Ak[k];
      }
    }
    float z1[kConvMaxK], z2[kConvMaxK], Ar[C];
    unsigned m1, m2;
    conv_block<C>(W, slope, u, z1, z2, m1, m2, Ar);
    (void)Ar;  // A as stored by the statistics pass is the one used
    float dy[kConvMaxK];
#pragma unroll
    for (int e = 0; e < kConvMaxK; ++e) {
      float sacc = 0.f;
#pragma unroll
      for (int k = 0; k < C; ++k) sacc += W.w3[k][e] * dAt[k];
      dy[e] = ((m2 >> e) & 1u) ? sacc : slope * sacc;
    }
    C2 = stage_mfma(S0, S1, lane, dy, z1, C2);  // dW2 += dy2 z1^T
    float dy1[kConvMaxK];
#pragma unroll
    for (int e = 0; e < kConvMaxK; ++e) {
      float sacc = 0.f;
#pragma unroll
      for (int q = 0; q < kConvMaxK; ++q) sacc += W.w2[q][e] * dy[q];
      dy1[e] = ((m1 >> e) & 1u) ? sacc : slope * sacc;
    }
    {
      float u16[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) u16[e] = e < 2 * C ? u[e < 2 * C ? e : 0] : 0.f;
      C1 = stage_mfma(S0, S1, lane, dy1, u16, C1);  // dW1 += dy1 u^T
    }
    {
      float a16[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) a16[e] = e < C ? dAt[e < C ? e : 0] : 0.f;
      C3 = stage_mfma(S0, S1, lane, a16, z2, C3);  // dW3 += dA z2^T
    }
    float du[2 * C];
#pragma unroll
    for (int e = 0; e < 2 * C; ++e) {
      float sacc = 0.f;
#pragma unroll
      for (int q = 0; q < kConvMaxK; ++q) sacc += W.w1[q][e] * dy1[q];
      du[e] = sacc;
    }
    if (!live) continue;
    // the statistics' weight terms at this pixel, per channel and tap
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const unsigned pofs = (unsigned)(b * C + k) * P;
      const float dcov = du[k], dvar = du[C + k];
      a.gcov[pofs + m] = dcov;
      a.gvar[pofs + m] = dvar;
      const T* Ik = reinterpret_cast<const T*>(a.I_lo) + pofs;
      const T* pk = reinterpret_cast<const T*>(a.p_lo) + pofs;
      // all 18 tap loads first (clamped, unconditional), then the terms
      float xi[9], xp[9], in[9], N = 0.f;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        int o;
        in[q] = conv_tap_clamped(i, j, q, r, h, w, o) ? 1.f : 0.f;
        xi[q] = to_f(Ik[o]);
        xp[q] = to_f(pk[o]);
        N += in[q] * W.d[k][q];
      }
      const float rN = 1.f / N;
      const float gmI = -dBk[k] * Ak[k], gmP = dBk[k];
      const float cu = u[k], vu = u[C + k];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const float di = xi[q] - mi[k], dp = xp[q] - mp[k];
        dacc[k][q] += in[q] * ((gmI * di + gmP * dp + dcov * (di * dp - cu) +
                                dvar * (di * di - vu)) * rN);
      }
    }
  }
  // this wave's sums into its own staging block (the other waves may still
  // be reading theirs): C[4 (lane / 16) + g][lane % 16]
  float* acc = S0;
  constexpr int oW1 = 9 * C;
  const int oW2 = oW1 + 2 * C * K, oW3 = oW2 + K * K;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int row = 4 * (lane >> 4) + g, col = lane & 15;
    if (row < K && col < K) acc[oW2 + row * K + col] = C2[g];
    if (row < K && col < 2 * C) acc[oW1 + row * 2 * C + col] = C1[g];
    if (row < C && col < K) acc[oW3 + row * K + col] = C3[g];
  }
#pragma unroll
  for (int k = 0; k < C; ++k)
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float v = wave_sum(dacc[k][q]);
      if (lane == 0) acc[9 * k + q] = v;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < a.nparam; e += 64 * kConvWaves) {
    float v = stage[0][0][e];
#pragma unroll
    for (int q = 1; q < kConvWaves; ++q) v += stage[q][0][e];
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
  const unsigned pofs = (unsigned)plane * P;
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
  auto gather = [&](unsigned o, float aq) __attribute__((always_inline)) {
    const float di = Im - a.mI[o], dpp = pm - a.mP[o];
    dI += aq * (a.gmI[o] + a.gcov[o] * dpp + 2.f * a.gvar[o] * di);
    dp += aq * (a.gmP[o] + a.gcov[o] * di);
  };
  if (inner) {  // every window touching m is whole: N = the weights' sum
#pragma unroll
    for (int q = 0; q < 9; ++q)
      gather(pofs + m - (q / 3 - 1) * r * w - (q % 3 - 1) * r, Dk[q] / Dsum);
  } else {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int oi = i - (q / 3 - 1) * r, oj = j - (q % 3 - 1) * r;
      if ((unsigned)oi < (unsigned)h && (unsigned)oj < (unsigned)w)
        gather(pofs + (unsigned)(oi * w + oj), Dk[q] / conv_norm(Dk, oi, oj, r, h, w));
    }
  }
  if (a.dI_lo) a.dI_lo[pofs + m] = dI;
  if (a.dp_lo) a.dp_lo[pofs + m] = dp;
}

// ------------------------------------------------------------ LDS-tiled gathers
//
// The window means and the inputs' gradients over output tiles of kCTH x kCTW
// pixels of one plane: the workgroup first stages the tile of each input
// plane with a halo of r rows and columns (zero outside the image) in LDS with
// coalesced row loads, then every thread takes its kCTH / 4 pixels of one
// column, reading the 9 taps from LDS.  Used up to dilation kConvTileMaxR (the
// LDS of six staged planes stays within 64 KB); the per-pixel kernels above
// take larger dilations.  The arithmetic and its order are those of the
// per-pixel kernels.  (The statistics and the window-mean adjoint stay per
// pixel: their longer per-pixel arithmetic gains less from shared loads than
// the LDS costs them in occupancy.)
// Tiles of 16 x 64 low-res pixels, up to dilation kConvTileMaxR (six staged
// planes with their halo stay within 64 KB).
constexpr int kConvTileH = 16, kConvTileW = 64, kConvTileMaxR = 8;
constexpr size_t conv_tile_lds(int r, int planes) {
  return (size_t)planes * (kConvTileH + 2 * r) * (kConvTileW + 2 * r) * sizeof(float);
}
constexpr int kCTH = kConvTileH, kCTW = kConvTileW;

// Stages the tiles of NP planes: every thread first issues all its loads (at
// most kStageIt rows x 2 columns per plane, addresses clamped into the image
// so that no load sits behind a branch), then writes them to LDS; zero
// outside the image.  Src(k, offset) reads plane k.
constexpr int kStageIt = (kCTH + 2 * kConvTileMaxR + 3) / 4;

template <int NP, typename Src>
__device__ __forceinline__ void conv_stage_n(Src src, int h, int w, int i0, int j0, int r,
                                             float* L, int LN) {
  const int LW = kCTW + 2 * r, LH = kCTH + 2 * r;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // rows of this wave (ty is the wave's index: a wave-uniform bound) and
  // whether this lane also holds a column of the second pass (the halo)
  const int nit = (LH - ty + 3) / 4;
  const bool col2 = tx + 64 < LW;
  float v[NP][kStageIt][2];
#pragma unroll
  for (int it = 0; it < kStageIt; ++it) {
    if (it >= nit) break;
    const int li = ty + 4 * it, i = i0 - r + li;
    const int ic = min(max(i, 0), h - 1);
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      if (c2 == 1 && !col2) continue;
      const int lj = tx + 64 * c2, j = j0 - r + lj;
      const int jc = min(max(j, 0), w - 1);
      const bool ok = (unsigned)i < (unsigned)h && (unsigned)j < (unsigned)w;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const float x = src(k, (size_t)ic * w + jc);
        v[k][it][c2] = ok ? x : 0.f;
      }
    }
  }
#pragma unroll
  for (int it = 0; it < kStageIt; ++it) {
    if (it >= nit) break;
    const int li = ty + 4 * it;
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      if (c2 == 1 && !col2) continue;
      const int lj = tx + 64 * c2;
#pragma unroll
      for (int k = 0; k < NP; ++k) L[k * LN + li * LW + lj] = v[k][it][c2];
    }
  }
}

// Abar = f_d(A), bbar = f_d(b).  Grid: (tiles across, tiles down, planes).
__global__ __launch_bounds__(256) void conv_fd_ab_tiled_kernel(ConvArgs a) {
  extern __shared__ float ctl[];
  const int h = a.h, w = a.w, r = a.r, plane = blockIdx.z;
  const int i0 = blockIdx.y * kCTH, j0 = blockIdx.x * kCTW;
  const int LW = kCTW + 2 * r, LN = LW * (kCTH + 2 * r);
  float* LA = ctl;
  float* LB = ctl + LN;
  const size_t pofs = (size_t)plane * h * w;
  const float *SA = a.A + pofs, *SB = a.B + pofs;
  conv_stage_n<2>([&](int k, size_t o) { return k == 0 ? SA[o] : SB[o]; }, h, w, i0, j0, r, ctl, LN);
  float Dk[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) Dk[q] = a.params[9 * (plane % a.c) + q];
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int j = j0 + tx;
#pragma unroll
  for (int k = 0; k < kCTH / 4; ++k) {
    const int ti = ty * (kCTH / 4) + k, i = i0 + ti;
    if (i >= h || j >= w) continue;
    float N = 0.f, sa = 0.f, sb = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      int o;
      if (conv_tap(i, j, q, r, h, w, o)) {
        const int l = (ti + r + (q / 3 - 1) * r) * LW + (tx + r + (q % 3 - 1) * r);
        N += Dk[q];
        sa += Dk[q] * LA[l];
        sb += Dk[q] * LB[l];
      }
    }
    a.abar[pofs + (size_t)i * w + j] = sa / N;
    a.bbar[pofs + (size_t)i * w + j] = sb / N;
  }
}

// dI_l, dp_l (as conv_inputs_grad_kernel).  Grid: (tiles across, tiles
// down, planes).
template <typename T>
__global__ __launch_bounds__(256) void conv_inputs_grad_tiled_kernel(ConvArgs a) {
  extern __shared__ float ctl[];
  const int h = a.h, w = a.w, r = a.r, plane = blockIdx.z;
  const int i0 = blockIdx.y * kCTH, j0 = blockIdx.x * kCTW;
  const int LW = kCTW + 2 * r, LN = LW * (kCTH + 2 * r);
  float* LmI = ctl;
  float* LmP = ctl + LN;
  float* LgmI = ctl + 2 * LN;
  float* LgmP = ctl + 3 * LN;
  float* Lgc = ctl + 4 * LN;
  float* Lgv = ctl + 5 * LN;
  const size_t pofs = (size_t)plane * h * w;
  const float* src6[6] = {a.mI + pofs,  a.mP + pofs,   a.gmI + pofs,
                          a.gmP + pofs, a.gcov + pofs, a.gvar + pofs};
  conv_stage_n<6>([&](int k, size_t o) { return src6[k][o]; }, h, w, i0, j0, r, ctl, LN);
  float Dk[9], Dsum = 0.f;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    Dk[q] = a.params[9 * (plane % a.c) + q];
    Dsum += Dk[q];
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int j = j0 + tx;
#pragma unroll 1
  for (int k = 0; k < kCTH / 4; ++k) {
    const int ti = ty * (kCTH / 4) + k, i = i0 + ti;
    if (i >= h || j >= w) continue;
    const size_t m = (size_t)i * w + j;
    const int lc = (ti + r) * LW + tx + r;
    const bool inner = i >= 2 * r && i < h - 2 * r && j >= 2 * r && j < w - 2 * r;
    const float Im = to_f(reinterpret_cast<const T*>(a.I_lo)[pofs + m]);
    const float pm = to_f(reinterpret_cast<const T*>(a.p_lo)[pofs + m]);
    float dI = 0.f, dp = 0.f;
    auto gather = [&](int l, float aq) __attribute__((always_inline)) {
      const float di = Im - LmI[l], dpp = pm - LmP[l];
      dI += aq * (LgmI[l] + Lgc[l] * dpp + 2.f * Lgv[l] * di);
      dp += aq * (LgmP[l] + Lgc[l] * di);
    };
    if (inner) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        gather(lc - (q / 3 - 1) * r * LW - (q % 3 - 1) * r, Dk[q] / Dsum);
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int oi = i - (q / 3 - 1) * r, oj = j - (q % 3 - 1) * r;
        if ((unsigned)oi < (unsigned)h && (unsigned)oj < (unsigned)w)
          gather(lc - (q / 3 - 1) * r * LW - (q % 3 - 1) * r,
                 Dk[q] / conv_norm(Dk, oi, oj, r, h, w));
      }
    }
    if (a.dI_lo) a.dI_lo[pofs + m] = dI;
    if (a.dp_lo) a.dp_lo[pofs + m] = dp;
  }
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

// One of four instantiations (channel counts 1..4, checked by the planner).
template <typename T>
void launch_conv_c(int c, void (*k1)(ConvArgs), void (*k2)(ConvArgs), void (*k3)(ConvArgs),
                   void (*k4)(ConvArgs), dim3 grid, dim3 block, hipStream_t s,
                   const ConvArgs& a) {
  void (*k)(ConvArgs) = c == 1 ? k1 : c == 2 ? k2 : c == 3 ? k3 : k4;
  hipLaunchKernelGGL(k, grid, block, 0, s, a);
}

// Tiles of the LDS-tiled stencil kernels: (across, down, planes).
inline dim3 conv_tile_grid(const ConvArgs& a) {
  return dim3((unsigned)((a.w + kCTW - 1) / kCTW), (unsigned)((a.h + kCTH - 1) / kCTH),
              (unsigned)(a.n * a.c));
}

// Abar, bbar: the tiled kernel up to kConvTileMaxR, else one thread per pixel.
inline void launch_fd_ab(const ConvArgs& a, hipStream_t s) {
  if (a.r <= kConvTileMaxR) {
    hipLaunchKernelGGL(conv_fd_ab_tiled_kernel, conv_tile_grid(a), dim3(256),
                       conv_tile_lds(a.r, 2), s, a);
  } else {
    const long long nplane = (long long)a.n * a.c * a.h * a.w;
    hipLaunchKernelGGL(conv_fd_ab_kernel, dim3((unsigned)((nplane + 255) / 256)), dim3(256), 0,
                       s, a);
  }
}


}  // namespace

template <typename T>
hipError_t conv_forward_t(const ConvPlan& cp, const ConvArgs& a0, const void* I_hi, void* q,
                          char* ws, hipStream_t s) {
  ConvArgs a = a0;
  const long long npix = (long long)a.n * a.h * a.w;
  prof_begin("gf_conv_stats", s);
  launch_conv_c<T>(a.c, conv_stats_kernel<T, 1>, conv_stats_kernel<T, 2>, conv_stats_kernel<T, 3>,
                   conv_stats_kernel<T, 4>, dim3((unsigned)((npix + 255) / 256)), dim3(256), s, a);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.mean_ab) {
    prof_begin("gf_conv_fd_ab", s);
    launch_fd_ab(a, s);
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
  launch_conv_c<T>(a.c, conv_stats_kernel<T, 1>, conv_stats_kernel<T, 2>, conv_stats_kernel<T, 3>,
                   conv_stats_kernel<T, 4>, dim3((unsigned)((npix + 255) / 256)), dim3(256), s, a);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.mean_ab) {
    prof_begin("gf_conv_fd_ab", s);
    launch_fd_ab(a, s);
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
  launch_conv_c<T>(a.c, conv_bwd_block_kernel<T, 1>, conv_bwd_block_kernel<T, 2>,
                   conv_bwd_block_kernel<T, 3>, conv_bwd_block_kernel<T, 4>, dim3(a.blk_grid),
                   dim3(64 * kConvWaves), s, a);
  prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.dI_lo || a.dp_lo) {
    prof_begin("gf_conv_inputs_grad", s);
    if (a.r <= kConvTileMaxR)
      hipLaunchKernelGGL((conv_inputs_grad_tiled_kernel<T>), conv_tile_grid(a), dim3(256),
                         conv_tile_lds(a.r, 6), s, a);
    else
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
