// HIP kernels of the fast guided filtering layer for gfx950 (MI355X).
//
// Forward (Sec. III-B/C, Eq. (1)-(2)):
//   coef_kernel   low-res tile in LDS: box statistics of the recentred guide
//                 and input, A = cov/(var+eps), b = mean_p - A mean_I, then
//                 their window means; writes Abar, bbar (low-res, fp32).
//   apply_kernel  streams the high-res guide: bilinear Abar/bbar taps are
//                 blended in registers (never stored at high resolution) and
//                 q = A_h G_h + b_h is written with non-temporal stores.
// Backward (Algorithm 1, plus the adjoint of the A/b window mean):
//   coef_kernel   recomputes Abar.
//   bwd_hi_kernel one wave per high-res block: dI_h = dq A_h, and the
//                 transposed bilinear of dq G_h and dq accumulated first
//                 vertically in registers, then horizontally through LDS,
//                 into per-block partial low-res planes (no atomics).
//   bwd_lo_kernel low-res tile: gathers the partial planes, recomputes the
//                 box statistics and runs the adjoint chain; f_mu^T(y) is the
//                 box SUM of y/N.  Writes dI_l, dp_l and per-tile deps partials.
//   eps_reduce_kernel  fixed-order sum of the deps partials.
// All reductions run in a fixed order, so results are bitwise reproducible.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_internal.h"

namespace gf {
namespace {

// ------------------------------------------------------------ element I/O

struct bf16 {
  uint16_t u;
};

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f(bf16 v) { return __uint_as_float((uint32_t)v.u << 16); }

template <typename T>
__device__ __forceinline__ T from_f(float v);
template <>
__device__ __forceinline__ float from_f<float>(float v) {
  return v;
}
template <>
__device__ __forceinline__ _Float16 from_f<_Float16>(float v) {
  return (_Float16)v;
}
template <>
__device__ __forceinline__ bf16 from_f<bf16>(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40u)};
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return bf16{(uint16_t)(u >> 16)};
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int BYTES>
struct Carrier;
template <>
struct Carrier<16> {
  typedef u32x4 type;
};
template <>
struct Carrier<8> {
  typedef u32x2 type;
};
template <>
struct Carrier<4> {
  typedef uint32_t type;
};
template <>
struct Carrier<2> {
  typedef uint16_t type;
};

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T* p, float (&out)[VEC]) {
  typedef typename Carrier<sizeof(T) * VEC>::type C;
  C c = *reinterpret_cast<const C*>(p);
  T t[VEC];
  __builtin_memcpy(t, &c, sizeof(C));
#pragma unroll
  for (int e = 0; e < VEC; ++e) out[e] = to_f(t[e]);
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_nt(T* p, const float (&v)[VEC]) {
  typedef typename Carrier<sizeof(T) * VEC>::type C;
  T t[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) t[e] = from_f<T>(v[e]);
  C c;
  __builtin_memcpy(&c, t, sizeof(C));
  __builtin_nontemporal_store(c, reinterpret_cast<C*>(p));
}

// ------------------------------------------------------------ geometry

// Pixels of the clipped window of radius r around index i on an axis of n.
__device__ __forceinline__ int wcount(int i, int r, int n) {
  return min(n - 1, i + r) - max(0, i - r) + 1;
}

// Half-pixel bilinear taps of high-res index y for an integer factor S over
// a low-res axis of length n: source s = (2y + 1 - S) / (2S), clamped at 0;
// taps floor(s) and floor(s)+1 (clamped to n-1) with weight frac(s).
struct Tap {
  int i0, i1;
  float w;
};
__device__ __forceinline__ Tap tap(int y, int S, int n) {
  Tap t;
  const int num = 2 * y + 1 - S;
  if (num < 0) {
    t.i0 = 0;
    t.i1 = min(1, n - 1);
    t.w = 0.f;
  } else {
    t.i0 = num / (2 * S);
    const int rem = num - t.i0 * 2 * S;
    t.w = (float)rem / (float)(2 * S);
    t.i1 = min(t.i0 + 1, n - 1);
  }
  return t;
}

// ------------------------------------------------------------ window statistics
//
// Mean, variance and covariance over a clipped (2r+1)^2 window, computed in
// two levels so that no step subtracts two large, nearly equal numbers
// (the law of total variance over the window's columns):
//   per column j of the window, over its rows:   cm = mean, cvv = sum (g-cm)^2,
//                                                 cvp = sum (g-cm_g)(p-cm_p)
//   over the window's columns:  mean = avg cm,
//     var = sum cvv / N + avg (cm_g - mean_g)^2,
//     cov = sum cvp / N + avg (cm_g - mean_g)(cm_p - mean_p).
// Only in-image pixels take part; N = rows x columns of the clipped window.

// Column pass: for every (row u of the output region, column v of the
// loaded region) write cm_g, cm_p, cvv, cvp to vt[0..3][u * nc + v].
// `row0` is the image row of output-region row 0, `lrow0`/`lcol0` the image
// row/column of loaded-region row/column 0 (loaded region nc columns wide).
__device__ __forceinline__ void column_stats(const float* sg, const float* sp, float* vt, int nr,
                                             int nc, int row0, int lrow0, int lcol0, int h,
                                             int w, int r) {
  const int V = nr * nc;
  for (int idx = threadIdx.x; idx < V; idx += blockDim.x) {
    const int u = idx / nc, v = idx - u * nc;
    const int gi = row0 + u, gj = lcol0 + v;
    float cg = 0.f, cp = 0.f, vv = 0.f, vp = 0.f;
    if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
      const int t0 = max(gi - r, 0) - lrow0, t1 = min(gi + r, h - 1) - lrow0;
      float s0 = 0.f, s1 = 0.f;
      for (int t = t0; t <= t1; ++t) {
        s0 += sg[t * nc + v];
        s1 += sp[t * nc + v];
      }
      const float inv = 1.f / (float)(t1 - t0 + 1);
      cg = s0 * inv;
      cp = s1 * inv;
      for (int t = t0; t <= t1; ++t) {
        const float dg = sg[t * nc + v] - cg, dp = sp[t * nc + v] - cp;
        vv += dg * dg;
        vp += dg * dp;
      }
    }
    vt[idx] = cg;
    vt[V + idx] = cp;
    vt[2 * V + idx] = vv;
    vt[3 * V + idx] = vp;
  }
}

struct WinStats {
  float mI, mP, var, cov;
};

// Row pass for one output pixel: `base` is the start of its row in the
// column-stat planes (plane stride V), gj its image column, lcol0 the image
// column of loaded column 0, nrow the number of window rows.
__device__ __forceinline__ WinStats window_stats(const float* vt, int V, int base, int gj,
                                                 int lcol0, int w, int r, int nrow) {
  const int c0 = max(gj - r, 0) - lcol0, c1 = min(gj + r, w - 1) - lcol0;
  const float* cmg = vt + base;
  const float* cmp = vt + V + base;
  const float* cvv = vt + 2 * V + base;
  const float* cvp = vt + 3 * V + base;
  float s0 = 0.f, s1 = 0.f;
  for (int c = c0; c <= c1; ++c) {
    s0 += cmg[c];
    s1 += cmp[c];
  }
  const int ncol = c1 - c0 + 1;
  const float invc = 1.f / (float)ncol;
  WinStats st;
  st.mI = s0 * invc;
  st.mP = s1 * invc;
  float bvv = 0.f, bvp = 0.f, wvv = 0.f, wvp = 0.f;
  for (int c = c0; c <= c1; ++c) {
    const float dg = cmg[c] - st.mI, dp = cmp[c] - st.mP;
    bvv += dg * dg;
    bvp += dg * dp;
    wvv += cvv[c];
    wvp += cvp[c];
  }
  const float invN = invc / (float)nrow;
  st.var = wvv * invN + bvv * invc;
  st.cov = wvp * invN + bvp * invc;
  return st;
}

// ------------------------------------------------------------ forward: low-res

struct CoefArgs {
  const void* I_lo;
  const void* p_lo;
  const float* eps;
  int eps_count, c, h, w, r, mean_ab, TH, TW;
  float* abar;  // [planes, h, w]
  float* bbar;  // [planes, h, w] or null
};

// One workgroup per TH x TW low-res output tile of one plane.  The guide and
// input are loaded with a halo of 2r (r when mean_ab == 0), recentred by the
// values at the tile centre (variance and covariance are shift invariant;
// the recentring keeps mean(G^2) - mean(G)^2 from cancelling), box-summed
// separably, turned into A and b on the tile plus a halo of r, and box-meaned
// again.  Pixels outside the image are zero in LDS, and every window mean is
// divided by its in-image count.
template <typename T>
__global__ __launch_bounds__(256) void coef_kernel(CoefArgs a) {
  extern __shared__ float lds[];
  const int plane = blockIdx.z;
  const float e = a.eps[a.eps_count == 1 ? 0 : plane / a.c];
  const int h = a.h, w = a.w, r = a.r, K = 2 * r + 1;
  const int i0 = blockIdx.y * a.TH, j0 = blockIdx.x * a.TW;
  const int hb = a.mean_ab ? r : 0;
  const int hal = hb + r;
  const int nr0 = a.TH + 2 * hal, nc0 = a.TW + 2 * hal;
  const int nr1 = a.TH + 2 * hb, nc1 = a.TW + 2 * hb;
  float* sg = lds;
  float* sp = sg + nr0 * nc0;
  float* vt = sp + nr0 * nc0;  // [4][nr1 * nc0]
  float* sa = vt + 4 * nr1 * nc0;
  float* sb = sa + nr1 * nc1;
  const size_t pofs = (size_t)plane * h * w;
  const T* G = reinterpret_cast<const T*>(a.I_lo) + pofs;
  const T* P = reinterpret_cast<const T*>(a.p_lo) + pofs;
  const int ic = min(i0 + a.TH / 2, h - 1), jc = min(j0 + a.TW / 2, w - 1);
  const float cg = to_f(G[(size_t)ic * w + jc]);
  const float cp = to_f(P[(size_t)ic * w + jc]);

  for (int idx = threadIdx.x; idx < nr0 * nc0; idx += 256) {
    const int u = idx / nc0, v = idx - u * nc0;
    const int gi = i0 - hal + u, gj = j0 - hal + v;
    float g = 0.f, p = 0.f;
    if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
      const size_t o = (size_t)gi * w + gj;
      g = to_f(G[o]) - cg;
      p = to_f(P[o]) - cp;
    }
    sg[idx] = g;
    sp[idx] = p;
  }
  __syncthreads();
  const int V1 = nr1 * nc0;
  column_stats(sg, sp, vt, nr1, nc0, i0 - hb, i0 - hal, j0 - hal, h, w, r);
  __syncthreads();
  for (int idx = threadIdx.x; idx < nr1 * nc1; idx += 256) {
    const int u = idx / nc1, v = idx - u * nc1;
    const int gi = i0 - hb + u, gj = j0 - hb + v;
    float A = 0.f, B = 0.f;
    if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
      const WinStats st = window_stats(vt, V1, u * nc0, gj, j0 - hal, w, r, wcount(gi, r, h));
      const float den = st.var + e;
      A = den > 0.f ? st.cov / den : 0.f;
      B = (st.mP + cp) - A * (st.mI + cg);
    }
    sa[idx] = A;
    sb[idx] = B;
  }
  __syncthreads();
  float* Ab = a.abar + pofs;
  float* Bb = a.bbar ? a.bbar + pofs : nullptr;
  if (!a.mean_ab) {
    for (int idx = threadIdx.x; idx < a.TH * a.TW; idx += 256) {
      const int u = idx / a.TW, v = idx - u * a.TW;
      const int gi = i0 + u, gj = j0 + v;
      if (gi < h && gj < w) {
        Ab[(size_t)gi * w + gj] = sa[idx];
        if (Bb) Bb[(size_t)gi * w + gj] = sb[idx];
      }
    }
    return;
  }
  const int V2 = a.TH * nc1;
  for (int idx = threadIdx.x; idx < V2; idx += 256) {
    const int u = idx / nc1, v = idx - u * nc1;
    float s0 = 0.f, s1 = 0.f;
    for (int t = 0; t < K; ++t) {
      s0 += sa[(u + t) * nc1 + v];
      s1 += sb[(u + t) * nc1 + v];
    }
    vt[idx] = s0;
    vt[V2 + idx] = s1;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < a.TH * a.TW; idx += 256) {
    const int u = idx / a.TW, v = idx - u * a.TW;
    const int gi = i0 + u, gj = j0 + v;
    if (gi >= h || gj >= w) continue;
    float s0 = 0.f, s1 = 0.f;
    const int base = u * nc1 + v;
    for (int t = 0; t < K; ++t) {
      s0 += vt[base + t];
      s1 += vt[V2 + base + t];
    }
    const float invN = 1.f / (float)(wcount(gi, r, h) * wcount(gj, r, w));
    Ab[(size_t)gi * w + gj] = s0 * invN;
    if (Bb) Bb[(size_t)gi * w + gj] = s1 * invN;
  }
}

// ------------------------------------------------------------ forward: high-res

struct ApplyArgs {
  const void* I_hi;
  void* q;
  const float* abar;
  const float* bbar;
  int h, w, H, W, RB, nrb, nxv;
  long long total;
};

// Horizontally interpolated low-res row `i` (clamped) at the VEC columns of
// this thread.
template <int VEC>
__device__ __forceinline__ void hrow(const float* L, int i, int h, int w, const int (&j0)[VEC],
                                     const int (&j1)[VEC], const float (&wx)[VEC],
                                     float (&out)[VEC]) {
  i = min(max(i, 0), h - 1);
  const float* row = L + (size_t)i * w;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const float a0 = row[j0[e]], a1 = row[j1[e]];
    out[e] = a0 + wx[e] * (a1 - a0);
  }
}

// One thread = VEC adjacent high-res columns x RB rows of one plane.  Rows
// are walked one low-res row block (S rows) at a time; the three low-res
// rows a block touches (i-1, i, i+1, clamped) are kept interpolated in
// registers, so each high-res pixel costs one blend and one FMA.
template <typename T, int S, int VEC>
__global__ __launch_bounds__(256) void apply_kernel(ApplyArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.total) return;
  const int xv = (int)(t % a.nxv);
  const long long rest = t / a.nxv;
  const int rb = (int)(rest % a.nrb);
  const int plane = (int)(rest / a.nrb);
  const int h = a.h, w = a.w, W = a.W;
  const int x0 = xv * VEC;
  int j0[VEC], j1[VEC];
  float wx[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const Tap tx = tap(x0 + e, S, w);
    j0[e] = tx.i0;
    j1[e] = tx.i1;
    wx[e] = tx.w;
  }
  const float* Ab = a.abar + (size_t)plane * h * w;
  const float* Bb = a.bbar + (size_t)plane * h * w;
  const size_t hofs = (size_t)plane * a.H * W + x0;
  const T* Gp = reinterpret_cast<const T*>(a.I_hi) + hofs;
  T* Qp = reinterpret_cast<T*>(a.q) + hofs;
  const int ib0 = rb * (a.RB / S);
  const int ib1 = min(ib0 + a.RB / S, h);
  float am[VEC], ac[VEC], ap[VEC], bm[VEC], bc[VEC], bp[VEC];
  hrow<VEC>(Ab, ib0 - 1, h, w, j0, j1, wx, am);
  hrow<VEC>(Bb, ib0 - 1, h, w, j0, j1, wx, bm);
  hrow<VEC>(Ab, ib0, h, w, j0, j1, wx, ac);
  hrow<VEC>(Bb, ib0, h, w, j0, j1, wx, bc);
  for (int i = ib0; i < ib1; ++i) {
    float g[S][VEC];
#pragma unroll
    for (int t = 0; t < S; ++t) load_vec<T, VEC>(Gp + (size_t)(S * i + t) * W, g[t]);
    hrow<VEC>(Ab, i + 1, h, w, j0, j1, wx, ap);
    hrow<VEC>(Bb, i + 1, h, w, j0, j1, wx, bp);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int num = 2 * t + 1 - S;
      float q[VEC];
      if (num < 0) {
        const float wy = (float)(num + 2 * S) / (float)(2 * S);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float A = am[e] + wy * (ac[e] - am[e]);
          const float B = bm[e] + wy * (bc[e] - bm[e]);
          q[e] = A * g[t][e] + B;
        }
      } else {
        const float wy = (float)num / (float)(2 * S);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float A = ac[e] + wy * (ap[e] - ac[e]);
          const float B = bc[e] + wy * (bp[e] - bc[e]);
          q[e] = A * g[t][e] + B;
        }
      }
      store_vec_nt<T, VEC>(Qp + (size_t)(S * i + t) * W, q);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      am[e] = ac[e];
      ac[e] = ap[e];
      bm[e] = bc[e];
      bc[e] = bp[e];
    }
  }
}

// ------------------------------------------------------------ backward: high-res

struct BwdHiArgs {
  const void* I_hi;
  const void* dq;
  void* dI_hi;  // may be null
  const float* abar;
  float* U;     // per-block partial planes
  int h, w, H, W, bh, tw, nby, nbx;
};

// One wave per block of bh low-res rows (S*bh high-res rows) x 64*VEC
// high-res columns.  The block writes the transposed-bilinear contributions
// of its own pixels to low-res rows i_a-1 .. i_a+bh and columns
// j_a-1 .. j_a+tw: a (bh+2) x (tw+2) partial plane for dA_bar (from dq*G_h)
// and one for db_bar (from dq).  The border rows/columns overlap the
// neighbouring blocks' and are summed by the low-res kernel.
template <typename T, int S, int VEC>
__global__ __launch_bounds__(64) void bwd_hi_kernel(BwdHiArgs a) {
  constexpr int TWH = 64 * VEC;  // high-res columns per block
  __shared__ float sR[2][TWH];
  const int lane = threadIdx.x;
  const int bx = blockIdx.x, by = blockIdx.y, plane = blockIdx.z;
  const int h = a.h, w = a.w, W = a.W, bh = a.bh, tw = a.tw;
  const int X_a = bx * TWH;
  const int x0 = X_a + lane * VEC;
  const bool valid = x0 < W;
  const int j_a = X_a / S;
  const int i_a = by * bh;
  const int i_b = min(i_a + bh, h);
  int j0[VEC], j1[VEC];
  float wx[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const Tap tx = tap(valid ? x0 + e : 0, S, w);
    j0[e] = tx.i0;
    j1[e] = tx.i1;
    wx[e] = tx.w;
  }
  const float* Ab = a.abar + (size_t)plane * h * w;
  const size_t hofs = (size_t)plane * a.H * W + (valid ? x0 : 0);
  const T* Gp = reinterpret_cast<const T*>(a.I_hi) + hofs;
  const T* Dp = reinterpret_cast<const T*>(a.dq) + hofs;
  T* Op = a.dI_hi ? reinterpret_cast<T*>(a.dI_hi) + hofs : nullptr;
  const int UW = tw + 2;
  const size_t UP = (size_t)(bh + 2) * UW;
  float* Ub = a.U + (((size_t)plane * a.nby + by) * a.nbx + bx) * 2 * UP;

  auto flush = [&](const float (&uA)[VEC], const float (&uB)[VEC], int lr) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      sR[0][lane * VEC + e] = uA[e];
      sR[1][lane * VEC + e] = uB[e];
    }
    __syncthreads();
    for (int k = lane; k < UW; k += 64) {
      const int j = j_a - 1 + k;
      float sa = 0.f, sb = 0.f;
      if (j >= 0 && j < w) {
        const int xlo = max(max(S * (j - 1), X_a), 0);
        const int xhi = min(min(S * (j + 2), X_a + TWH), W);
        for (int x = xlo; x < xhi; ++x) {
          const Tap tx = tap(x, S, w);
          const float wt = (tx.i0 == j ? 1.f - tx.w : 0.f) + (tx.i1 == j ? tx.w : 0.f);
          sa += wt * sR[0][x - X_a];
          sb += wt * sR[1][x - X_a];
        }
      }
      Ub[(size_t)lr * UW + k] = sa;
      Ub[UP + (size_t)lr * UW + k] = sb;
    }
    __syncthreads();
  };

  float am[VEC], ac[VEC], ap[VEC];
  float pA[VEC], cA[VEC], nA[VEC], pB[VEC], cB[VEC], nB[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) pA[e] = cA[e] = nA[e] = pB[e] = cB[e] = nB[e] = 0.f;
  hrow<VEC>(Ab, i_a - 1, h, w, j0, j1, wx, am);
  hrow<VEC>(Ab, i_a, h, w, j0, j1, wx, ac);
  for (int i = i_a; i < i_b; ++i) {
    float g[S][VEC], d[S][VEC];
    if (valid) {
#pragma unroll
      for (int t = 0; t < S; ++t) {
        load_vec<T, VEC>(Dp + (size_t)(S * i + t) * W, d[t]);
        load_vec<T, VEC>(Gp + (size_t)(S * i + t) * W, g[t]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < S; ++t)
#pragma unroll
        for (int e = 0; e < VEC; ++e) d[t][e] = g[t][e] = 0.f;
    }
    hrow<VEC>(Ab, i + 1, h, w, j0, j1, wx, ap);
    const bool top = (i == 0), bot = (i == h - 1);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int num = 2 * t + 1 - S;
      float o[VEC];
      if (num < 0) {
        const float wy = (float)(num + 2 * S) / (float)(2 * S);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          o[e] = d[t][e] * (am[e] + wy * (ac[e] - am[e]));
          const float vA = d[t][e] * g[t][e], vB = d[t][e];
          if (top) {
            cA[e] += vA;
            cB[e] += vB;
          } else {
            pA[e] += (1.f - wy) * vA;
            cA[e] += wy * vA;
            pB[e] += (1.f - wy) * vB;
            cB[e] += wy * vB;
          }
        }
      } else {
        const float wy = (float)num / (float)(2 * S);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          o[e] = d[t][e] * (ac[e] + wy * (ap[e] - ac[e]));
          const float vA = d[t][e] * g[t][e], vB = d[t][e];
          if (bot) {
            cA[e] += vA;
            cB[e] += vB;
          } else {
            cA[e] += (1.f - wy) * vA;
            nA[e] += wy * vA;
            cB[e] += (1.f - wy) * vB;
            nB[e] += wy * vB;
          }
        }
      }
      if (Op && valid) store_vec_nt<T, VEC>(Op + (size_t)(S * i + t) * W, o);
    }
    flush(pA, pB, i - i_a);  // low-res row i-1 is complete
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      pA[e] = cA[e];
      cA[e] = nA[e];
      nA[e] = 0.f;
      pB[e] = cB[e];
      cB[e] = nB[e];
      nB[e] = 0.f;
      am[e] = ac[e];
      ac[e] = ap[e];
    }
  }
  flush(pA, pB, i_b - i_a);      // row i_b - 1
  flush(cA, cB, i_b - i_a + 1);  // row i_b (contributions of the last rows)
}

// ------------------------------------------------------------ backward: low-res

struct BwdLoArgs {
  const void* I_lo;
  const void* p_lo;
  const float* eps;
  int eps_count, c;
  const float* U;
  int bh, tw, nby, nbx;
  int h, w, r, mean_ab, TH, TW, ntx, nty;
  float* dI_lo;     // may be null
  float* dp_lo;     // may be null
  float* eps_part;  // [planes][nty * ntx]
};

// Sum of the partial planes that cover low-res pixel (i, j): the block that
// owns it plus, on a block border, the neighbour whose halo row/column it is.
__device__ __forceinline__ void gather_u(const BwdLoArgs& a, int plane, int i, int j, float& uA,
                                         float& uB) {
  const int bh = a.bh, tw = a.tw, UW = tw + 2;
  const size_t UP = (size_t)(bh + 2) * UW;
  const int b0 = i / bh, c0 = j / tw;
  int bys[2] = {b0, -1}, bxs[2] = {c0, -1};
  if (i % bh == 0 && b0 > 0) bys[1] = b0 - 1;
  else if (i % bh == bh - 1 && b0 + 1 < a.nby) bys[1] = b0 + 1;
  if (j % tw == 0 && c0 > 0) bxs[1] = c0 - 1;
  else if (j % tw == tw - 1 && c0 + 1 < a.nbx) bxs[1] = c0 + 1;
  float sA = 0.f, sB = 0.f;
  for (int q = 0; q < 2; ++q) {
    const int by = bys[q];
    if (by < 0) continue;
    for (int s = 0; s < 2; ++s) {
      const int bx = bxs[s];
      if (bx < 0) continue;
      const float* blk = a.U + (((size_t)plane * a.nby + by) * a.nbx + bx) * 2 * UP;
      const size_t o = (size_t)(i - (by * bh - 1)) * UW + (j - (bx * tw - 1));
      sA += blk[o];
      sB += blk[UP + o];
    }
  }
  uA = sA;
  uB = sB;
}

// One workgroup per TH x TW low-res tile.  LDS holds the recentred guide and
// input and the gathered upstream planes on the tile plus a halo of 2r; the
// statistics and the adjoint quantities live on the tile plus a halo of r.
template <typename T>
__global__ __launch_bounds__(256) void bwd_lo_kernel(BwdLoArgs a) {
  extern __shared__ float lds[];
  __shared__ float red[256];
  const int plane = blockIdx.z;
  const float e = a.eps[a.eps_count == 1 ? 0 : plane / a.c];
  const int h = a.h, w = a.w, r = a.r, K = 2 * r + 1;
  const int i0 = blockIdx.y * a.TH, j0 = blockIdx.x * a.TW;
  const int TH = a.TH, TW = a.TW;
  const int nr0 = TH + 4 * r, nc0 = TW + 4 * r;
  const int nr1 = TH + 2 * r, nc1 = TW + 2 * r;
  const int R0 = nr0 * nc0, R1 = nr1 * nc1;
  float* sg = lds;
  float* sp = sg + R0;
  float* su = sp + R0;
  float* sv = su + R0;
  float* vt = sv + R0;      // [6][nr1 * nc0], later [4][TH * nc1]
  float* X = vt + 6 * nr1 * nc0;  // [4][R1]
  const size_t pofs = (size_t)plane * h * w;
  const T* G = reinterpret_cast<const T*>(a.I_lo) + pofs;
  const T* P = reinterpret_cast<const T*>(a.p_lo) + pofs;
  const int ic = min(i0 + TH / 2, h - 1), jc = min(j0 + TW / 2, w - 1);
  const float cg = to_f(G[(size_t)ic * w + jc]);
  const float cp = to_f(P[(size_t)ic * w + jc]);

  for (int idx = threadIdx.x; idx < R0; idx += 256) {
    const int u = idx / nc0, v = idx - u * nc0;
    const int gi = i0 - 2 * r + u, gj = j0 - 2 * r + v;
    float g = 0.f, p = 0.f, uA = 0.f, uB = 0.f;
    if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
      const size_t o = (size_t)gi * w + gj;
      g = to_f(G[o]) - cg;
      p = to_f(P[o]) - cp;
      gather_u(a, plane, gi, gj, uA, uB);
      if (a.mean_ab) {
        const float invN = 1.f / (float)(wcount(gi, r, h) * wcount(gj, r, w));
        uA *= invN;
        uB *= invN;
      }
    }
    sg[idx] = g;
    sp[idx] = p;
    su[idx] = uA;
    sv[idx] = uB;
  }
  __syncthreads();
  const int V1 = nr1 * nc0;
  column_stats(sg, sp, vt, nr1, nc0, i0 - r, i0 - 2 * r, j0 - 2 * r, h, w, r);
  if (a.mean_ab) {  // column sums of the upstream planes (already divided by N)
    for (int idx = threadIdx.x; idx < V1; idx += 256) {
      const int u = idx / nc0, v = idx - u * nc0;
      float s4 = 0.f, s5 = 0.f;
      for (int t = 0; t < K; ++t) {
        s4 += su[(u + t) * nc0 + v];
        s5 += sv[(u + t) * nc0 + v];
      }
      vt[4 * V1 + idx] = s4;
      vt[5 * V1 + idx] = s5;
    }
  }
  __syncthreads();
  float deps_acc = 0.f;
  for (int idx = threadIdx.x; idx < R1; idx += 256) {
    const int u = idx / nc1, v = idx - u * nc1;
    const int gi = i0 - r + u, gj = j0 - r + v;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
    if (gi >= 0 && gi < h && gj >= 0 && gj < w) {
      const int nrow = wcount(gi, r, h);
      const WinStats st = window_stats(vt, V1, u * nc0, gj, j0 - 2 * r, w, r, nrow);
      float s4, s5;
      if (a.mean_ab) {  // dA = f_mu^T(dAbar) = box sum of dAbar / N; same for db
        s4 = 0.f;
        s5 = 0.f;
        const int base = u * nc0 + v;
        for (int t = 0; t < K; ++t) {
          s4 += vt[4 * V1 + base + t];
          s5 += vt[5 * V1 + base + t];
        }
      } else {  // dA, db are the upstream planes themselves
        const int o = (u + r) * nc0 + (v + r);
        s4 = su[o];
        s5 = sv[o];
      }
      const float invN = 1.f / (float)(nrow * wcount(gj, r, w));
      const float mI = st.mI, mP = st.mP;  // recentred means
      const float var = st.var, cov = st.cov;
      const float den = var + e;
      const float A = den > 0.f ? cov / den : 0.f;
      const float dA = s4, db = s5;
      // b = mean_p - A mean_I (actual means), A = cov / (var + eps)
      const float dAt = dA - db * (mI + cg);
      float dcov = 0.f, dvar = 0.f;
      if (den > 0.f) {
        dcov = dAt / den;
        dvar = -dAt * A / den;
      }
      const float dmI = -db * A - dcov * mP - 2.f * dvar * mI;
      const float dmP = db - dcov * mI;
      x0 = dmI * invN;
      x1 = dmP * invN;
      x2 = dcov * invN;
      x3 = dvar * invN;
      if (u >= r && u < r + TH && v >= r && v < r + TW) deps_acc += dvar;
    }
    X[idx] = x0;
    X[R1 + idx] = x1;
    X[2 * R1 + idx] = x2;
    X[3 * R1 + idx] = x3;
  }
  __syncthreads();
  const int V2 = TH * nc1;
  for (int idx = threadIdx.x; idx < V2; idx += 256) {
    const int u = idx / nc1, v = idx - u * nc1;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int t = 0; t < K; ++t) {
      const int o = (u + t) * nc1 + v;
      s0 += X[o];
      s1 += X[R1 + o];
      s2 += X[2 * R1 + o];
      s3 += X[3 * R1 + o];
    }
    vt[idx] = s0;
    vt[V2 + idx] = s1;
    vt[2 * V2 + idx] = s2;
    vt[3 * V2 + idx] = s3;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TH * TW; idx += 256) {
    const int u = idx / TW, v = idx - u * TW;
    const int gi = i0 + u, gj = j0 + v;
    if (gi >= h || gj >= w) continue;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    const int base = u * nc1 + v;
    for (int t = 0; t < K; ++t) {
      s0 += vt[base + t];
      s1 += vt[V2 + base + t];
      s2 += vt[2 * V2 + base + t];
      s3 += vt[3 * V2 + base + t];
    }
    const int o = (u + 2 * r) * nc0 + (v + 2 * r);
    const float g = sg[o], p = sp[o];
    const size_t go = pofs + (size_t)gi * w + gj;
    if (a.dI_lo) a.dI_lo[go] = s0 + 2.f * s3 * g + s2 * p;
    if (a.dp_lo) a.dp_lo[go] = s1 + s2 * g;
  }
  // fixed-order block reduction of the tile's deps contribution
  red[threadIdx.x] = deps_acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    a.eps_part[(size_t)plane * a.ntx * a.nty + blockIdx.y * a.ntx + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void eps_reduce_kernel(const float* part, int per_plane,
                                                          int c, int n, int eps_count,
                                                          float* deps) {
  __shared__ float red[256];
  const int k = blockIdx.x;
  const size_t lo = (size_t)(eps_count == 1 ? 0 : k * c) * per_plane;
  const size_t hi = (size_t)(eps_count == 1 ? n * c : (k + 1) * c) * per_plane;
  float s = 0.f;
  for (size_t q = lo + threadIdx.x; q < hi; q += 256) s += part[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) deps[k] = red[0];
}

// ------------------------------------------------------------ dispatch

template <typename T>
hipError_t launch_coef(const Plan& p, const void* I_lo, const void* p_lo, const float* eps,
                       int eps_count, float* abar, float* bbar, hipStream_t s) {
  CoefArgs a{I_lo, p_lo, eps, eps_count, p.c, p.h, p.w, p.r, p.mean_ab, p.coTH, p.coTW, abar,
             bbar};
  dim3 grid((p.w + p.coTW - 1) / p.coTW, (p.h + p.coTH - 1) / p.coTH, p.planes);
  prof_begin("gf_coef", s);
  hipLaunchKernelGGL(coef_kernel<T>, grid, dim3(256), p.coLDS, s, a);
  prof_end(s);
  return hipGetLastError();
}

template <typename T, int S, int VEC>
hipError_t launch_apply_t(const Plan& p, const FwdArgs& f, hipStream_t s) {
  ApplyArgs a{f.I_hi, f.q, reinterpret_cast<const float*>(f.ws + p.off_abar),
              reinterpret_cast<const float*>(f.ws + p.off_bbar), p.h, p.w, p.H, p.W, p.RB,
              p.nrb, p.nxv, (long long)p.planes * p.nrb * p.nxv};
  const unsigned blocks = (unsigned)((a.total + 255) / 256);
  prof_begin("gf_apply", s);
  hipLaunchKernelGGL((apply_kernel<T, S, VEC>), dim3(blocks), dim3(256), 0, s, a);
  prof_end(s);
  return hipGetLastError();
}

template <typename T, int S, int VEC>
hipError_t launch_bwd_hi_t(const Plan& p, const BwdArgs& b, hipStream_t s) {
  BwdHiArgs a{b.I_hi, b.dq, b.dI_hi, reinterpret_cast<const float*>(b.ws + p.off_abar),
              reinterpret_cast<float*>(b.ws + p.off_u), p.h, p.w, p.H, p.W, p.bh, p.tw, p.nby,
              p.nbx};
  prof_begin("gf_bwd_hi", s);
  hipLaunchKernelGGL((bwd_hi_kernel<T, S, VEC>), dim3(p.nbx, p.nby, p.planes), dim3(64), 0, s,
                     a);
  prof_end(s);
  return hipGetLastError();
}

template <typename T, int VEC>
hipError_t apply_by_s(const Plan& p, const FwdArgs& f, hipStream_t s) {
  switch (p.S) {
    case 1: return launch_apply_t<T, 1, VEC>(p, f, s);
    case 2: return launch_apply_t<T, 2, VEC>(p, f, s);
    case 4: return launch_apply_t<T, 4, VEC>(p, f, s);
    case 8: return launch_apply_t<T, 8, VEC>(p, f, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int VEC>
hipError_t bwd_hi_by_s(const Plan& p, const BwdArgs& b, hipStream_t s) {
  switch (p.S) {
    case 1: return launch_bwd_hi_t<T, 1, VEC>(p, b, s);
    case 2: return launch_bwd_hi_t<T, 2, VEC>(p, b, s);
    case 4: return launch_bwd_hi_t<T, 4, VEC>(p, b, s);
    case 8: return launch_bwd_hi_t<T, 8, VEC>(p, b, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t forward_t(const Plan& p, const FwdArgs& f, hipStream_t s) {
  float* abar = reinterpret_cast<float*>(f.ws + p.off_abar);
  float* bbar = reinterpret_cast<float*>(f.ws + p.off_bbar);
  hipError_t err = launch_coef<T>(p, f.I_lo, f.p_lo, f.eps, f.eps_count, abar, bbar, s);
  if (err != hipSuccess) return err;
  constexpr int V = 16 / sizeof(T);
  return p.VEC == V ? apply_by_s<T, V>(p, f, s) : apply_by_s<T, 1>(p, f, s);
}

template <typename T>
hipError_t backward_t(const Plan& p, const BwdArgs& b, hipStream_t s) {
  float* abar = reinterpret_cast<float*>(b.ws + p.off_abar);
  hipError_t err = launch_coef<T>(p, b.I_lo, b.p_lo, b.eps, b.eps_count, abar, nullptr, s);
  if (err != hipSuccess) return err;
  constexpr int V = 16 / sizeof(T);
  err = p.VEC == V ? bwd_hi_by_s<T, V>(p, b, s) : bwd_hi_by_s<T, 1>(p, b, s);
  if (err != hipSuccess) return err;
  if (!b.dI_lo && !b.dp_lo && !b.deps) return hipSuccess;
  float* part = reinterpret_cast<float*>(b.ws + p.off_eps);
  BwdLoArgs a{b.I_lo, b.p_lo, b.eps, b.eps_count, p.c,
              reinterpret_cast<const float*>(b.ws + p.off_u), p.bh, p.tw, p.nby, p.nbx,
              p.h, p.w, p.r, p.mean_ab, p.loTH, p.loTW, p.lo_ntx, p.lo_nty,
              b.dI_lo, b.dp_lo, part};
  prof_begin("gf_bwd_lo", s);
  hipLaunchKernelGGL(bwd_lo_kernel<T>, dim3(p.lo_ntx, p.lo_nty, p.planes), dim3(256), p.loLDS,
                     s, a);
  prof_end(s);
  err = hipGetLastError();
  if (err != hipSuccess || !b.deps) return err;
  prof_begin("gf_eps_reduce", s);
  hipLaunchKernelGGL(eps_reduce_kernel, dim3(b.eps_count), dim3(256), 0, s, part,
                     p.lo_ntx * p.lo_nty, p.c, p.n, b.eps_count, b.deps);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_forward(const Plan& p, const FwdArgs& a, hipStream_t s) {
  switch (p.dtype) {
    case GF_F32: return forward_t<float>(p, a, s);
    case GF_F16: return forward_t<_Float16>(p, a, s);
    case GF_BF16: return forward_t<bf16>(p, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_backward(const Plan& p, const BwdArgs& a, hipStream_t s) {
  switch (p.dtype) {
    case GF_F32: return backward_t<float>(p, a, s);
    case GF_F16: return backward_t<_Float16>(p, a, s);
    case GF_BF16: return backward_t<bf16>(p, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gf
