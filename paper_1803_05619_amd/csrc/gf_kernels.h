#pragma once
// HIP kernels of the fast guided filtering layer for gfx950 (MI355X).
// Included once per I/O element type by gf_f32.hip, gf_f16.hip and
// gf_bf16.hip, which instantiate the launchers for that type.
//
// Forward (Sec. III-B/C, Eq. (1)-(2)):
//   coef_kernel   low-res column walker: box statistics of the recentred
//                 guide and input, A = cov/(var+eps), b = mean_p - A mean_I,
//                 then their window means; writes Abar, bbar (low-res, fp32).
//   apply_kernel  streams the high-res guide: bilinear Abar/bbar taps are
//                 blended in registers (never stored at high resolution) and
//                 q = A_h G_h + b_h is written; non-temporal loads and stores.
// Backward (Algorithm 1, plus the adjoint of the A/b window mean):
//   coef_kernel   recomputes Abar (and bbar when the forward runs too).
//   bwd_hi_kernel one wave per band of high-res rows (stacked four to a
//                 workgroup for FP32 at S >= 4): dI_h = dq A_h (and q in the
//                 fused pass), and the transposed bilinear of dq G_h and dq
//                 accumulated vertically in registers, then horizontally by
//                 lane shuffles or through LDS, into partial low-res planes
//                 per block (no atomics).
//   bwd_lo_kernel low-res column walker: gathers the partial planes,
//                 recomputes the box statistics and runs the adjoint chain;
//                 f_mu^T(y) is the box SUM of y/N.  Writes dI_l, dp_l and
//                 per-segment deps partials.
//   eps_reduce_kernel  fixed-order sum of the deps partials.
// All reductions run in a fixed order, so results are bitwise reproducible.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

template <>
struct Carrier<32> {
  typedef u32x8 type;
};
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

// Streaming (non-temporal) loads and stores of the high-res planes, which
// are read once and written once: they do not displace the low-res
// coefficient rows and partial planes from the caches (measured: the fused
// FP32 pass 217 -> 208 us with non-temporal loads).
template <typename T, int VEC>
__device__ __forceinline__ void load_vec_nt(const T* p, float (&out)[VEC]) {
  typedef typename Carrier<sizeof(T) * VEC>::type C;
  C c = __builtin_nontemporal_load(reinterpret_cast<const C*>(p));
  T t[VEC];
  __builtin_memcpy(t, &c, sizeof(C));
#pragma unroll
  for (int e = 0; e < VEC; ++e) out[e] = to_f(t[e]);
}

// The same in two steps: the raw vector (held in flight, packed for the half
// types), then its elements as float.
template <typename T, int VEC>
using RawVec = typename Carrier<sizeof(T) * VEC>::type;
template <typename T, int VEC>
__device__ __forceinline__ RawVec<T, VEC> load_raw_nt(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const RawVec<T, VEC>*>(p));
}
template <typename T, int VEC>
__device__ __forceinline__ void unpack_vec(const RawVec<T, VEC>& c, float (&out)[VEC]) {
  T t[VEC];
  __builtin_memcpy(t, &c, sizeof(c));
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

// Synchronisation of the lanes of ONE wave around LDS exchanges.  Every
// kernel that uses it runs single-wave workgroups: the LDS operations of a
// wave execute in order, so a wavefront-scope fence (which orders them in the
// compiler without waiting for outstanding global loads, unlike a workgroup
// barrier) is all that is needed, and prefetched loads stay in flight.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal with the hardware instruction (about 1 ulp); the low-res
// kernels use it for window counts and variance denominators.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Whole-wave lane shifts by DPP (wave_shl:1, wave_shr:1); bound_ctrl makes
// the lane shifted in from beyond the wave read 0.  The walkers call them
// with every lane of the wave active (outside divergent branches).
__device__ __forceinline__ float lane_next(float v) {  // the value of lane + 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_prev(float v) {  // the value of lane - 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
// The values of lanes lane - R .. lane + R (index k holds lane + k - R).
template <int R>
__device__ __forceinline__ void lane_window(float v, float (&o)[2 * R + 1]) {
  o[R] = v;
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    o[R + m] = lane_next(o[R + m - 1]);
    o[R - m] = lane_prev(o[R - m + 1]);
  }
}
template <int R>
__device__ __forceinline__ float lane_sum(float v) {
  float o[2 * R + 1];
  lane_window<R>(v, o);
  float s = o[0];
#pragma unroll
  for (int k = 1; k < 2 * R + 1; ++k) s += o[k];
  return s;
}

// Raw buffer accesses for the low-res walkers: a resource over one plane
// (base and byte size in scalar registers), a per-lane byte offset (fixed
// for a wave: its column) and a wave-uniform byte offset (the row).  The
// address arithmetic stays scalar, and accesses beyond the resource's size
// read 0 / are dropped by the hardware.  Word 3 is the gfx9-family default
// (32-bit data format, untyped).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                           (int)(unsigned)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 2, "32- or 16-bit elements");
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                       unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// XCD-aware workgroup order.  The dispatcher hands consecutive workgroups
// to the 8 XCDs in turn, each XCD with its own L2.  With run = m > 1 the
// linear workgroup id is remapped so that, within every 8m consecutive
// workgroups, XCD k runs the contiguous m of them starting at k m
// (neighbouring blocks, which share low-res taps, then meet in one L2 while
// the whole chip still works on one region of the image); run = 1 gives
// XCD k the contiguous k-th eighth of all the work.  A bijection on [0, n).
__device__ __forceinline__ long long xcd_order(long long p, long long n, int run) {
  if (run <= 0) return p;
  const long long m = run == 1 ? n / 8 : run;
  const long long chunk = 8 * m;
  if (m == 0 || p >= n / chunk * chunk) return p;
  const long long q = p % chunk;
  return p - q + (q % 8) * m + q / 8;
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

// Corner-aligned taps (align_corners): source s = y (n - 1) / (N - 1) on a
// low-res axis of length n (high-res N = S n); exact integer quotient and
// remainder, so floor(s) is exact.
__device__ __forceinline__ Tap tap_ac(int y, int n, int N) {
  Tap t;
  if (N <= 1) {
    t.i0 = t.i1 = 0;
    t.w = 0.f;
    return t;
  }
  const long long num = (long long)y * (n - 1);
  const int den = N - 1;
  t.i0 = (int)(num / den);
  t.w = (float)(num - (long long)t.i0 * den) / (float)den;
  t.i1 = min(t.i0 + 1, n - 1);
  return t;
}

template <bool AC>
__device__ __forceinline__ Tap tap_t(int y, int S, int n, int N) {
  if constexpr (AC)
    return tap_ac(y, n, N);
  else
    return tap(y, S, n);
}

// Weights of high-res row y (in low-res row block i) on the low-res rows
// i-1, i, i+1 under corner alignment (its taps are (i-1, i) or (i, i+1),
// clamped at the last row).
struct RowW {
  float m, c, p;
};
__device__ __forceinline__ RowW row_weights_ac(int y, int i, int h, int H) {
  const Tap t = tap_ac(y, h, H);
  RowW r;
  if (t.i0 < i) {
    r.m = 1.f - t.w;
    r.c = t.w;
    r.p = 0.f;
  } else if (t.i1 == t.i0) {
    r.m = 0.f;
    r.c = 1.f;
    r.p = 0.f;
  } else {
    r.m = 0.f;
    r.c = 1.f - t.w;
    r.p = t.w;
  }
  return r;
}

// ------------------------------------------------------------ low-res column walkers
//
// The low-res kernels run one wave per strip of 64 adjacent columns (one
// lane per column) and walk down a segment of rows, kPF rows per block.
// Vertical windows live in registers (radii up to 8) or in per-wave LDS
// ring buffers (each lane only touches its own column); horizontal windows
// take the neighbouring lanes' values by DPP lane shifts (small radii) or
// from a row buffer in LDS after a wave-level sync.  Global rows are fetched
// one block ahead.  Everything that depends on the radius is a compile-time
// constant, so the window loops unroll.  Pixels outside the image are stored
// as zeros and excluded from every window by explicit row/column masks
// (window sums run over the in-image part only).
//
// Window statistics are computed in two levels so that no step subtracts two
// large, nearly equal numbers (the law of total variance over the window's
// columns):
//   per column, over the window's rows:  cm = mean, cvv = sum (g - cm_g)^2,
//                                        cvp = sum (g - cm_g)(p - cm_p)
//   over the window's columns:           mean = avg cm,
//     var = sum cvv / N + avg (cm_g - mean_g)^2,
//     cov = sum cvp / N + avg (cm_g - mean_g)(cm_p - mean_p).

constexpr int kPF = kWalkBlock;  // rows per block (and rows fetched ahead)

struct WinStats {
  float mI, mP, var, cov;
};

__device__ __forceinline__ bool row_ok(int t, int h) { return (unsigned)t < (unsigned)h; }

// Vertical window of one lane (its own column) for the walkers: NW rows,
// row xb + OFF + t at index t while the block starting at row xb is
// processed.  In registers (index t must be a compile-time constant after
// unrolling; advance() shifts by one block) or in a per-wave LDS ring of KR
// rows indexed by absolute row (advance() is a no-op).
template <typename V, int NW, int OFF, int KR, bool REG>
struct VWin;

template <typename V, int NW, int OFF, int KR>
struct VWin<V, NW, OFF, KR, true> {
  V v[NW];
  __device__ __forceinline__ void init(V* /*ring*/, int /*x0*/, int /*lane*/, V zero) {
#pragma unroll
    for (int t = 0; t < NW; ++t) v[t] = zero;
  }
  __device__ __forceinline__ V& at(int /*xb*/, int t) { return v[t]; }
  __device__ __forceinline__ void advance() {
#pragma unroll
    for (int t = 0; t + kWalkBlock < NW; ++t) v[t] = v[t + kWalkBlock];
  }
};

template <typename V, int NW, int OFF, int KR>
struct VWin<V, NW, OFF, KR, false> {
  V* ring;
  int x0, lane;
  __device__ __forceinline__ void init(V* r, int x, int l, V /*zero*/) {
    ring = r;
    x0 = x;
    lane = l;
  }
  __device__ __forceinline__ V& at(int xb, int t) {
    return ring[(int)((unsigned)(xb + OFF + t - x0) % (unsigned)KR) * 64 + lane];
  }
  __device__ __forceinline__ void advance() {}
};

// Column statistics of the K = 2R+1 rows rc-R .. rc+R given in v (rows
// outside the image hold zeros and are masked out).
template <int R, bool IN = false>
__device__ __forceinline__ float4 column_stats_v(const float2 (&v)[2 * R + 1], int rc, int h) {
  constexpr int K = 2 * R + 1;
  int nrow = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) nrow += (IN || row_ok(rc - R + k, h)) ? 1 : 0;
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s0 += v[k].x;
    s1 += v[k].y;
  }
  const float inv = rcp((float)nrow);
  const float cg = s0 * inv, cp = s1 * inv;
  float vv = 0.f, vp = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool ok = IN || row_ok(rc - R + k, h);
    const float dg = ok ? v[k].x - cg : 0.f;
    const float dp = ok ? v[k].y - cp : 0.f;
    vv += dg * dg;
    vp += dg * dp;
  }
  return make_float4(cg, cp, vv, vp);
}

// Window statistics from the column statistics of the window's columns
// (lanes lane-R .. lane+R): cx, cy their column means, wv, wp the sums of
// their cvv, cvp; cmask[k] = 1 for in-image columns.
template <int R>
__device__ __forceinline__ WinStats window_stats_c(const float (&cx)[2 * R + 1],
                                                   const float (&cy)[2 * R + 1], float wv,
                                                   float wp, const float (&cmask)[2 * R + 1],
                                                   float inv_ncol, float invN) {
  constexpr int K = 2 * R + 1;
  float s0 = cx[0], s1 = cy[0];
#pragma unroll
  for (int k = 1; k < K; ++k) {
    s0 += cx[k];
    s1 += cy[k];
  }
  WinStats st;
  st.mI = s0 * inv_ncol;
  st.mP = s1 * inv_ncol;
  float bv = 0.f, bp = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float dg = cmask[k] * (cx[k] - st.mI);
    const float dp = cy[k] - st.mP;
    bv += dg * dg;
    bp += dg * dp;
  }
  st.var = wv * invN + bv * inv_ncol;
  st.cov = wp * invN + bp * inv_ncol;
  return st;
}

// The same from an LDS row of column statistics (entries of lanes
// lane-R .. lane+R).
template <int R>
__device__ __forceinline__ WinStats window_stats(const float4* cs, int lane,
                                                 const float (&cmask)[2 * R + 1], float inv_ncol,
                                                 float invN) {
  constexpr int K = 2 * R + 1;
  float cx[K], cy[K], wv = 0.f, wp = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float4 c = cs[lane + k - R];
    cx[k] = c.x;
    cy[k] = c.y;
    wv += c.z;
    wp += c.w;
  }
  return window_stats_c<R>(cx, cy, wv, wp, cmask, inv_ncol, invN);
}

// The same from this lane's own column statistics, the neighbours' by DPP.
template <int R>
__device__ __forceinline__ WinStats window_stats_dpp(float4 c, const float (&cmask)[2 * R + 1],
                                                     float inv_ncol, float invN) {
  constexpr int K = 2 * R + 1;
  float cx[K], cy[K];
  lane_window<R>(c.x, cx);
  lane_window<R>(c.y, cy);
  return window_stats_c<R>(cx, cy, lane_sum<R>(c.z), lane_sum<R>(c.w), cmask, inv_ncol, invN);
}

// ------------------------------------------------------------ forward: low-res



// Abar, bbar (A, b when MAB is false) of a strip of 64 - 2(R + R_ab) output
// columns x TR output rows.  The guide and input are recentred by their
// values at the segment centre (variance and covariance are shift
// invariant; b is formed from the actual means).  Blocks whose rows and
// windows all lie inside the image and the segment run without row checks.
// Lanes without a result compute one anyway and select zero, so that each
// phase is one basic block (the DPP shifts then fold into the adds).
template <typename TG, typename TP, int R, bool MAB>
__device__ __forceinline__ void coef_body(const CoefArgs& a, const int bx, const int by,
                                          const int plane) {
  constexpr int K = 2 * R + 1;
  constexpr int HB = MAB ? R : 0;
  constexpr int HAL = R + HB;
  constexpr int TWo = 64 - 2 * HAL;
  constexpr int KR = walker_ring_rows(R, kPF, kCoefRingPow2Max);
  constexpr bool REG = coef_reg_window(R);
  constexpr bool DPP = coef_lane_dpp(R);
  constexpr int NW = 2 * R + kPF;
  extern __shared__ float4 lds4[];
  // LDS when the horizontal windows do not use DPP: [kPF][64] column
  // statistics, [kPF][64] column sums of (A, b); then the rings (large R)
  float4* cs = lds4;
  float2* vs = reinterpret_cast<float2*>(cs + kPF * 64);
  float2* rings = DPP ? reinterpret_cast<float2*>(lds4) : vs + kPF * 64;
  // vertical windows: recentred (g, p) rows xb-2R.., (A, b) rows xb-3R..
  VWin<float2, NW, -2 * R, KR, REG> gp;
  VWin<float2, NW, -3 * R, KR, REG> ab;
  const int lane = threadIdx.x;
  const float e = a.eps[a.eps_count == 1 ? 0 : plane / a.c];
  const int h = a.h, w = a.w;
  const int j0 = bx * TWo;
  const int jl = j0 - HAL;  // image column of lane 0
  const int j = jl + lane;
  const bool colin = (unsigned)j < (unsigned)w;
  const int i0 = by * a.TR, i1 = min(i0 + a.TR, h);
  const size_t pofs = (size_t)plane * h * w;
  const TG* G = reinterpret_cast<const TG*>(a.I_lo) + pofs;
  const TP* P = reinterpret_cast<const TP*>(a.p_lo) + pofs;
  const size_t hw = (size_t)h * w;
  const __amdgpu_buffer_rsrc_t gR = buf_rsrc(G, hw * sizeof(TG));
  const __amdgpu_buffer_rsrc_t pR = buf_rsrc(P, hw * sizeof(TP));
  const __amdgpu_buffer_rsrc_t aR = buf_rsrc(a.abar + pofs, hw * 4);
  const __amdgpu_buffer_rsrc_t bR = buf_rsrc(a.bbar ? a.bbar + pofs : a.abar, a.bbar ? hw * 4 : 0);
  const int ic = min(i0 + a.TR / 2, h - 1), jc = min(max(j0 + TWo / 2, 0), w - 1);
  const float cg = to_f(G[(size_t)ic * w + jc]);
  const float cp = to_f(P[(size_t)ic * w + jc]);
  float cmask[K];
  float ncol = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cmask[k] = ((unsigned)(j + k - R) < (unsigned)w) ? 1.f : 0.f;
    ncol += cmask[k];
  }
  const float inv_ncol = rcp(fmaxf(ncol, 1.f));
  const bool a_lane = colin && lane >= R && lane < 64 - R;  // lanes that form (A, b)
  const bool out_lane = colin && lane >= HAL && lane < HAL + TWo;
  const unsigned jo = (unsigned)(colin ? j : 0) * 4u;  // output byte offset in a row
  const int x0 = i0 - HAL, xend = i1 + HAL;  // input rows walked
  gp.init(rings, x0, lane, make_float2(0.f, 0.f));
  ab.init(rings + KR * 64, x0, lane, make_float2(0.f, 0.f));

  // Loads are unconditional (clamped row) and the queue holds the raw
  // values: a load inside a divergent branch, or arithmetic right after it,
  // would make the wave wait for it there instead of a block later.
  const int jcl = min(max(j, 0), w - 1);
  const unsigned jg = (unsigned)jcl * sizeof(TG), jp = (unsigned)jcl * sizeof(TP);
  auto load = [&](int x, TG& g, TP& p) __attribute__((always_inline)) {
    const unsigned o = (unsigned)(min(max(x, 0), h - 1) * w);
    g = buf_ld<TG>(gR, jg, o * (unsigned)sizeof(TG));
    p = buf_ld<TP>(pR, jp, o * (unsigned)sizeof(TP));
  };
  // 1 / N for the window of row t (interior rows: K rows)
  auto inv_count = [&](auto tag, int t) __attribute__((always_inline)) {
    constexpr bool IN = decltype(tag)::value;
    const int nrow = IN ? K : min(t + R, h - 1) - max(t - R, 0) + 1;
    return inv_ncol * rcp((float)nrow);
  };
  // (A, b) from the window statistics; zero where the lane forms none
  auto coef_of = [&](const WinStats& st, bool ok) __attribute__((always_inline)) {
    const float den = st.var + e;
    const float A = den > 0.f ? st.cov * rcp(den) : 0.f;
    const float B = (st.mP + cp) - A * (st.mI + cg);
    return ok ? make_float2(A, B) : make_float2(0.f, 0.f);
  };
  auto put_ab = [&](int xb, int d, int rc, float2 v) __attribute__((always_inline)) {
    if (!MAB) {
      if (rc >= i0 && rc < i1 && out_lane) {
        const unsigned ro = (unsigned)(rc * w) * 4u;
        buf_st(v.x, aR, jo, ro);
        if (a.bbar) buf_st(v.y, bR, jo, ro);
      }
    } else {
      ab.at(xb, 2 * R + d) = v;  // row rc
    }
  };
  auto put_bar = [&](auto tag, int ra, float sa, float sb) __attribute__((always_inline)) {
    const float invN = inv_count(tag, ra);
    if (out_lane) {
      const unsigned ro = (unsigned)(ra * w) * 4u;
      buf_st(sa * invN, aR, jo, ro);
      if (a.bbar) buf_st(sb * invN, bR, jo, ro);
    }
  };

  auto block = [&](auto tag, int xb, TG (&gq)[kPF], TP (&pq)[kPF]) __attribute__((always_inline)) {
    constexpr bool IN = decltype(tag)::value;
#pragma unroll
    for (int d = 0; d < kPF; ++d) {
      const int x = xb + d;
      const bool ok = colin && (IN || row_ok(x, h));
      if (IN || x < xend)
        gp.at(xb, 2 * R + d) =
            ok ? make_float2(to_f(gq[d]) - cg, to_f(pq[d]) - cp) : make_float2(0.f, 0.f);
    }
    // the queue's rows are consumed: fetch the next block's
#pragma unroll
    for (int d = 0; d < kPF; ++d) load(xb + kPF + d, gq[d], pq[d]);
    // rows rc = x - R whose windows are complete with this block
#pragma unroll
    for (int d = 0; d < kPF; ++d) {
      const int rc = xb + d - R;
      if (!(IN || (xb + d >= i0 + R - HB && xb + d < xend))) continue;
      float2 v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = gp.at(xb, d + k);  // rows rc-R .. rc+R
      const bool rok = IN || row_ok(rc, h);
      float4 st = column_stats_v<R, IN>(v, rc, h);
      if (!(colin && rok)) st = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (DPP) {
        const WinStats ws = window_stats_dpp<R>(st, cmask, inv_ncol, inv_count(tag, rc));
        put_ab(xb, d, rc, coef_of(ws, a_lane && rok));
      } else {
        cs[d * 64 + lane] = st;
      }
    }
    if constexpr (!DPP) {
      wave_sync();
#pragma unroll
      for (int d = 0; d < kPF; ++d) {
        const int rc = xb + d - R;
        if (!(IN || (xb + d >= i0 + R - HB && xb + d < xend))) continue;
        // lanes 0 .. R-1 and 64-R .. 63 form no (A, b): their window would leave the row
        const int lc = min(max(lane, R), 63 - R);
        const WinStats ws = window_stats<R>(cs + d * 64, lc, cmask, inv_ncol, inv_count(tag, rc));
        put_ab(xb, d, rc, coef_of(ws, a_lane && (IN || row_ok(rc, h))));
      }
    }
    if (MAB) {
      // rows ra = x - 2R whose (A, b) windows are complete
#pragma unroll
      for (int d = 0; d < kPF; ++d) {
        const int ra = xb + d - 2 * R;
        if (!(IN || (xb + d >= i0 + 2 * R && xb + d < xend))) continue;
        float2 v = ab.at(xb, d);  // row ra-R; outside the image: zeros
#pragma unroll
        for (int k = 1; k < K; ++k) {
          const float2 u = ab.at(xb, d + k);
          v.x += u.x;
          v.y += u.y;
        }
        if constexpr (DPP) {
          put_bar(tag, ra, lane_sum<R>(v.x), lane_sum<R>(v.y));
        } else {
          vs[d * 64 + lane] = v;
        }
      }
      if constexpr (!DPP) {
        wave_sync();
#pragma unroll
        for (int d = 0; d < kPF; ++d) {
          const int ra = xb + d - 2 * R;
          if (!(IN || (xb + d >= i0 + 2 * R && xb + d < xend)) || !out_lane) continue;
          float sa = 0.f, sb = 0.f;
#pragma unroll
          for (int k = 0; k < K; ++k) {  // columns outside the image hold zeros
            const float2 u = vs[d * 64 + lane + k - R];
            sa += u.x;
            sb += u.y;
          }
          put_bar(tag, ra, sa, sb);
        }
      }
    }
    if constexpr (!DPP) wave_sync();
  };

  TG gq[kPF];
  TP pq[kPF];
#pragma unroll
  for (int d = 0; d < kPF; ++d) load(x0 + d, gq[d], pq[d]);
  // blocks before, inside and after the interior range (xin <= xb <= xlim);
  // three loops rather than a branch per block keep the register
  // allocation of the loop-carried windows simple
  // (interior: the block's rows, the windows of its statistics rows
  // rc = x - R and of its (A, b) rows ra = x - 2R lie inside the image, every
  // phase's row is live)
  const int xin = max(x0 + 2 * HAL, 3 * R), xlim = min(xend, h) - kPF;
  int base = x0;
  for (; base < xend && (base < xin || base > xlim); base += kPF) {
    block(std::false_type{}, base, gq, pq);
    gp.advance();
    ab.advance();
  }
  for (; base <= xlim; base += kPF) {
    block(std::true_type{}, base, gq, pq);
    gp.advance();
    ab.advance();
  }
  for (; base < xend; base += kPF) {
    block(std::false_type{}, base, gq, pq);
    gp.advance();
    ab.advance();
  }
}

// The (strip, row tile, plane) of this workgroup; with `xcd` the launch order
// is remapped so that each XCD (workgroups are dispatched to the 8 XCDs in
// turn) takes a contiguous run of tiles, whose shared halo rows and columns
// then meet in that XCD's L2.
__device__ __forceinline__ void lo_tile(int xcd, int& bx, int& by, int& bz) {
  const long long nx = gridDim.x, nxy = nx * gridDim.y;
  const long long lin = xcd_order(blockIdx.x + nx * blockIdx.y + nxy * blockIdx.z,
                                  nxy * gridDim.z, xcd);
  bx = (int)(lin % nx);
  by = (int)((lin / nx) % gridDim.y);
  bz = (int)(lin / nxy);
}

template <typename TG, typename TP, int R, bool MAB>
__global__ __launch_bounds__(64) void coef_kernel(CoefArgs a) {
  int bx, by, bz;
  lo_tile(a.xcd, bx, by, bz);
  coef_body<TG, TP, R, MAB>(a, bx, by, bz);
}

// ------------------------------------------------------------ forward: high-res



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
// registers, so each high-res pixel costs one blend and one FMA.  Two
// register buffers alternate: while block i is computed, block i+1 is in
// flight (its loads are issued after the low-res tap loads of block i, so
// waiting for those does not wait for it).
template <typename TG, typename TQ, int S, int VEC, bool AC>
__device__ __forceinline__ void apply_body(const ApplyArgs& a, const long long blk) {
  const long long t = blk * 256 + threadIdx.x;
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
    const Tap tx = tap_t<AC>(x0 + e, S, w, W);
    j0[e] = tx.i0;
    j1[e] = tx.i1;
    wx[e] = tx.w;
  }
  const float* Ab = a.abar + (size_t)plane * h * w;
  const float* Bb = a.bbar + (size_t)plane * h * w;
  const size_t hofs = (size_t)plane * a.H * W + x0;
  const TG* Gp = reinterpret_cast<const TG*>(a.I_hi) + hofs;
  TQ* Qp = reinterpret_cast<TQ*>(a.q) + hofs;
  const int ib0 = rb * (a.RB / S);
  const int ib1 = min(ib0 + a.RB / S, h);
  float am[VEC], ac[VEC], ap[VEC], bm[VEC], bc[VEC], bp[VEC];
  hrow<VEC>(Ab, ib0 - 1, h, w, j0, j1, wx, am);
  hrow<VEC>(Bb, ib0 - 1, h, w, j0, j1, wx, bm);
  hrow<VEC>(Ab, ib0, h, w, j0, j1, wx, ac);
  hrow<VEC>(Bb, ib0, h, w, j0, j1, wx, bc);

  auto load_block = [&](int i, float (&g)[S][VEC]) __attribute__((always_inline)) {
#pragma unroll
    for (int t2 = 0; t2 < S; ++t2) load_vec_nt<TG, VEC>(Gp + (size_t)(S * i + t2) * W, g[t2]);
  };
  auto body = [&](int i, float (&g)[S][VEC], float (&gn)[S][VEC]) __attribute__((always_inline)) {
    hrow<VEC>(Ab, i + 1, h, w, j0, j1, wx, ap);
    hrow<VEC>(Bb, i + 1, h, w, j0, j1, wx, bp);
    if (i + 1 < ib1) load_block(i + 1, gn);
#pragma unroll
    for (int t2 = 0; t2 < S; ++t2) {
      const int num = 2 * t2 + 1 - S;
      float q[VEC];
      if constexpr (AC) {
        const RowW rw = row_weights_ac(S * i + t2, i, h, a.H);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float A = rw.m * am[e] + rw.c * ac[e] + rw.p * ap[e];
          const float B = rw.m * bm[e] + rw.c * bc[e] + rw.p * bp[e];
          q[e] = A * g[t2][e] + B;
        }
      } else if (num < 0) {
        const float wy = (float)(num + 2 * S) / (float)(2 * S);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float A = am[e] + wy * (ac[e] - am[e]);
          const float B = bm[e] + wy * (bc[e] - bm[e]);
          q[e] = A * g[t2][e] + B;
        }
      } else {
        const float wy = (float)num / (float)(2 * S);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float A = ac[e] + wy * (ap[e] - ac[e]);
          const float B = bc[e] + wy * (bp[e] - bc[e]);
          q[e] = A * g[t2][e] + B;
        }
      }
      store_vec_nt<TQ, VEC>(Qp + (size_t)(S * i + t2) * W, q);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      am[e] = ac[e];
      ac[e] = ap[e];
      bm[e] = bc[e];
      bc[e] = bp[e];
    }
  };
  float ga[S][VEC], gb[S][VEC];
  load_block(ib0, ga);
  for (int i = ib0; i < ib1; i += 2) {
    body(i, ga, gb);
    if (i + 1 < ib1) body(i + 1, gb, ga);
  }
}

template <typename TG, typename TQ, int S, int VEC, bool AC>
__global__ __launch_bounds__(256) void apply_kernel(ApplyArgs a) {
  apply_body<TG, TQ, S, VEC, AC>(a, xcd_order(blockIdx.x, gridDim.x, a.xcd));
}

// ------------------------------------------------------------ backward: high-res



// One wave per band of bh low-res rows (S*bh high-res rows) x 64*VEC
// high-res columns; hw bands stacked vertically form a workgroup.  A
// band's transposed-bilinear contributions reach low-res rows i_a-1 ..
// i_a+bh and columns j_a-1 .. j_a+tw: (bh+2) x (tw+2) partial rows for
// dA_bar (from dq*G_h) and for db_bar (from dq).  The waves write them into
// LDS (even and odd waves into separate buffers, so that no two waves of a
// buffer share a row) and the workgroup writes the sums of the two buffers
// as one (hw*bh+2) x (tw+2) partial block; the border rows/columns
// overlap the neighbouring blocks' and are summed by the low-res kernel.
//
// Vertical: per high-res row, each lane adds its VEC values, weighted, into
// accumulators of the low-res rows i-1, i, i+1 of the current row block;
// after the block, row i-1 is complete and is flushed horizontally.
// Horizontal: when the lane's VEC columns are whole low-res blocks
// (VEC % S == 0) the weights are compile-time constants and the two
// contributions that cross into the neighbouring lanes' columns move with
// one lane shuffle each; otherwise (S = 8 with 4 columns per lane, the
// VEC = 1 fallback, corner alignment) through an LDS row.
// Loads of the next rows are issued before the current ones are computed.
// FWD: the same pass also writes the forward output q = A_h G_h + b_h
// (type TQ), reading the bbar rows alongside Abar's: one read of G_h and dq
// for both directions.
template <typename TG, typename TD, typename TO, typename TQ, int S, int VEC, bool AC, bool FWD>
__device__ __forceinline__ void bwd_hi_body(const BwdHiArgs& a, const int bx, const int byg,
                                            const int plane) {
  constexpr int TWH = 64 * VEC;  // high-res columns per block
  // register flush: compile-time half-pixel weights over whole low-res
  // columns per lane; otherwise (corner alignment, VEC < S) through LDS
  constexpr bool REG = (VEC % S) == 0 && !AC;
  constexpr int NB = REG ? VEC / S : 1;  // low-res columns per lane
  constexpr int UW = TWH / S + 2;        // partial-row width (tw + 2)
  __shared__ float sR[REG ? 1 : kHiWaves][2][REG ? 1 : TWH];
  extern __shared__ float ush[];  // [even, odd waves][dA_bar, db_bar][ubh + 2][UW]
  // stacked bands (merge) or one wave per workgroup (the same indexing, constant-folded)
  constexpr bool merge = hi_merge(std::is_same<TD, float>::value, S);
  const int lane = merge ? threadIdx.x & 63 : threadIdx.x;
  const int wave = merge ? threadIdx.x >> 6 : 0;
  const int hw = merge ? a.hw : 1;
  const int by = byg * hw + wave;  // this wave's band
  const int h = a.h, w = a.w, W = a.W, bh = a.bh;
  const int URW = hw * bh + 2;          // rows of the merged partial block
  const int UPm = URW * UW;             // floats per quantity
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
    const Tap tx = tap_t<AC>(valid ? x0 + e : 0, S, w, W);
    j0[e] = tx.i0;
    j1[e] = tx.i1;
    wx[e] = tx.w;
  }
  const float* Ab = a.abar + (size_t)plane * h * w;
  const size_t hofs = (size_t)plane * a.H * W + (valid ? x0 : 0);
  const TG* Gp = reinterpret_cast<const TG*>(a.I_hi) + hofs;
  const TD* Dp = reinterpret_cast<const TD*>(a.dq) + hofs;
  TO* Op = a.dI_hi ? reinterpret_cast<TO*>(a.dI_hi) + hofs : nullptr;
  const float* Bb = FWD ? a.bbar + (size_t)plane * h * w : nullptr;
  TQ* Qp = FWD ? reinterpret_cast<TQ*>(a.q) + hofs : nullptr;
  // this wave's rows of the merge buffers (row lr of the band: merged row
  // wave * bh + lr); single-wave workgroups (the variant without merge, the
  // same layout) write their partial block straight to global memory
  float* Ub = ush + (wave & 1) * 2 * UPm + wave * bh * UW;
  float* Ug = a.U + (((size_t)plane * a.nby + byg) * a.nbx + bx) * 2 * (size_t)UPm;
  auto put = [&](int k, float v) __attribute__((always_inline)) {
    if constexpr (merge)
      Ub[k] = v;
    else
      Ug[k] = v;
  };
  // the image's last workgroup may hold empty bands (never without merge:
  // there nby = ceil(h / bh))
  const bool active = !merge || i_a < h;
  if constexpr (merge) {
    // Rows of the merge buffers that no wave writes must read as zero: in
    // this wave's buffer the gap before the next wave of the same parity
    // (its own rows too when its band is empty), and, from wave 0, the odd
    // buffer's rows above wave 1's.  No other wave touches these rows, so no
    // barrier is needed before the bands are computed.  (Rows that only a
    // partial last band leaves unwritten lie below the image and are never
    // read.)
    float* own = ush + (wave & 1) * 2 * UPm;
    const int z0 = active ? wave * bh + bh + 2 : wave * bh;
    const int z1 = wave + 2 < hw ? (wave + 2) * bh : URW;
    for (int k = z0 * UW + lane; k < z1 * UW; k += 64) {
      own[k] = 0.f;
      own[UPm + k] = 0.f;
    }
    if (wave == 0)
      for (int k = lane; k < bh * UW; k += 64) {
        ush[2 * UPm + k] = 0.f;
        ush[3 * UPm + k] = 0.f;
      }
  }
  // this lane's first low-res column (register path) and the image-edge clamps
  const int jb = x0 / S;
  const bool left_edge = (x0 == 0);
  const bool right_edge = valid && (jb + NB == w);

  // Horizontal transposed interpolation of one completed low-res row
  // (vertical sums uA/uB over this lane's VEC columns) into row lr of the
  // block's partial planes.
  auto flush = [&](const float (&uA)[VEC], const float (&uB)[VEC], int lr) __attribute__((always_inline)) {
    if constexpr (REG) {
      float oA[NB], oB[NB];
#pragma unroll
      for (int m = 0; m < NB; ++m) oA[m] = oB[m] = 0.f;
      float lA = 0.f, lB = 0.f, rA = 0.f, rB = 0.f;  // spills to jb-1 and jb+NB
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int m = e / S, t2 = e % S;
        const int num = 2 * t2 + 1 - S;
        if (num < 0) {  // taps (jb+m-1, jb+m)
          const float w1 = (float)(num + 2 * S) / (float)(2 * S);
          const float cA = (1.f - w1) * uA[e], cB = (1.f - w1) * uB[e];
          oA[m] += w1 * uA[e];
          oB[m] += w1 * uB[e];
          if (m == 0) {
            if (left_edge) {  // source clamped to column 0: all weight there
              oA[0] += cA;
              oB[0] += cB;
            } else {
              lA += cA;
              lB += cB;
            }
          } else {
            oA[m - 1] += cA;
            oB[m - 1] += cB;
          }
        } else {  // taps (jb+m, jb+m+1)
          const float w1 = (float)num / (float)(2 * S);
          const float cA = w1 * uA[e], cB = w1 * uB[e];
          oA[m] += (1.f - w1) * uA[e];
          oB[m] += (1.f - w1) * uB[e];
          if (m == NB - 1) {
            if (right_edge) {  // second tap clamped to the last column
              oA[m] += cA;
              oB[m] += cB;
            } else {
              rA += cA;
              rB += cB;
            }
          } else {
            oA[m + 1] += cA;
            oB[m + 1] += cB;
          }
        }
      }
      // lane l's right spill is column jb of lane l+1; its left spill is the
      // last column of lane l-1
      const float inA = __shfl_up(rA, 1), inB = __shfl_up(rB, 1);
      const float fromA = __shfl_down(lA, 1), fromB = __shfl_down(lB, 1);
      if (lane > 0) {
        oA[0] += inA;
        oB[0] += inB;
      }
      if (lane < 63) {
        oA[NB - 1] += fromA;
        oB[NB - 1] += fromB;
      }
      const int rowA = lr * UW, rowB = UPm + lr * UW;
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        put(rowA + 1 + lane * NB + m, oA[m]);
        put(rowB + 1 + lane * NB + m, oB[m]);
      }
      if (lane == 0) {
        put(rowA, lA);
        put(rowB, lB);
      }
      if (lane == 63) {
        put(rowA + UW - 1, rA);
        put(rowB + UW - 1, rB);
      }
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        sR[wave][0][lane * VEC + e] = uA[e];
        sR[wave][1][lane * VEC + e] = uB[e];
      }
      wave_sync();
      for (int k = lane; k < UW; k += 64) {
        const int j = j_a - 1 + k;
        float sa = 0.f, sb = 0.f;
        if (j >= 0 && j < w) {
          const int xlo = max(max(S * (j - 1), X_a), 0);
          const int xhi = min(min(S * (j + 2), X_a + TWH), W);
          for (int x = xlo; x < xhi; ++x) {
            const Tap tx = tap_t<AC>(x, S, w, W);
            const float wt = (tx.i0 == j ? 1.f - tx.w : 0.f) + (tx.i1 == j ? tx.w : 0.f);
            sa += wt * sR[wave][0][x - X_a];
            sb += wt * sR[wave][1][x - X_a];
          }
        }
        put(lr * UW + k, sa);
        put(UPm + lr * UW + k, sb);
      }
      wave_sync();
    }
  };

  float am[VEC], ac[VEC], ap[VEC];
  float bm[FWD ? VEC : 1], bc[FWD ? VEC : 1], bp[FWD ? VEC : 1];
  float pA[VEC], cA[VEC], nA[VEC], pB[VEC], cB[VEC], nB[VEC];

  // unconditional loads (lanes past the image edge re-read column 0 and
  // are zeroed), so that no load sits in a divergent branch
  // Rows are loaded in units of SR rows (a low-res row block at S <= 4,
  // half of one at S = 8: the two register buffers then hold 2 x 4 rows of
  // G and dq, not 2 x 8) while the previous unit is computed.  The buffers
  // hold the raw vectors (two half elements per register for the half
  // types), converted row by row where they are used: the FP16 fused pass
  // 170 -> 148 VGPRs, a third wave per SIMD.
  constexpr int SR = S >= 8 ? S / 2 : S;
  constexpr int NH = S / SR;
  typedef RawVec<TD, VEC> RD;
  typedef RawVec<TG, VEC> RG;
  auto load_unit = [&](int i, int u, RD (&d)[SR], RG (&g)[SR]) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < SR; ++t) {
      d[t] = load_raw_nt<TD, VEC>(Dp + (size_t)(S * i + SR * u + t) * W);
      g[t] = load_raw_nt<TG, VEC>(Gp + (size_t)(S * i + SR * u + t) * W);
    }
  };
  // unit U of low-res row block i
  auto part = [&](auto uc, int i, RD (&dr)[SR], RG (&gr)[SR], RD (&dn)[SR], RG (&gn)[SR])
                  __attribute__((always_inline)) {
    constexpr int U = decltype(uc)::value;
    if constexpr (U == 0) {
      hrow<VEC>(Ab, i + 1, h, w, j0, j1, wx, ap);
      if constexpr (FWD) hrow<VEC>(Bb, i + 1, h, w, j0, j1, wx, bp);
    }
    if constexpr (U + 1 < NH)
      load_unit(i, U + 1, dn, gn);
    else if (i + 1 < i_b)
      load_unit(i + 1, 0, dn, gn);
    const bool top = (i == 0), bot = (i == h - 1);
#pragma unroll
    for (int t = 0; t < SR; ++t) {
      const int t2 = SR * U + t;  // row within the block
      const int num = 2 * t2 + 1 - S;
      float o[VEC], qo[FWD ? VEC : 1];
      float d[1][VEC], g[1][VEC];  // this row as float (index 0)
      unpack_vec<TD, VEC>(dr[t], d[0]);
      unpack_vec<TG, VEC>(gr[t], g[0]);
      // weights of this row on the low-res rows i-1, i, i+1; at the image's
      // first/last row block the source row is clamped and all weight goes
      // to row i (selected as weights, not as branches over accumulators)
      if constexpr (AC) {
        const RowW rw = row_weights_ac(S * i + t2, i, h, a.H);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float dv = valid ? d[0][e] : 0.f;
          const float Av = rw.m * am[e] + rw.c * ac[e] + rw.p * ap[e];
          if constexpr (FWD)
            qo[e] = Av * g[0][e] + (rw.m * bm[e] + rw.c * bc[e] + rw.p * bp[e]);
          o[e] = dv * Av;
          const float vA = dv * g[0][e], vB = dv;
          pA[e] += rw.m * vA;
          cA[e] += rw.c * vA;
          nA[e] += rw.p * vA;
          pB[e] += rw.m * vB;
          cB[e] += rw.c * vB;
          nB[e] += rw.p * vB;
        }
      } else if (num < 0) {
        const float wy = (float)(num + 2 * S) / (float)(2 * S);
        const float wp = top ? 0.f : 1.f - wy, wc = top ? 1.f : wy;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float dv = valid ? d[0][e] : 0.f;
          const float Av = am[e] + wy * (ac[e] - am[e]);
          if constexpr (FWD) qo[e] = Av * g[0][e] + (bm[e] + wy * (bc[e] - bm[e]));
          o[e] = dv * Av;
          const float vA = dv * g[0][e], vB = dv;
          pA[e] += wp * vA;
          cA[e] += wc * vA;
          pB[e] += wp * vB;
          cB[e] += wc * vB;
        }
      } else {
        const float wy = (float)num / (float)(2 * S);
        const float wc = bot ? 1.f : 1.f - wy, wn = bot ? 0.f : wy;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float dv = valid ? d[0][e] : 0.f;
          const float Av = ac[e] + wy * (ap[e] - ac[e]);
          if constexpr (FWD) qo[e] = Av * g[0][e] + (bc[e] + wy * (bp[e] - bc[e]));
          o[e] = dv * Av;
          const float vA = dv * g[0][e], vB = dv;
          cA[e] += wc * vA;
          nA[e] += wn * vA;
          cB[e] += wc * vB;
          nB[e] += wn * vB;
        }
      }
      if (Op && valid) store_vec_nt<TO, VEC>(Op + (size_t)(S * i + t2) * W, o);
      if constexpr (FWD)
        if (valid) store_vec_nt<TQ, VEC>(Qp + (size_t)(S * i + t2) * W, qo);
    }
    if constexpr (U + 1 < NH) return;
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
      if constexpr (FWD) {
        bm[e] = bc[e];
        bc[e] = bp[e];
      }
    }
  };
  if (active) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) pA[e] = cA[e] = nA[e] = pB[e] = cB[e] = nB[e] = 0.f;
    hrow<VEC>(Ab, i_a - 1, h, w, j0, j1, wx, am);
    hrow<VEC>(Ab, i_a, h, w, j0, j1, wx, ac);
    if constexpr (FWD) {
      hrow<VEC>(Bb, i_a - 1, h, w, j0, j1, wx, bm);
      hrow<VEC>(Bb, i_a, h, w, j0, j1, wx, bc);
    }
    RD da[SR], db[SR];
    RG ga[SR], gb[SR];
    load_unit(i_a, 0, da, ga);
    if constexpr (NH == 1) {
      for (int i = i_a; i < i_b; i += 2) {
        part(std::integral_constant<int, 0>{}, i, da, ga, db, gb);
        if (i + 1 < i_b) part(std::integral_constant<int, 0>{}, i + 1, db, gb, da, ga);
      }
    } else {
      for (int i = i_a; i < i_b; ++i) {
        part(std::integral_constant<int, 0>{}, i, da, ga, db, gb);
        part(std::integral_constant<int, 1>{}, i, db, gb, da, ga);
      }
    }
    flush(pA, pB, i_b - i_a);      // row i_b - 1
    flush(cA, cB, i_b - i_a + 1);  // row i_b (contributions of the last rows)
  }
  if constexpr (merge) {
    __syncthreads();
    // the merged partial block: sum of the even and odd waves' buffers
    for (int k = threadIdx.x; k < 2 * UPm; k += 64 * hw) Ug[k] = ush[k] + ush[2 * UPm + k];
  }
}

template <typename TG, typename TD, typename TO, typename TQ, int S, int VEC, bool AC, bool FWD>
__global__ __launch_bounds__(64 * kHiWaves) void bwd_hi_kernel(BwdHiArgs a) {
  const long long nwg = (long long)gridDim.x * gridDim.y * gridDim.z;
  const long long lin = xcd_order(
      blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z), nwg,
      a.xcd);
  bwd_hi_body<TG, TD, TO, TQ, S, VEC, AC, FWD>(a, (int)(lin % gridDim.x),
                                      (int)((lin / gridDim.x) % gridDim.y),
                                  (int)(lin / ((long long)gridDim.x * gridDim.y)));
}

// ------------------------------------------------------------ backward: low-res



// The partial planes that cover low-res pixel (i, j) are the block that owns
// it plus, on a block border, the neighbour whose halo row/column it is
// (weights wb, wc = 1).  Four reads per plane are always issued (absent
// neighbours re-read the owner, with weight 0) so that no load sits in a
// divergent branch.
struct URaw {
  float a00, a01, a10, a11, v00, v01, v10, v11;
};

// Per-lane (column) part of the partial-plane addressing: byte offsets
// (block column, column within the block) of the block column c0 that owns
// column j and, on a block border, of its neighbour c1 (weight wc).
struct UCol {
  unsigned o0, o1;
  float wc;
};
// Per-row part: byte offsets (block row, row within the block) of the block
// row b0 owning row i and of the neighbour b1 (weight wb).
struct URow {
  unsigned o0, o1;
  float wb;
};

__device__ __forceinline__ UCol u_col(const BwdLoArgs& a, int j) {
  const int tw = a.tw, UP2 = 2 * (a.bh + 2) * (tw + 2);
  const int c0 = j / tw, rj = j - c0 * tw;
  int c1 = c0;
  float wc = 0.f;
  if (rj == 0 && c0 > 0) {
    c1 = c0 - 1;
    wc = 1.f;
  } else if (rj == tw - 1 && c0 + 1 < a.nbx) {
    c1 = c0 + 1;
    wc = 1.f;
  }
  return UCol{4u * (unsigned)(c0 * UP2 + (j - (c0 * tw - 1))),
              4u * (unsigned)(c1 * UP2 + (j - (c1 * tw - 1))), wc};
}

// Row i's block row b0 = i / bh as a multiply-high by bmul = ceil(2^32 / bh),
// exact while i * bh < 2^32.
__device__ __forceinline__ URow u_row(const BwdLoArgs& a, unsigned bmul, int i) {
  const int bh = a.bh, UW = a.tw + 2, UP2 = 2 * (bh + 2) * UW;
  const int b0 = (int)__umulhi((unsigned)i, bmul), ri = i - b0 * bh;
  int b1 = b0;
  float wb = 0.f;
  if (ri == 0 && b0 > 0) {
    b1 = b0 - 1;
    wb = 1.f;
  } else if (ri == bh - 1 && b0 + 1 < a.nby) {
    b1 = b0 + 1;
    wb = 1.f;
  }
  return URow{4u * (unsigned)(b0 * a.nbx * UP2 + (i - (b0 * bh - 1)) * UW),
              4u * (unsigned)(b1 * a.nbx * UP2 + (i - (b1 * bh - 1)) * UW), wb};
}

// The four partial-plane reads per plane (ub: UP * 4, the byte offset of the
// second plane of a block's partials).  The neighbouring block row's reads
// are skipped on rows inside a block (weight wb = 0, the same for the whole
// wave): their terms are zero either way.
__device__ __forceinline__ URaw gather_u_raw(__amdgpu_buffer_rsrc_t r, unsigned ub, const URow& ro,
                                             const UCol& co) {
  URaw z;
  z.a00 = buf_ld<float>(r, co.o0, ro.o0);
  z.a01 = buf_ld<float>(r, co.o1, ro.o0);
  z.v00 = buf_ld<float>(r, co.o0, ro.o0 + ub);
  z.v01 = buf_ld<float>(r, co.o1, ro.o0 + ub);
  if (ro.wb != 0.f) {
    z.a10 = buf_ld<float>(r, co.o0, ro.o1);
    z.a11 = buf_ld<float>(r, co.o1, ro.o1);
    z.v10 = buf_ld<float>(r, co.o0, ro.o1 + ub);
    z.v11 = buf_ld<float>(r, co.o1, ro.o1 + ub);
  } else {
    z.a10 = z.a11 = z.v10 = z.v11 = 0.f;
  }
  return z;
}

// Adjoint of the low-res part (Algorithm 1, plus the adjoint of the A/b
// window mean): one wave per strip of 64 - 4R output columns x TR output
// rows.  Per input row: the recentred guide/input and the gathered upstream
// planes dAbar, dbbar (divided by the window count N when MAB, so that
// f_mu^T(y) = box sum of y/N); per row whose window is complete: statistics,
// A, and the adjoint quantities X = (dmean_I, dmean_p, dcov, dvar) / N; per
// row whose X window is complete: box sums of X give dG and dp.  Blocks
// whose rows and windows all lie inside the image and the segment run
// without row checks.
template <typename TG, typename TP, int R, bool MAB>
__device__ __forceinline__ void bwd_lo_body(const BwdLoArgs& a, const int bx, const int by,
                                            const int plane) {
  constexpr int K = 2 * R + 1;
  constexpr int TWo = 64 - 4 * R;
  constexpr int KR = walker_ring_rows(R, kPF, kBwdLoRingPow2Max);
  constexpr bool REG = bwd_lo_reg_window(R);
  constexpr bool DPP = bwd_lo_lane_dpp(R);
  constexpr int NW = 2 * R + kPF;
  extern __shared__ float4 lds4[];
  // LDS when the horizontal windows do not use DPP: [kPF][64] column
  // statistics, column sums of (dAbar, dbbar), column sums of X; then the
  // rings (large R)
  float4* cs = lds4;
  float2* cu = reinterpret_cast<float2*>(cs + kPF * 64);
  float4* vs = reinterpret_cast<float4*>(cu + kPF * 64);
  float4* rings = DPP ? lds4 : vs + kPF * 64;
  // vertical windows: (g', p', dAbar, dbbar) rows xb-2R.., X rows xb-3R..
  VWin<float4, NW, -2 * R, KR, REG> in;
  VWin<float4, NW, -3 * R, KR, REG> xr;
  const int lane = threadIdx.x;
  const float e = a.eps[a.eps_count == 1 ? 0 : plane / a.c];
  const int h = a.h, w = a.w;
  const int j0 = bx * TWo;
  const int jl = j0 - 2 * R;
  const int j = jl + lane;
  const bool colin = (unsigned)j < (unsigned)w;
  const int i0 = by * a.TR, i1 = min(i0 + a.TR, h);
  const size_t pofs = (size_t)plane * h * w;
  const size_t hw = (size_t)h * w;
  const TG* G = reinterpret_cast<const TG*>(a.I_lo) + pofs;
  const TP* P = reinterpret_cast<const TP*>(a.p_lo) + pofs;
  const __amdgpu_buffer_rsrc_t gR = buf_rsrc(G, hw * sizeof(TG));
  const __amdgpu_buffer_rsrc_t pR = buf_rsrc(P, hw * sizeof(TP));
  const __amdgpu_buffer_rsrc_t dgR = buf_rsrc(a.dI_lo ? a.dI_lo + pofs : nullptr, a.dI_lo ? hw * 4 : 0);
  const __amdgpu_buffer_rsrc_t dpR = buf_rsrc(a.dp_lo ? a.dp_lo + pofs : nullptr, a.dp_lo ? hw * 4 : 0);
  const int ic = min(i0 + a.TR / 2, h - 1), jc = min(max(j0 + TWo / 2, 0), w - 1);
  const float cg = to_f(G[(size_t)ic * w + jc]);
  const float cp = to_f(P[(size_t)ic * w + jc]);
  float cmask[K];
  float ncol = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cmask[k] = ((unsigned)(j + k - R) < (unsigned)w) ? 1.f : 0.f;
    ncol += cmask[k];
  }
  const float inv_ncol = rcp(fmaxf(ncol, 1.f));
  const bool x_lane = colin && lane >= R && lane < 64 - R;  // lanes that form X
  const bool out_col = colin && lane >= 2 * R && lane < 2 * R + TWo;
  const unsigned jo = (unsigned)(colin ? j : 0) * 4u;  // output byte offset in a row
  const int x0 = i0 - 2 * R, xend = i1 + 2 * R;
  in.init(rings, x0, lane, make_float4(0.f, 0.f, 0.f, 0.f));
  xr.init(rings + KR * 64, x0, lane, make_float4(0.f, 0.f, 0.f, 0.f));
  float deps_acc = 0.f;

  // Loads are unconditional (clamped row) and the queue holds the raw
  // values: a load inside a divergent branch, or arithmetic right after it,
  // would make the wave wait for it there instead of a block later.
  const int jcl = min(max(j, 0), w - 1);
  const unsigned jg = (unsigned)jcl * sizeof(TG), jp = (unsigned)jcl * sizeof(TP);
  struct Raw {
    TG g;
    TP p;
    URaw u;
    float wb;
  };
  const size_t UP = (size_t)(a.bh + 2) * (a.tw + 2);
  const size_t uplane = (size_t)a.nby * a.nbx * 2 * UP;  // floats per plane
  const __amdgpu_buffer_rsrc_t uR = buf_rsrc(a.U + (size_t)plane * uplane, uplane * 4);
  const unsigned ub = (unsigned)UP * 4u;
  const UCol ucol = u_col(a, jcl);
  const unsigned bmul = 0xffffffffu / (unsigned)a.bh + 1u;
  auto load = [&](int x) __attribute__((always_inline)) {
    const int xc = min(max(x, 0), h - 1);
    const unsigned o = (unsigned)(xc * w);
    const URow ro = u_row(a, bmul, xc);
    return Raw{buf_ld<TG>(gR, jg, o * (unsigned)sizeof(TG)),
               buf_ld<TP>(pR, jp, o * (unsigned)sizeof(TP)), gather_u_raw(uR, ub, ro, ucol),
               ro.wb};
  };
  // 1 / N for the window of row t (interior rows: K rows)
  auto inv_count = [&](auto tag, int t) __attribute__((always_inline)) {
    constexpr bool IN = decltype(tag)::value;
    const int nrow = IN ? K : min(t + R, h - 1) - max(t - R, 0) + 1;
    return inv_ncol * rcp((float)nrow);
  };
  // X of row rc from its window statistics and upstream dA, db (zero where
  // the lane forms none); adds dvar to the lane's deps where it is an output
  auto adjoint = [&](int rc, bool ok, const WinStats& st, float dA, float db, float invN)
                     __attribute__((always_inline)) {
    const float den = st.var + e;
    const float rden = den > 0.f ? rcp(den) : 0.f;  // A := 0 when var + eps == 0
    const float A = st.cov * rden;
    // b = mean_p - A mean_I (actual means), A = cov / (var + eps)
    const float dAt = dA - db * (st.mI + cg);
    // one-pixel windows (R = 0): var and cov do not depend on the pixel, and
    // their terms would only cancel up to rounding against terms of size
    // dA / eps
    const float dcov = R == 0 ? 0.f : dAt * rden;
    const float dvar = R == 0 ? 0.f : -dAt * A * rden;
    // var = E[g'^2] - mI'^2, cov = E[g'p'] - mI' mP' (recentred g', p')
    const float dmI = -db * A - dcov * st.mP - 2.f * dvar * st.mI;
    const float dmP = db - dcov * st.mI;
    if (rc >= i0 && rc < i1) deps_acc += out_col ? dvar : 0.f;
    return ok ? make_float4(dmI * invN, dmP * invN, dcov * invN, dvar * invN)
              : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  auto put_out = [&](int rx, float4 B, float4 gpv) __attribute__((always_inline)) {
    const unsigned ro = (unsigned)(rx * w) * 4u;
    if (a.dI_lo) buf_st(B.x + 2.f * B.w * gpv.x + B.z * gpv.y, dgR, jo, ro);
    if (a.dp_lo) buf_st(B.y + B.z * gpv.x, dpR, jo, ro);
  };

  auto block = [&](auto tag, int xb, Raw (&q)[kPF]) __attribute__((always_inline)) {
    constexpr bool IN = decltype(tag)::value;
#pragma unroll
    for (int d = 0; d < kPF; ++d) {
      const int x = xb + d;
      if (!IN && x >= xend) continue;
      const bool ok = colin && (IN || row_ok(x, h));
      const float wb = q[d].wb, wc = ucol.wc;
      const URaw& z = q[d].u;
      float u = (z.a00 + wc * z.a01) + wb * (z.a10 + wc * z.a11);
      float vv = (z.v00 + wc * z.v01) + wb * (z.v10 + wc * z.v11);
      if (MAB) {  // f_mu^T(y) = box sum of y / N: divide by N here
        const float invN = inv_count(tag, x);
        u *= invN;
        vv *= invN;
      }
      in.at(xb, 2 * R + d) = ok ? make_float4(to_f(q[d].g) - cg, to_f(q[d].p) - cp, u, vv)
                                : make_float4(0.f, 0.f, 0.f, 0.f);  // row x
    }
    // the queue's rows are consumed: fetch the next block's
#pragma unroll
    for (int d = 0; d < kPF; ++d) q[d] = load(xb + kPF + d);
    // rows rc = x - R whose windows are complete with this block
#pragma unroll
    for (int d = 0; d < kPF; ++d) {
      const int rc = xb + d - R;
      if (!(IN || (xb + d >= i0 && xb + d < xend))) continue;
      const bool rok = IN || row_ok(rc, h);
      float4 v[K];
      int nrow = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        v[k] = in.at(xb, d + k);  // row rc-R+k
        nrow += (IN || row_ok(rc - R + k, h)) ? 1 : 0;
      }
      float4 st;
      float2 su;
      st.x = v[0].x;
      st.y = v[0].y;
      su.x = v[0].z;
      su.y = v[0].w;
#pragma unroll
      for (int k = 1; k < K; ++k) {
        st.x += v[k].x;
        st.y += v[k].y;
        su.x += v[k].z;
        su.y += v[k].w;
      }
      const float inv = rcp((float)max(nrow, 1));
      st.x *= inv;
      st.y *= inv;
      st.z = 0.f;
      st.w = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool ok = IN || row_ok(rc - R + k, h);
        const float dg = ok ? v[k].x - st.x : 0.f;
        const float dp = ok ? v[k].y - st.y : 0.f;
        st.z += dg * dg;
        st.w += dg * dp;
      }
      if (!(colin && rok)) {
        st = make_float4(0.f, 0.f, 0.f, 0.f);
        su = make_float2(0.f, 0.f);
      }
      if constexpr (DPP) {
        const float invN = inv_count(tag, rc);
        const WinStats ws = window_stats_dpp<R>(st, cmask, inv_ncol, invN);
        float dA, db;
        if (MAB) {  // f_mu^T of the upstream planes: box sums of dAbar/N, dbbar/N
          dA = lane_sum<R>(su.x);
          db = lane_sum<R>(su.y);
        } else {
          const float4 c = in.at(xb, d + R);  // row rc
          dA = c.z;
          db = c.w;
        }
        xr.at(xb, 2 * R + d) = adjoint(rc, x_lane && rok, ws, dA, db, invN);  // row rc
      } else {
        cs[d * 64 + lane] = st;
        cu[d * 64 + lane] = su;
      }
    }
    if constexpr (!DPP) {
      wave_sync();
#pragma unroll
      for (int d = 0; d < kPF; ++d) {
        const int rc = xb + d - R;
        if (!(IN || (xb + d >= i0 && xb + d < xend))) continue;
        const bool ok = x_lane && (IN || row_ok(rc, h));
        const float invN = inv_count(tag, rc);
        // lanes 0 .. R-1 and 64-R .. 63 form no X: their window would leave the row
        const int lc = min(max(lane, R), 63 - R);
        const WinStats st = window_stats<R>(cs + d * 64, lc, cmask, inv_ncol, invN);
        float dA, db;
        if (MAB) {  // f_mu^T of the upstream planes: box sums of dAbar/N, dbbar/N
          dA = 0.f;
          db = 0.f;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float2 c = cu[d * 64 + lc + k - R];
            dA += c.x;
            db += c.y;
          }
        } else {
          const float4 c = in.at(xb, d + R);  // row rc
          dA = c.z;
          db = c.w;
        }
        xr.at(xb, 2 * R + d) = adjoint(rc, ok, st, dA, db, invN);  // row rc
      }
    }
    // rows rx = x - 2R whose X windows are complete
#pragma unroll
    for (int d = 0; d < kPF; ++d) {
      const int rx = xb + d - 2 * R;
      if (!(IN || (xb + d >= i0 + 2 * R && xb + d < xend))) continue;
      float4 sum = xr.at(xb, d);  // rows rx-R .. rx+R; outside the image: zeros
#pragma unroll
      for (int k = 1; k < K; ++k) {
        const float4 v = xr.at(xb, d + k);
        sum.x += v.x;
        sum.y += v.y;
        sum.z += v.z;
        sum.w += v.w;
      }
      if constexpr (DPP) {
        const float4 B = make_float4(lane_sum<R>(sum.x), lane_sum<R>(sum.y), lane_sum<R>(sum.z),
                                     lane_sum<R>(sum.w));
        if (out_col) put_out(rx, B, in.at(xb, d));  // in.at(xb, d): row rx
      } else {
        vs[d * 64 + lane] = sum;
      }
    }
    if constexpr (!DPP) {
      wave_sync();
#pragma unroll
      for (int d = 0; d < kPF; ++d) {
        const int rx = xb + d - 2 * R;
        if (!(IN || (xb + d >= i0 + 2 * R && xb + d < xend)) || !out_col) continue;
        float4 B = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < K; ++k) {  // columns outside the image hold zeros
          const float4 v = vs[d * 64 + lane + k - R];
          B.x += v.x;
          B.y += v.y;
          B.z += v.z;
          B.w += v.w;
        }
        put_out(rx, B, in.at(xb, d));  // in.at(xb, d): row rx
      }
      wave_sync();
    }
  };

  Raw q[kPF];
#pragma unroll
  for (int d = 0; d < kPF; ++d) q[d] = load(x0 + d);
  // blocks before, inside and after the interior range (xin <= xb <= xlim);
  // three loops rather than a branch per block keep the register
  // allocation of the loop-carried windows simple
  // (interior: the block's rows, their windows and those of the statistics
  // rows rc = x - R lie inside the image, every phase's row is live)
  const int xin = max(x0 + 4 * R, 2 * R), xlim = min(xend, h - R) - kPF;
  int base = x0;
  for (; base < xend && (base < xin || base > xlim); base += kPF) {
    block(std::false_type{}, base, q);
    in.advance();
    xr.advance();
  }
  for (; base <= xlim; base += kPF) {
    block(std::true_type{}, base, q);
    in.advance();
    xr.advance();
  }
  for (; base < xend; base += kPF) {
    block(std::false_type{}, base, q);
    in.advance();
    xr.advance();
  }
  // fixed-order wave reduction of this strip's deps contribution
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) deps_acc += __shfl_xor(deps_acc, off);
  if (lane == 0)
    a.eps_part[((size_t)plane * a.pny + by) * a.pnx + bx] = deps_acc;
}

template <typename TG, typename TP, int R, bool MAB>
__global__ __launch_bounds__(64) void bwd_lo_kernel(BwdLoArgs a) {
  int bx, by, bz;
  lo_tile(a.xcd, bx, by, bz);
  bwd_lo_body<TG, TP, R, MAB>(a, bx, by, bz);
}

__global__ __launch_bounds__(256) void eps_reduce_kernel(const float* part, int per_plane,
                                                          int c, int n, int eps_count,
                                                          float* deps) {
  // fixed order: strided per-thread sums, a shuffle tree per wave, then the
  // four waves' sums in wave order
  __shared__ float red[4];
  const int k = blockIdx.x;
  const size_t lo = (size_t)(eps_count == 1 ? 0 : k * c) * per_plane;
  const size_t hi = (size_t)(eps_count == 1 ? n * c : (k + 1) * c) * per_plane;
  float s = 0.f;
  for (size_t q = lo + threadIdx.x; q < hi; q += 256) s += part[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) deps[k] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ------------------------------------------------------------ any size ratio
//
// Problems whose high-res size is not one integer factor {1, 2, 4, 8} of the
// low-res size on both axes (the problem statement of Sec. III-A allows any
// h_lo <= h_hi, w_lo <= w_hi).  The bilinear taps of every high-res row and
// column come from exact integer quotients of the source coordinate, so the
// kernels below take any ratio, per axis, and both alignments.
//
//   apply_gen_kernel     q = A_h G_h + b_h; a thread walks RB rows of VEC
//                        columns and keeps the two interpolated low-res rows
//                        its current row taps (recomputed when the tap row
//                        moves).
//   bwd_gen_rows_kernel  vertical adjoint: one thread per (low-res row i,
//                        VEC high-res columns) sums the high-res rows whose
//                        taps touch row i, weighted, into V (low-res rows x
//                        high-res columns, dA_bar and db_bar parts); the rows
//                        whose first tap is i also get dI_h = dq A_h (and q in
//                        the fused pass), so each high-res pixel is written
//                        once.  High-res rows are read by the (at most two)
//                        low-res rows they touch.
//   bwd_gen_cols_kernel  horizontal adjoint: one thread per low-res pixel sums
//                        its V row over the columns whose taps touch it,
//                        into the partial-plane layout of the low-res
//                        backward as one block per plane.
// No atomics: each output is one thread's fixed-order sum.

// Taps of high-res index y on a low-res axis of n samples (high-res N >= n):
// half-pixel source ((2y + 1) n - N) / (2N), clamped at 0, or corner-aligned
// y (n - 1) / (N - 1); floor from the exact integer quotient, the weight
// from the exact remainder (one rounding).
template <bool AC>
__device__ __forceinline__ Tap tap_gen(int y, int n, int N) {
  Tap t;
  if constexpr (AC) {
    if (N <= 1 || n <= 1) {
      t.i0 = t.i1 = 0;
      t.w = 0.f;
      return t;
    }
    const long long num = (long long)y * (n - 1);
    const long long den = N - 1;
    t.i0 = (int)(num / den);
    t.w = (float)(num - (long long)t.i0 * den) / (float)den;
  } else {
    const long long num = (long long)(2 * y + 1) * n - N;
    if (num <= 0) {
      t.i0 = 0;
      t.i1 = min(1, n - 1);
      t.w = 0.f;
      return t;
    }
    const long long den = 2LL * N;
    t.i0 = (int)(num / den);
    t.w = (float)(num - (long long)t.i0 * den) / (float)den;
  }
  t.i1 = min(t.i0 + 1, n - 1);
  return t;
}

// Smallest high-res index whose first tap is >= k (N when there is none):
// the high-res rows (columns) that touch low-res row i are
// [first_tap_ge(i - 1), first_tap_ge(i + 1)).
template <bool AC>
__device__ __forceinline__ int first_tap_ge(int k, int n, int N) {
  if (k <= 0) return 0;
  long long y;
  if constexpr (AC) {
    if (n <= 1) return N;
    const long long a = (long long)k * (N - 1), b = n - 1;
    y = (a + b - 1) / b;
  } else {
    const long long a = 2LL * N * k + N - n, b = 2LL * n;
    y = (a + b - 1) / b;
  }
  return (int)min((long long)N, y);
}

// Weight of high-res index y's taps on low-res index i.
__device__ __forceinline__ float tap_weight(const Tap& t, int i) {
  return (t.i0 == i ? 1.f - t.w : 0.f) + (t.i1 == i ? t.w : 0.f);
}

template <typename TG, typename TQ, int VEC, bool AC>
__global__ __launch_bounds__(256) void apply_gen_kernel(GenArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.total) return;
  const int xv = (int)(t % a.nxv);
  const long long rest = t / a.nxv;
  const int rb = (int)(rest % a.nrb);
  const int plane = (int)(rest / a.nrb);
  const int h = a.h, w = a.w, H = a.H, W = a.W;
  const int x0 = xv * VEC;
  int j0[VEC], j1[VEC];
  float wx[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const Tap tx = tap_gen<AC>(x0 + e, w, W);
    j0[e] = tx.i0;
    j1[e] = tx.i1;
    wx[e] = tx.w;
  }
  const float* Ab = a.abar + (size_t)plane * h * w;
  const float* Bb = a.bbar + (size_t)plane * h * w;
  const size_t hofs = (size_t)plane * H * W + x0;
  const TG* Gp = reinterpret_cast<const TG*>(a.G_hi) + hofs;
  TQ* Qp = reinterpret_cast<TQ*>(a.q) + hofs;
  float a0[VEC], a1[VEC], b0[VEC], b1[VEC];
  int r0 = -1, r1 = -1;  // low-res rows held in a0/b0 and a1/b1
  const int y_end = min(H, (rb + 1) * a.RB);
  for (int y = rb * a.RB; y < y_end; ++y) {
    const Tap ty = tap_gen<AC>(y, h, H);
    if (ty.i0 != r0) {
      if (ty.i0 == r1) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          a0[e] = a1[e];
          b0[e] = b1[e];
        }
      } else {
        hrow<VEC>(Ab, ty.i0, h, w, j0, j1, wx, a0);
        hrow<VEC>(Bb, ty.i0, h, w, j0, j1, wx, b0);
      }
      r0 = ty.i0;
      hrow<VEC>(Ab, ty.i1, h, w, j0, j1, wx, a1);
      hrow<VEC>(Bb, ty.i1, h, w, j0, j1, wx, b1);
      r1 = ty.i1;
    }
    float g[VEC], q[VEC];
    load_vec_nt<TG, VEC>(Gp + (size_t)y * W, g);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const float A = a0[e] + ty.w * (a1[e] - a0[e]);
      const float B = b0[e] + ty.w * (b1[e] - b0[e]);
      q[e] = A * g[e] + B;
    }
    store_vec_nt<TQ, VEC>(Qp + (size_t)y * W, q);
  }
}

template <typename TG, typename TD, typename TO, typename TQ, int VEC, bool AC, bool FWD>
__global__ __launch_bounds__(256) void bwd_gen_rows_kernel(GenArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.total) return;
  const int xv = (int)(t % a.nxv);
  const long long rest = t / a.nxv;
  const int i = (int)(rest % a.h);
  const int plane = (int)(rest / a.h);
  const int h = a.h, w = a.w, H = a.H, W = a.W;
  const int x0 = xv * VEC;
  int j0[VEC], j1[VEC];
  float wx[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const Tap tx = tap_gen<AC>(x0 + e, w, W);
    j0[e] = tx.i0;
    j1[e] = tx.i1;
    wx[e] = tx.w;
  }
  // the coefficient rows of the high-res rows whose first tap is i: rows i
  // and i + 1 (clamped)
  const float* Ab = a.abar + (size_t)plane * h * w;
  float a0[VEC], a1[VEC], b0[VEC], b1[VEC];
  const bool need_a = a.dI_hi != nullptr || FWD;
  if (need_a) {
    hrow<VEC>(Ab, i, h, w, j0, j1, wx, a0);
    hrow<VEC>(Ab, min(i + 1, h - 1), h, w, j0, j1, wx, a1);
  }
  if constexpr (FWD) {
    const float* Bb = a.bbar + (size_t)plane * h * w;
    hrow<VEC>(Bb, i, h, w, j0, j1, wx, b0);
    hrow<VEC>(Bb, min(i + 1, h - 1), h, w, j0, j1, wx, b1);
  }
  const size_t hofs = (size_t)plane * H * W + x0;
  const TG* Gp = reinterpret_cast<const TG*>(a.G_hi) + hofs;
  const TD* Dp = reinterpret_cast<const TD*>(a.dq) + hofs;
  TO* Op = reinterpret_cast<TO*>(a.dI_hi) + hofs;
  TQ* Qp = reinterpret_cast<TQ*>(a.q) + hofs;
  float vA[VEC], vB[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) vA[e] = vB[e] = 0.f;
  const int y_beg = first_tap_ge<AC>(i - 1, h, H), y_end = first_tap_ge<AC>(i + 1, h, H);
  for (int y = y_beg; y < y_end; ++y) {
    const Tap ty = tap_gen<AC>(y, h, H);
    const float wy = tap_weight(ty, i);
    float g[VEC], d[VEC];
    load_vec_nt<TG, VEC>(Gp + (size_t)y * W, g);
    load_vec_nt<TD, VEC>(Dp + (size_t)y * W, d);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      vA[e] += wy * (d[e] * g[e]);
      vB[e] += wy * d[e];
    }
    if (ty.i0 == i) {
      if (a.dI_hi) {
        float o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = d[e] * (a0[e] + ty.w * (a1[e] - a0[e]));
        store_vec_nt<TO, VEC>(Op + (size_t)y * W, o);
      }
      if constexpr (FWD) {
        float q[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          q[e] = (a0[e] + ty.w * (a1[e] - a0[e])) * g[e] + (b0[e] + ty.w * (b1[e] - b0[e]));
        store_vec_nt<TQ, VEC>(Qp + (size_t)y * W, q);
      }
    }
  }
  float* V = a.V + (size_t)plane * 2 * h * W + (size_t)i * W + x0;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    V[e] = vA[e];
    V[(size_t)h * W + e] = vB[e];
  }
}

// One thread per low-res pixel (i, j) of a plane; writes dA_bar and db_bar
// at row i + 1, column j + 1 of the plane's single partial block
// (2 x (h + 2) x (w + 2) floats, the layout the low-res backward gathers).
template <bool AC>
__global__ __launch_bounds__(256) void bwd_gen_cols_kernel(GenArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  const int h = a.h, w = a.w, W = a.W;
  if (t >= (long long)a.planes * h * w) return;
  const int j = (int)(t % w);
  const long long rest = t / w;
  const int i = (int)(rest % h);
  const int plane = (int)(rest / h);
  const float* VA = a.V + (size_t)plane * 2 * h * W + (size_t)i * W;
  const float* VB = VA + (size_t)h * W;
  float sA = 0.f, sB = 0.f;
  const int x_beg = first_tap_ge<AC>(j - 1, w, W), x_end = first_tap_ge<AC>(j + 1, w, W);
  for (int x = x_beg; x < x_end; ++x) {
    const float wt = tap_weight(tap_gen<AC>(x, w, W), j);
    sA += wt * VA[x];
    sB += wt * VB[x];
  }
  const size_t UP = (size_t)(h + 2) * (w + 2);
  float* U = a.U + (size_t)plane * 2 * UP + (size_t)(i + 1) * (w + 2) + (j + 1);
  U[0] = sA;
  U[UP] = sB;
}

// ------------------------------------------------------------ batched (multi-problem) kernels

template <typename T>
__device__ __forceinline__ T* rebase(char* ws, T* rel) {
  return rel ? reinterpret_cast<T*>(ws + (reinterpret_cast<uintptr_t>(rel) - 1)) : nullptr;
}

// Item whose tile range holds tile t: a ballot over the ascending bases.
// Every lane of the wave gets the same (uniform) answer.
__device__ __forceinline__ int find_item(const long long* base, int count, long long t) {
  const int lane = threadIdx.x & 63;
  int k = 0;
  for (int c0 = 0; c0 < count; c0 += 64) {
    const int i = c0 + lane;
    const bool le = i < count && base[min(i, count - 1)] <= t;
    const unsigned long long m = __ballot(le);
    k += __popcll(m);
    if (m != ~0ull) break;
  }
  return k - 1;
}

template <typename Args>
__device__ __forceinline__ const MultiItem<Args>& item_of(const MultiLaunch& m, long long t,
                                                          long long& local) {
  const int k = find_item(m.base, m.count, t);
  const MultiItem<Args>& it = reinterpret_cast<const MultiItem<Args>*>(m.items)[k];
  local = t - it.base;
  return it;
}

template <typename TG, typename TP, int R, bool MAB>
__global__ __launch_bounds__(64) void coef_multi_kernel(MultiLaunch m) {
  for (long long t = blockIdx.x; t < m.total; t += gridDim.x) {
    long long l;
    const MultiItem<CoefArgs>& it = item_of<CoefArgs>(m, t, l);
    CoefArgs a = it.a;
    a.abar = rebase(m.ws, a.abar);
    a.bbar = rebase(m.ws, a.bbar);
    const long long xy = (long long)it.nx * it.ny;
    coef_body<TG, TP, R, MAB>(a, (int)(l % it.nx), (int)((l / it.nx) % it.ny), (int)(l / xy));
  }
}

template <typename TG, typename TQ, int S, int VEC, bool AC>
__global__ __launch_bounds__(256) void apply_multi_kernel(MultiLaunch m) {
  for (long long t = blockIdx.x; t < m.total; t += gridDim.x) {
    long long l;
    const MultiItem<ApplyArgs>& it = item_of<ApplyArgs>(m, t, l);
    ApplyArgs a = it.a;
    a.abar = rebase(m.ws, a.abar);
    a.bbar = rebase(m.ws, a.bbar);
    apply_body<TG, TQ, S, VEC, AC>(a, l);
  }
}

template <typename TG, typename TD, typename TO, typename TQ, int S, int VEC, bool AC, bool FWD>
__global__ __launch_bounds__(64 * kHiWaves) void bwd_hi_multi_kernel(MultiLaunch m) {
  for (long long t = blockIdx.x; t < m.total; t += gridDim.x) {
    long long l;
    const MultiItem<BwdHiArgs>& it = item_of<BwdHiArgs>(m, t, l);
    BwdHiArgs a = it.a;
    a.abar = rebase(m.ws, a.abar);
    a.U = rebase(m.ws, a.U);
    a.bbar = rebase(m.ws, a.bbar);
    const long long xy = (long long)it.nx * it.ny;
    bwd_hi_body<TG, TD, TO, TQ, S, VEC, AC, FWD>(a, (int)(l % it.nx), (int)((l / it.nx) % it.ny),
                                    (int)(l / xy));
    if constexpr (hi_merge(std::is_same<TD, float>::value, S))
      __syncthreads();  // the next tile clears the LDS this one's write-out reads
  }
}

template <typename TG, typename TP, int R, bool MAB>
__global__ __launch_bounds__(64) void bwd_lo_multi_kernel(MultiLaunch m) {
  for (long long t = blockIdx.x; t < m.total; t += gridDim.x) {
    long long l;
    const MultiItem<BwdLoArgs>& it = item_of<BwdLoArgs>(m, t, l);
    BwdLoArgs a = it.a;
    a.U = rebase(m.ws, a.U);
    a.eps_part = rebase(m.ws, a.eps_part);
    const long long xy = (long long)it.nx * it.ny;
    bwd_lo_body<TG, TP, R, MAB>(a, (int)(l % it.nx), (int)((l / it.nx) % it.ny), (int)(l / xy));
  }
}

// One workgroup per item with a deps output: fixed-order sum of its partials.
__global__ __launch_bounds__(256) void eps_multi_kernel(const EpsItem* items, char* ws) {
  __shared__ float red[4];  // same order as eps_reduce_kernel
  const EpsItem it = items[blockIdx.x];
  const float* part = rebase(ws, it.part);
  float s = 0.f;
  for (long long q = threadIdx.x; q < it.count; q += 256) s += part[q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *it.deps = ((red[0] + red[1]) + red[2]) + red[3];
}

#include "gf_wide.h"

template <typename TG, typename TP, int MODE>
__global__ __launch_bounds__(kWideBT) void wide_stats_multi_kernel(MultiLaunch m, int R) {
  for (long long t = blockIdx.x; t < m.total; t += gridDim.x) {
    long long l;
    BwdLoArgs a;
    int nx, ny;
    if constexpr (MODE == kWideCoef) {
      const MultiItem<CoefArgs>& it = item_of<CoefArgs>(m, t, l);
      CoefArgs c = it.a;
      c.abar = rebase(m.ws, c.abar);
      c.bbar = rebase(m.ws, c.bbar);
      c.X = rebase(m.ws, c.X);
      a = wide_coef_args(c);
      nx = it.nx;
      ny = it.ny;
    } else {
      const MultiItem<BwdLoArgs>& it = item_of<BwdLoArgs>(m, t, l);
      a = it.a;
      a.U = rebase(m.ws, a.U);
      a.eps_part = rebase(m.ws, a.eps_part);
      a.X = rebase(m.ws, a.X);
      nx = it.nx;
      ny = it.ny;
    }
    const long long xy = (long long)nx * ny;
    wide_stats_body<TG, TP, MODE>(a, (int)(l % nx), (int)((l / nx) % ny), (int)(l / xy), R);
  }
}

template <typename TG, typename TP, int MODE>
__global__ __launch_bounds__(kWideBT) void wide_box_multi_kernel(MultiLaunch m, int R) {
  for (long long t = blockIdx.x; t < m.total; t += gridDim.x) {
    long long l;
    BwdLoArgs a;
    int nx, ny;
    if constexpr (MODE == kWideCoef) {
      const MultiItem<CoefArgs>& it = item_of<CoefArgs>(m, t, l);
      CoefArgs c = it.a;
      c.abar = rebase(m.ws, c.abar);
      c.bbar = rebase(m.ws, c.bbar);
      c.X = rebase(m.ws, c.X);
      a = wide_coef_args(c);
      nx = it.nx;
      ny = it.ny;
    } else {
      const MultiItem<BwdLoArgs>& it = item_of<BwdLoArgs>(m, t, l);
      a = it.a;
      a.X = rebase(m.ws, a.X);
      nx = it.nx;
      ny = it.ny;
    }
    const long long xy = (long long)nx * ny;
    wide_box_body<TG, TP, MODE>(a, (int)(l % nx), (int)((l / nx) % ny), (int)(l / xy), R);
  }
}

// ------------------------------------------------------------ dispatch

// Calls f(std::integral_constant<int, R>) for the runtime radius r.
constexpr int kMaxR = 10;
template <int R = 0, typename F>
hipError_t with_radius(int r, F&& f) {
  if constexpr (R > kMaxR) {
    return hipErrorInvalidValue;
  } else {
    if (r == R) return f(std::integral_constant<int, R>{});
    return with_radius<R + 1>(r, f);
  }
}

template <typename TG, typename TP>
hipError_t launch_coef(const Plan& p, const void* I_lo, const void* p_lo, const float* eps,
                       int eps_count, float* abar, float* bbar, float* X, hipStream_t s) {
  CoefArgs a{I_lo, p_lo, eps, eps_count, p.c, p.h, p.w, p.coTR, abar, bbar, p.lo_xcd,
             p.mean_ab ? X : nullptr};
  const dim3 grid(p.co_nx, p.co_ny, p.planes);
  if (p.wide_co) {
    const BwdLoArgs wa = wide_coef_args(a);
    prof_begin("gf_coef", s);
    hipLaunchKernelGGL((wide_stats_kernel<TG, TP, kWideCoef>), grid, dim3(kWideBT),
                       wide_lds_bytes(4), s, wa, p.r);
    prof_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !p.mean_ab) return e;
    prof_begin("gf_coef_mean", s);
    hipLaunchKernelGGL((wide_box_kernel<TG, TP, kWideCoef>), grid, dim3(kWideBT), wide_lds_bytes(2),
                       s, wa, p.r);
    prof_end(s);
    return hipGetLastError();
  }
  prof_begin("gf_coef", s);
  hipError_t err = with_radius(p.r, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    if (p.mean_ab)
      hipLaunchKernelGGL((coef_kernel<TG, TP, R, true>), grid, dim3(64), p.coLDS, s, a);
    else
      hipLaunchKernelGGL((coef_kernel<TG, TP, R, false>), grid, dim3(64), p.coLDS, s, a);
    return hipGetLastError();
  });
  prof_end(s);
  return err;
}

template <typename TG, typename TQ, int S, int VEC, bool AC>
hipError_t launch_apply_t(const Plan& p, const void* G_hi, void* q, const float* abar,
                          const float* bbar, hipStream_t s) {
  ApplyArgs a{G_hi, q, abar, bbar, p.h, p.w, p.H, p.W, p.RB,
              p.nrb, p.nxv, (long long)p.planes * p.nrb * p.nxv, p.xcd};
  const unsigned blocks = (unsigned)((a.total + 255) / 256);
  prof_begin("gf_apply", s);
  hipLaunchKernelGGL((apply_kernel<TG, TQ, S, VEC, AC>), dim3(blocks), dim3(256), 0, s, a);
  prof_end(s);
  return hipGetLastError();
}

template <typename TG, typename TD, typename TO, typename TQ, int S, int VEC, bool AC, bool FWD>
hipError_t launch_bwd_hi_t(const Plan& p, const void* G_hi, const void* dq, void* out,
                           const float* abar, float* U, const float* bbar, void* q,
                           hipStream_t s) {
  if ((p.hw > 1) != hi_merge(std::is_same<TD, float>::value, S)) return hipErrorInvalidValue;
  BwdHiArgs a{G_hi, dq, out, abar, U, p.h, p.w, p.H, p.W, p.bh, p.tw, p.nby, p.nbx, p.hw,
              p.xcd, bbar, q};
  prof_begin(FWD ? "gf_fwd_bwd_hi" : "gf_bwd_hi", s);
  hipLaunchKernelGGL((bwd_hi_kernel<TG, TD, TO, TQ, S, VEC, AC, FWD>),
                     dim3(p.nbx, p.nby, p.planes), dim3(64 * p.hw), p.hiLDS, s, a);
  prof_end(s);
  return hipGetLastError();
}

// High-res launch shapes: VEC = 4 elements per lane-load (16 bytes of
// float, 8 of a half type), or 1 when the width is not a multiple of 4.
// Wider lanes (8 half elements, or VEC = S = 8 so that a lane covers a whole
// low-res column) double the double-buffered rows held in registers and cut
// occupancy to one or two waves per SIMD; at S = 8 a lane covers half a
// low-res column and the backward flushes its row sums through LDS.
constexpr int kVec = 4;

// Calls f(integral_constant S, integral_constant VEC, integral_constant AC)
// for the plan's factor, vector width and alignment.
template <typename F>
hipError_t with_hires_shape(int S, int VEC, int ac, F&& f) {
  auto by_vec = [&](auto sc) -> hipError_t {
    auto by_ac = [&](auto vc) -> hipError_t {
      if (ac) return f(sc, vc, std::integral_constant<bool, true>{});
      return f(sc, vc, std::integral_constant<bool, false>{});
    };
    if (VEC == 1) return by_ac(std::integral_constant<int, 1>{});
    return by_ac(std::integral_constant<int, kVec>{});
  };
  switch (S) {
    case 1: return by_vec(std::integral_constant<int, 1>{});
    case 2: return by_vec(std::integral_constant<int, 2>{});
    case 4: return by_vec(std::integral_constant<int, 4>{});
    case 8: return by_vec(std::integral_constant<int, 8>{});
  }
  return hipErrorInvalidValue;
}

// Any size ratio: the general high-res kernels (VEC 4 or 1, both alignments).
template <typename F>
hipError_t with_gen_shape(int VEC, int ac, F&& f) {
  auto by_ac = [&](auto vc) -> hipError_t {
    if (ac) return f(vc, std::integral_constant<bool, true>{});
    return f(vc, std::integral_constant<bool, false>{});
  };
  if (VEC == 1) return by_ac(std::integral_constant<int, 1>{});
  return by_ac(std::integral_constant<int, kVec>{});
}

inline GenArgs gen_args(const Plan& p, const void* G_hi, const void* dq, void* out, void* q,
                        const float* abar, const float* bbar, float* V, float* U) {
  return GenArgs{G_hi, dq, out, q, abar, bbar, V, U, p.planes, p.h, p.w, p.H, p.W, p.RB,
                 p.nrb, p.nxv, 0};
}

template <typename TG, typename TQ>
hipError_t launch_apply_gen(const Plan& p, const void* G_hi, void* q, const float* abar,
                            const float* bbar, hipStream_t s) {
  GenArgs a = gen_args(p, G_hi, nullptr, nullptr, q, abar, bbar, nullptr, nullptr);
  a.total = (long long)p.planes * p.nrb * p.nxv;
  const unsigned blocks = (unsigned)((a.total + 255) / 256);
  prof_begin("gf_apply_gen", s);
  hipError_t e = with_gen_shape(p.VEC, p.ac, [&](auto vc, auto acc) {
    hipLaunchKernelGGL((apply_gen_kernel<TG, TQ, decltype(vc)::value, decltype(acc)::value>),
                       dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
  });
  prof_end(s);
  return e;
}

// Vertical then horizontal adjoint into one partial block per plane (and
// dI_h, and q with the forward).
template <typename TG, typename TD, typename TO, typename TQ>
hipError_t launch_bwd_gen(const Plan& p, const void* G_hi, const void* dq, void* out,
                          const float* abar, float* U, float* V, const float* bbar, void* q,
                          hipStream_t s) {
  GenArgs a = gen_args(p, G_hi, dq, out, q, abar, bbar, V, U);
  a.total = (long long)p.planes * p.h * p.nxv;
  prof_begin(q ? "gf_fwd_bwd_gen_rows" : "gf_bwd_gen_rows", s);
  hipError_t e = with_gen_shape(p.VEC, p.ac, [&](auto vc, auto acc) {
    constexpr int VV = decltype(vc)::value;
    constexpr bool AA = decltype(acc)::value;
    const unsigned blocks = (unsigned)((a.total + 255) / 256);
    if (q)
      hipLaunchKernelGGL((bwd_gen_rows_kernel<TG, TD, TO, TQ, VV, AA, true>), dim3(blocks),
                         dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((bwd_gen_rows_kernel<TG, TD, TO, TQ, VV, AA, false>), dim3(blocks),
                         dim3(256), 0, s, a);
    return hipGetLastError();
  });
  prof_end(s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)(((long long)p.planes * p.h * p.w + 255) / 256);
  prof_begin("gf_bwd_gen_cols", s);
  if (p.ac)
    hipLaunchKernelGGL((bwd_gen_cols_kernel<true>), dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((bwd_gen_cols_kernel<false>), dim3(blocks), dim3(256), 0, s, a);
  prof_end(s);
  return hipGetLastError();
}

template <typename TG, typename TQ>
hipError_t launch_apply(const Plan& p, const void* G_hi, void* q, const float* abar,
                        const float* bbar, hipStream_t s) {
  if (p.gen) return launch_apply_gen<TG, TQ>(p, G_hi, q, abar, bbar, s);
  return with_hires_shape(p.S, p.VEC, p.ac, [&](auto sc, auto vc, auto acc) {
    return launch_apply_t<TG, TQ, decltype(sc)::value, decltype(vc)::value, decltype(acc)::value>(
        p, G_hi, q, abar, bbar, s);
  });
}

// With q set, the fused pass: forward output and backward in one read of
// G_h and dq (bbar needed then).
// V: the general kernels' vertical adjoint (workspace at off_v; unused for
// the integer factors).
template <typename TG, typename TD, typename TO, typename TQ = TD>
hipError_t launch_bwd_hi(const Plan& p, const void* G_hi, const void* dq, void* out,
                         const float* abar, float* U, float* V, hipStream_t s,
                         const float* bbar = nullptr, void* q = nullptr) {
  if (p.gen) return launch_bwd_gen<TG, TD, TO, TQ>(p, G_hi, dq, out, abar, U, V, bbar, q, s);
  return with_hires_shape(p.S, p.VEC, p.ac, [&](auto sc, auto vc, auto acc) {
    constexpr int SS = decltype(sc)::value, VV = decltype(vc)::value;
    constexpr bool AA = decltype(acc)::value;
    if (q)
      return launch_bwd_hi_t<TG, TD, TO, TQ, SS, VV, AA, true>(p, G_hi, dq, out, abar, U, bbar,
                                                               q, s);
    return launch_bwd_hi_t<TG, TD, TO, TQ, SS, VV, AA, false>(p, G_hi, dq, out, abar, U,
                                                              nullptr, nullptr, s);
  });
}

template <typename TG, typename TP>
hipError_t launch_bwd_lo(const Plan& p, const void* G_lo, const void* p_lo, const float* eps,
                         int eps_count, const float* U, float* dG_lo, float* dp_lo,
                         float* part, float* X, hipStream_t s) {
  BwdLoArgs a{G_lo, p_lo, eps, eps_count, p.c, U, p.ubh, p.tw, p.nby, p.nbx,
              p.h, p.w, p.loTR, dG_lo, dp_lo, part, p.lo_nx, p.lo_ny, X, p.lo_xcd};
  const dim3 grid(p.lo_nx, p.lo_ny, p.planes);
  if (p.wide_lo) {
    prof_begin("gf_bwd_lo", s);
    if (p.mean_ab)
      hipLaunchKernelGGL((wide_stats_kernel<TG, TP, kWideBwdMab>), grid, dim3(kWideBT), p.loLDS, s,
                         a, p.r);
    else
      hipLaunchKernelGGL((wide_stats_kernel<TG, TP, kWideBwdPlain>), grid, dim3(kWideBT), p.loLDS,
                         s, a, p.r);
    prof_end(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin("gf_bwd_lo_out", s);
    hipLaunchKernelGGL((wide_box_kernel<TG, TP, kWideBwdMab>), grid, dim3(kWideBT),
                       wide_lds_bytes(4), s, a, p.r);
    prof_end(s);
    return hipGetLastError();
  }
  prof_begin("gf_bwd_lo", s);
  hipError_t err = with_radius(p.r, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    if (p.mean_ab)
      hipLaunchKernelGGL((bwd_lo_kernel<TG, TP, R, true>), grid, dim3(64), p.loLDS, s, a);
    else
      hipLaunchKernelGGL((bwd_lo_kernel<TG, TP, R, false>), grid, dim3(64), p.loLDS, s, a);
    return hipGetLastError();
  });
  prof_end(s);
  return err;
}

hipError_t launch_eps_reduce(const Plan& p, const float* part, int eps_count, float* deps,
                             hipStream_t s) {
  prof_begin("gf_eps_reduce", s);
  hipLaunchKernelGGL(eps_reduce_kernel, dim3(eps_count), dim3(256), 0, s, part,
                     p.lo_nx * p.lo_ny, p.c, p.n, eps_count, deps);
  prof_end(s);
  return hipGetLastError();
}

template <typename T>
hipError_t forward_t(const Plan& p, const FwdArgs& f, hipStream_t s) {
  float* abar = reinterpret_cast<float*>(f.ws + p.off_abar);
  float* bbar = reinterpret_cast<float*>(f.ws + p.off_bbar);
  hipError_t err = launch_coef<T, T>(p, f.I_lo, f.p_lo, f.eps, f.eps_count, abar, bbar,
                                     reinterpret_cast<float*>(f.ws + p.off_x), s);
  if (err != hipSuccess) return err;
  return launch_apply<T, T>(p, f.I_hi, f.q, abar, bbar, s);
}

// With b.q set, the forward runs in the same passes: the coefficient kernel
// writes bbar too and the high-res pass also writes q.
template <typename T>
hipError_t backward_t(const Plan& p, const BwdArgs& b, hipStream_t s) {
  float* abar = reinterpret_cast<float*>(b.ws + p.off_abar);
  float* bbar = b.q ? reinterpret_cast<float*>(b.ws + p.off_bbar) : nullptr;
  float* U = reinterpret_cast<float*>(b.ws + p.off_u);
  hipError_t err = launch_coef<T, T>(p, b.I_lo, b.p_lo, b.eps, b.eps_count, abar, bbar,
                                     reinterpret_cast<float*>(b.ws + p.off_x), s);
  if (err != hipSuccess) return err;
  // with the forward: one high-res pass writes q, dI_h and the partial planes
  float* V = reinterpret_cast<float*>(b.ws + p.off_v);
  err = launch_bwd_hi<T, T, T, T>(p, b.I_hi, b.dq, b.dI_hi, abar, U, V, s, bbar, b.q);
  if (err != hipSuccess) return err;
  if (!b.dI_lo && !b.dp_lo && !b.deps) return hipSuccess;
  float* part = reinterpret_cast<float*>(b.ws + p.off_eps);
  err = launch_bwd_lo<T, T>(p, b.I_lo, b.p_lo, b.eps, b.eps_count, U, b.dI_lo, b.dp_lo, part,
                            reinterpret_cast<float*>(b.ws + p.off_x), s);
  if (err != hipSuccess || !b.deps) return err;
  return launch_eps_reduce(p, part, b.eps_count, b.deps, s);
}

// ------------------------------------------------------------ batched launchers

// Per-class kernel names for the timing records (radius or factor).
#define GF_R_NAMES(base)                                                                    \
  {base "_r0", base "_r1", base "_r2", base "_r3", base "_r4", base "_r5", base "_r6",      \
   base "_r7", base "_r8", base "_r9", base "_r10"}
__host__ inline const char* class_name_r(int kind, int R) {
  static const char* coef[] = GF_R_NAMES("gf_coef_multi");
  static const char* lo[] = GF_R_NAMES("gf_bwd_lo_multi");
  if (R < 0 || R > 10) return kind == kClassCoef ? "gf_coef_multi" : "gf_bwd_lo_multi";
  return kind == kClassCoef ? coef[R] : lo[R];
}
#undef GF_R_NAMES
__host__ inline const char* class_name_s(int kind, int S) {
  const int k = S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : 3;
  static const char* apply[] = {"gf_apply_multi_s1", "gf_apply_multi_s2", "gf_apply_multi_s4",
                                "gf_apply_multi_s8"};
  static const char* hi[] = {"gf_bwd_hi_multi_s1", "gf_bwd_hi_multi_s2", "gf_bwd_hi_multi_s4",
                             "gf_bwd_hi_multi_s8"};
  return kind == kClassApply ? apply[k] : hi[k];
}

template <typename TG, typename TP>
hipError_t launch_coef_multi(const BatchClass& c, char* ws, hipStream_t s) {
  MultiLaunch m = c.m;
  m.ws = ws;
  prof_begin(class_name_r(kClassCoef, c.R), s);
  if (c.wide) {
    const dim3 g(m.grid);
    hipLaunchKernelGGL((wide_stats_multi_kernel<TG, TP, kWideCoef>), g, dim3(kWideBT),
                       wide_lds_bytes(4), s, m, c.R);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && c.MAB) {
      hipLaunchKernelGGL((wide_box_multi_kernel<TG, TP, kWideCoef>), g, dim3(kWideBT),
                         wide_lds_bytes(2), s, m, c.R);
      e = hipGetLastError();
    }
    prof_end(s);
    return e;
  }
  hipError_t err = with_radius(c.R, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    if (c.MAB)
      hipLaunchKernelGGL((coef_multi_kernel<TG, TP, R, true>), dim3(m.grid), dim3(64), c.lds, s, m);
    else
      hipLaunchKernelGGL((coef_multi_kernel<TG, TP, R, false>), dim3(m.grid), dim3(64), c.lds, s,
                         m);
    return hipGetLastError();
  });
  prof_end(s);
  return err;
}

template <typename TG, typename TP>
hipError_t launch_bwd_lo_multi(const BatchClass& c, char* ws, hipStream_t s) {
  MultiLaunch m = c.m;
  m.ws = ws;
  prof_begin(class_name_r(kClassBwdLo, c.R), s);
  if (c.wide) {
    const dim3 g(m.grid);
    if (c.MAB)
      hipLaunchKernelGGL((wide_stats_multi_kernel<TG, TP, kWideBwdMab>), g, dim3(kWideBT), c.lds, s,
                         m, c.R);
    else
      hipLaunchKernelGGL((wide_stats_multi_kernel<TG, TP, kWideBwdPlain>), g, dim3(kWideBT), c.lds,
                         s, m, c.R);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL((wide_box_multi_kernel<TG, TP, kWideBwdMab>), g, dim3(kWideBT),
                         wide_lds_bytes(4), s, m, c.R);
      e = hipGetLastError();
    }
    prof_end(s);
    return e;
  }
  hipError_t err = with_radius(c.R, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    if (c.MAB)
      hipLaunchKernelGGL((bwd_lo_multi_kernel<TG, TP, R, true>), dim3(m.grid), dim3(64), c.lds, s,
                         m);
    else
      hipLaunchKernelGGL((bwd_lo_multi_kernel<TG, TP, R, false>), dim3(m.grid), dim3(64), c.lds,
                         s, m);
    return hipGetLastError();
  });
  prof_end(s);
  return err;
}

template <typename TG, typename TQ>
hipError_t launch_apply_multi(const BatchClass& c, char* ws, hipStream_t s) {
  MultiLaunch m = c.m;
  m.ws = ws;
  prof_begin(class_name_s(kClassApply, c.S), s);
  const hipError_t e = with_hires_shape(c.S, c.VEC, c.AC, [&](auto sc, auto vc, auto acc) {
    hipLaunchKernelGGL((apply_multi_kernel<TG, TQ, decltype(sc)::value, decltype(vc)::value,
                                           decltype(acc)::value>),
                       dim3(m.grid), dim3(256), 0, s, m);
    return hipGetLastError();
  });
  prof_end(s);
  return e;
}

template <typename TG, typename TD, typename TO>
hipError_t launch_bwd_hi_multi(const BatchClass& c, char* ws, hipStream_t s, bool fwd) {
  MultiLaunch m = c.m;
  m.ws = ws;
  prof_begin(class_name_s(kClassBwdHi, c.S), s);
  const hipError_t e = with_hires_shape(c.S, c.VEC, c.AC, [&](auto sc, auto vc, auto acc) {
    constexpr int SS = decltype(sc)::value, VV = decltype(vc)::value;
    constexpr bool AA = decltype(acc)::value;
    if ((c.hw > 1) != hi_merge(std::is_same<TD, float>::value, SS)) return hipErrorInvalidValue;
    if (fwd)
      hipLaunchKernelGGL((bwd_hi_multi_kernel<TG, TD, TO, TD, SS, VV, AA, true>), dim3(m.grid),
                         dim3(64 * c.hw), c.lds, s, m);
    else
      hipLaunchKernelGGL((bwd_hi_multi_kernel<TG, TD, TO, TD, SS, VV, AA, false>), dim3(m.grid),
                         dim3(64 * c.hw), c.lds, s, m);
    return hipGetLastError();
  });
  prof_end(s);
  return e;
}

// Forward (mode bit 1) and/or backward (bit 2) of every item; with both,
// the coefficients are computed once.
template <typename T>
hipError_t batched_t(const BatchLaunch& b, int mode, char* ws, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (const BatchClass& c : b.coef)
    if ((e = launch_coef_multi<T, T>(c, ws, s)) != hipSuccess) return e;
  // forward and backward: one high-res pass writes q, dI_h and the partials
  const bool fused = (mode & GF_RUN_FORWARD) && (mode & GF_RUN_BACKWARD);
  if ((mode & GF_RUN_FORWARD) && !fused)
    for (const BatchClass& c : b.apply)
      if ((e = launch_apply_multi<T, T>(c, ws, s)) != hipSuccess) return e;
  if (mode & GF_RUN_BACKWARD) {
    for (const BatchClass& c : b.bwd_hi)
      if ((e = launch_bwd_hi_multi<T, T, T>(c, ws, s, fused)) != hipSuccess) return e;
    for (const BatchClass& c : b.bwd_lo)
      if ((e = launch_bwd_lo_multi<T, T>(c, ws, s)) != hipSuccess) return e;
    if (b.eps_count > 0) {
      prof_begin("gf_eps_multi", s);
      hipLaunchKernelGGL(eps_multi_kernel, dim3(b.eps_count), dim3(256), 0, s, b.eps_items, ws);
      prof_end(s);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace
}  // namespace gf
