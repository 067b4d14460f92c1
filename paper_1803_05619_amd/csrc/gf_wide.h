// Wide low-res walkers for large radii: the backward from radius
// wide_bwd_min_r(), the coefficients from wide_coef_min_r() (included by
// gf_kernels.h inside its namespace; the helpers they use are defined there).
//
// The column walkers of gf_kernels.h form every window with direct
// (2r + 1)-tap sums, down the column and across the lanes, and keep 64 - 4r
// (64 - 2r without the A/b window mean) of a wave's 64 columns: their work
// per output grows with r, and at r = 8 half the lanes are halo.  Here a
// workgroup of 256 threads owns a strip of 256 input columns (256 - 2r
// outputs) and walks down its rows in blocks of kWideB rows; every box sum
// is a running sum, so the work per output does not depend on r:
//   - down the walk, each thread keeps its column's running sums over the
//     last 2r + 1 rows (add the row that enters, subtract the row that
//     leaves; both rows' loads are issued one block ahead, the leaving one
//     is an L2 hit);
//   - across the strip, the column sums of a block's rows go to LDS and the
//     threads, re-partitioned as (row, run of kWideSeg consecutive columns),
//     slide a running sum along the row.
// The sums run in FP64: the guide and input are recentred by a reference
// value, and with sums of squares exact to ~1e-16 relative the variance
// E[g^2] - E[g]^2 loses nothing to cancellation; the running sums do not
// drift along the walk (FP64 adds run at the unpacked FP32 rate on MI355X).
// A nested box (the window mean of A and b, and the backward's transposed
// box of X) is a second pass over a plane that the first writes, rather
// than a ring of rows in LDS.

constexpr int kWideSeg = 4;  // columns per thread in the horizontal passes
static_assert(wide_row(64) == 64 + 64 / kWideSeg, "the planner's LDS rows pad one per kWideSeg");

// In-image rows (or columns) of the window of radius R centred at t.
__device__ __forceinline__ int clip_count(int t, int R, int n) {
  return min(t + R, n - 1) - max(t - R, 0) + 1;
}

// LDS rows of the horizontal passes: one array per FP64 quantity (structure
// of arrays), each row of NT columns padded by one element per kWideSeg
// columns.  Those passes' threads read columns kWideSeg apart; unpadded, the
// lanes of a wave would fall on a few banks, padded (a stride of 5 FP64
// elements) 32 lanes cover 32 distinct bank pairs.
__device__ __forceinline__ int wp(int c) { return c + c / kWideSeg; }

struct WRows {
  double* base;
  int row;  // padded row length
  __device__ __forceinline__ double* q(int ch, int d) const { return base + (ch * kWideB + d) * row; }
  __device__ __forceinline__ double4 get4(int d, int c) const {
    const int o = wp(c);
    return make_double4(q(0, d)[o], q(1, d)[o], q(2, d)[o], q(3, d)[o]);
  }
  __device__ __forceinline__ void put4(int d, int c, double4 v) const {
    const int o = wp(c);
    q(0, d)[o] = v.x;
    q(1, d)[o] = v.y;
    q(2, d)[o] = v.z;
    q(3, d)[o] = v.w;
  }
  __device__ __forceinline__ double2 get2(int ch, int d, int c) const {
    const int o = wp(c);
    return make_double2(q(ch, d)[o], q(ch + 1, d)[o]);
  }
  __device__ __forceinline__ void put2(int ch, int d, int c, double2 v) const {
    const int o = wp(c);
    q(ch, d)[o] = v.x;
    q(ch + 1, d)[o] = v.y;
  }
};

__device__ __forceinline__ double4 d4add(double4 a, double4 b) {
  return make_double4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ double4 d4sub(double4 a, double4 b) {
  return make_double4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}

// ------------------------------------------------------------ the two passes
//
// wide_stats  per pixel: the window statistics and
//             - backward: dA and db (the box sums of dAbar/N and dbbar/N with
//               the window mean, else the gathered values themselves) and the
//               adjoint quantities X = (dmean_I, dmean_p, dcov, dvar) / N,
//               written to a plane (16 bytes per pixel) by the strip that
//               owns the pixel; the strip's sum of dvar goes to the deps
//               partials;
//             - coefficients: A and b, written to a plane (8 bytes per
//               pixel) with the window mean, else as the outputs;
// wide_box    box sums of that plane: dI_l = B0 + 2 B3 g' + B2 p' and
//             dp_l = B1 + B2 g' (backward), or Abar and bbar (coefficients).
// Both recentre the guide and input by the plane's value at its centre
// pixel, so that the second pass's g', p' match the first pass's means.
constexpr int kWideBT = 256;  // threads (input columns) of the backward walkers

template <typename TG, typename TP>
__device__ __forceinline__ void plane_centre(const BwdLoArgs& a, const TG* G, const TP* P,
                                             float& cg, float& cp) {
  const size_t o = (size_t)(a.h / 2) * a.w + a.w / 2;
  cg = to_f(G[o]);
  cp = to_f(P[o]);
}

// Pass modes: the backward with and without the A/b window mean, and the
// coefficients (pass 1 writes (A, b) per pixel, as a float2 plane in X with
// the window mean, else straight to the Abar and bbar planes, which the
// coefficient passes receive as dI_lo and dp_lo).
enum { kWideBwdMab = 0, kWideBwdPlain = 1, kWideCoef = 2 };

// The backward's X plane in FP64 (32 bytes per pixel) for FP32 I/O, else
// FP32 (16 bytes).  X's entries are differences of terms that grow with
// 1 / (var + eps) (dmean_p = db - dcov mean_I', with dcov up to |dA| / eps),
// and the second pass forms dI_l, dp_l as B1 + B2 g' from their window sums:
// where a flat region lies away from the plane's reference value these
// terms cancel to a few parts in 1e4, so with FP32 X the rounding of each
// term shows (2e-4 of max |dp_l| at eps = 1e-8 on FP32 I/O).  With FP64 X
// and an FP64 epilogue and combination only the final rounding to FP32
// remains.  For the half types the I/O rounding dominates and X stays FP32.
template <typename TP, int MODE>
__device__ __host__ constexpr bool wide_x64() {
  return MODE != kWideCoef && std::is_same<TP, float>::value;
}

template <typename TG, typename TP, int MODE>
__device__ __forceinline__ void wide_stats_body(const BwdLoArgs& a, const int bx, const int by,
                                                const int plane, const int R) {
  constexpr bool MAB = MODE == kWideBwdMab, COEF = MODE == kWideCoef;
  constexpr bool X64 = wide_x64<TP, MODE>();
  constexpr int kTPR = kWideBT / kWideB;
  extern __shared__ double4 wlds[];
  // padded rows of (g', p', g'^2, g'p') and (dAbar/N, dbbar/N) column sums
  constexpr int ROW = kWideBT + kWideBT / kWideSeg;
  const WRows CS{reinterpret_cast<double*>(wlds), ROW};
  __shared__ float red[kWideBT / 64];
  const int K = 2 * R + 1, TWo = kWideBT - 2 * R;
  const int t = threadIdx.x;
  const int h = a.h, w = a.w;
  const float e = a.eps[a.eps_count == 1 ? 0 : plane / a.c];
  const int j0 = bx * TWo, jl = j0 - R, j = jl + t;
  const bool colin = (unsigned)j < (unsigned)w;
  const int i0 = by * a.TR, i1 = min(i0 + a.TR, h);
  const int x0 = i0 - R, xend = i1 + R;
  const size_t pofs = (size_t)plane * h * w, hw = (size_t)h * w;
  const TG* G = reinterpret_cast<const TG*>(a.I_lo) + pofs;
  const TP* P = reinterpret_cast<const TP*>(a.p_lo) + pofs;
  const __amdgpu_buffer_rsrc_t gR = buf_rsrc(G, hw * sizeof(TG));
  const __amdgpu_buffer_rsrc_t pR = buf_rsrc(P, hw * sizeof(TP));
  float cg, cp;
  plane_centre(a, G, P, cg, cp);
  const double cgd = cg, cpd = cp;  // recentring in FP64: exact for every I/O type
  const int jcl = min(max(j, 0), w - 1);
  const unsigned jg = (unsigned)jcl * sizeof(TG), jp = (unsigned)jcl * sizeof(TP);
  // the upstream partial planes (dAbar, dbbar of the high-res backward)
  const size_t UP = COEF ? 0 : (size_t)(a.bh + 2) * (a.tw + 2);
  const size_t uplane = COEF ? 0 : (size_t)a.nby * a.nbx * 2 * UP;
  const __amdgpu_buffer_rsrc_t uR = buf_rsrc(COEF ? nullptr : a.U + (size_t)plane * uplane, uplane * 4);
  const unsigned ub = (unsigned)UP * 4u;
  const UCol ucol = COEF ? UCol{0u, 0u, 0.f} : u_col(a, jcl);
  const unsigned bmul = COEF ? 0u : 0xffffffffu / (unsigned)a.bh + 1u;
  const int ncol_j = clip_count(jcl, R, w);
  // (dAbar, dbbar) at (x, j), divided by the window count with the window
  // mean (f_mu^T(y) is the box sum of y / N); zero outside the image
  // raw loads of one block row, issued one block ahead: the guide and
  // input of the entering row x and of the leaving row x - K, and the
  // partial-plane gathers of x and x - K (with the window mean) or of the
  // statistics row x - R (without)
  struct Q {
    TG g0, g1;
    TP p0, p1;
    URaw z0, z1;
    float wb0, wb1;
  };
  Q q[kWideB];
  auto fetch = [&](int xb) __attribute__((always_inline)) {
#pragma unroll
    for (int d = 0; d < kWideB; ++d) {
      const int x = xb + d, xl = x - K;
      const unsigned o = (unsigned)(min(max(x, 0), h - 1) * w);
      const unsigned ol = (unsigned)(min(max(xl, 0), h - 1) * w);
      q[d].g0 = buf_ld<TG>(gR, jg, o * (unsigned)sizeof(TG));
      q[d].p0 = buf_ld<TP>(pR, jp, o * (unsigned)sizeof(TP));
      q[d].g1 = buf_ld<TG>(gR, jg, ol * (unsigned)sizeof(TG));
      q[d].p1 = buf_ld<TP>(pR, jp, ol * (unsigned)sizeof(TP));
      if constexpr (COEF) continue;
      const URow r0 = u_row(a, bmul, min(max(MAB ? x : x - R, 0), h - 1));
      q[d].z0 = gather_u_raw(uR, ub, r0, ucol);
      q[d].wb0 = r0.wb;
      if (MAB) {
        const URow r1 = u_row(a, bmul, min(max(xl, 0), h - 1));
        q[d].z1 = gather_u_raw(uR, ub, r1, ucol);
        q[d].wb1 = r1.wb;
      }
    }
  };
  // (dAbar, dbbar) at (x, j) from its gathered partials, divided by the
  // window count with the window mean (f_mu^T(y) is the box sum of y / N);
  // zero outside the image
  auto upstream = [&](int x, const URaw& z, float wb) __attribute__((always_inline)) {
    const float wc = ucol.wc;
    float u = (z.a00 + wc * z.a01) + wb * (z.a10 + wc * z.a11);
    float v = (z.v00 + wc * z.v01) + wb * (z.v10 + wc * z.v11);
    if (MAB) {
      const float invN = 1.f / (float)(clip_count(min(max(x, 0), h - 1), R, h) * ncol_j);
      u *= invN;
      v *= invN;
    }
    const bool ok = colin && row_ok(x, h);
    return ok ? make_float2(u, v) : make_float2(0.f, 0.f);
  };
  double sg = 0.0, sp = 0.0, sgg = 0.0, sgp = 0.0, su = 0.0, sv = 0.0;
  float deps_acc = 0.f;
  fetch(x0);
  for (int xb = x0; xb < xend; xb += kWideB) {
#pragma unroll
    for (int d = 0; d < kWideB; ++d) {
      const int x = xb + d, xl = x - K;
      if (x < xend) {
        const bool ok = colin && row_ok(x, h);
        const bool okl = colin && xl >= x0 && row_ok(xl, h);
        const double g = ok ? (double)to_f(q[d].g0) - cgd : 0.0;
        const double p = ok ? (double)to_f(q[d].p0) - cpd : 0.0;
        const double g2 = okl ? (double)to_f(q[d].g1) - cgd : 0.0;
        const double p2 = okl ? (double)to_f(q[d].p1) - cpd : 0.0;
        sg += g - g2;
        sp += p - p2;
        sgg += g * g - g2 * g2;
        sgp += g * p - g2 * p2;
        if constexpr (COEF) {
        } else if (MAB) {
          const float2 in = upstream(x, q[d].z0, q[d].wb0);
          const float2 out = xl >= x0 ? upstream(xl, q[d].z1, q[d].wb1) : make_float2(0.f, 0.f);
          su += (double)in.x - (double)out.x;
          sv += (double)in.y - (double)out.y;
        } else {
          const float2 c = upstream(x - R, q[d].z0, q[d].wb0);  // the statistics row's own
          su = c.x;
          sv = c.y;
        }
      }
      CS.put4(d, t, make_double4(sg, sp, sgg, sgp));  // row rc = x - R
      if constexpr (!COEF) CS.put2(4, d, t, make_double2(su, sv));
    }
    fetch(xb + kWideB);
    __syncthreads();
    {
      const int d = t / kTPR, s = t % kTPR;
      const int rc = xb + d - R;
      const int c0 = R + s * kWideSeg;
      if (xb + d < xend && rc >= i0 && rc < i1 && c0 < kWideBT - R) {
        const int nrow = clip_count(rc, R, h);
        double4 W = CS.get4(d, c0 - R), W2 = make_double4(0.0, 0.0, 0.0, 0.0);
        double2 U = MAB ? CS.get2(4, d, c0 - R) : make_double2(0.0, 0.0), U2 = make_double2(0.0, 0.0);
        for (int k = c0 - R + 1; k < c0 + R; k += 2) {
          W = d4add(W, CS.get4(d, k));
          W2 = d4add(W2, CS.get4(d, k + 1));
          if (MAB) {
            const double2 v = CS.get2(4, d, k), v2 = CS.get2(4, d, k + 1);
            U.x += v.x;
            U.y += v.y;
            U2.x += v2.x;
            U2.y += v2.y;
          }
        }
        W = d4add(W, W2);
        U.x += U2.x;
        U.y += U2.y;
        float4* Xrow = reinterpret_cast<float4*>(a.X + 4 * (pofs + (size_t)rc * w));
        double4* X64row = reinterpret_cast<double4*>(a.X + 8 * (pofs + (size_t)rc * w));
        float2* ABrow = reinterpret_cast<float2*>(a.X + 2 * (pofs + (size_t)rc * w));
#pragma unroll
        for (int uu = 0; uu < kWideSeg; ++uu) {
          const int c = c0 + uu;
          if (c >= kWideBT - R) break;
          if (uu > 0) {
            W = d4sub(d4add(W, CS.get4(d, c + R)), CS.get4(d, c - R - 1));
            if (MAB) {
              const double2 in = CS.get2(4, d, c + R), out = CS.get2(4, d, c - R - 1);
              U.x += in.x - out.x;
              U.y += in.y - out.y;
            }
          }
          const int jj = jl + c;
          if ((unsigned)jj < (unsigned)w) {
            const int N = nrow * clip_count(jj, R, w);
            const double Nd = (double)N;
            const float invN = 1.f / (float)N;
            // a one-pixel window (radius 0) has var = cov = 0 exactly, which
            // the running sums only approach (their rounding along the walk)
            const bool pix = R == 0;
            const float var = pix ? 0.f : (float)(W.z * Nd - W.x * W.x) * (invN * invN);
            const float cov = pix ? 0.f : (float)(W.w * Nd - W.x * W.y) * (invN * invN);
            const float mg = (float)W.x * invN, mp = (float)W.y * invN;
            if constexpr (COEF) {
              const float den = var + e;
              const float A = den > 0.f ? cov * rcp(den) : 0.f;
              const float B = (mp + cp) - A * (mg + cg);
              if (a.X) {
                ABrow[jj] = make_float2(A, B);
              } else {
                a.dI_lo[pofs + (size_t)rc * w + jj] = A;
                if (a.dp_lo) a.dp_lo[pofs + (size_t)rc * w + jj] = B;
              }
              continue;
            }
            // dA, db: the box sums of dAbar/N, dbbar/N (or the values)
            const double2 uc = MAB ? U : CS.get2(4, d, c);
            if constexpr (X64) {
              const double invNd = 1.0 / Nd;
              const double mgd = W.x * invNd, mpd = W.y * invNd;
              const double vard = pix ? 0.0 : (W.z * Nd - W.x * W.x) * (invNd * invNd);
              const double covd = pix ? 0.0 : (W.w * Nd - W.x * W.y) * (invNd * invNd);
              const double den = vard + (double)e;
              const double rden = den > 0.0 ? 1.0 / den : 0.0;  // A := 0 when var + eps == 0
              const double A = covd * rden;
              const double dAt = uc.x - uc.y * (mgd + cgd);
              // one-pixel windows: var and cov do not depend on the pixel
              const double dcov = pix ? 0.0 : dAt * rden;
              const double dvar = pix ? 0.0 : -dAt * A * rden;
              const double dmI = -uc.y * A - dcov * mpd - 2.0 * dvar * mgd;
              const double dmP = uc.y - dcov * mgd;
              deps_acc += (float)dvar;
              X64row[jj] = make_double4(dmI * invNd, dmP * invNd, dcov * invNd, dvar * invNd);
              continue;
            }
            const float dA = (float)uc.x, db = (float)uc.y;
            const float den = var + e;
            const float rden = den > 0.f ? rcp(den) : 0.f;  // A := 0 when var + eps == 0
            const float A = cov * rden;
            const float dAt = dA - db * (mg + cg);
            // one-pixel windows: var and cov do not depend on the pixel
            const float dcov = pix ? 0.f : dAt * rden;
            const float dvar = pix ? 0.f : -dAt * A * rden;
            const float dmI = -db * A - dcov * mp - 2.f * dvar * mg;
            const float dmP = db - dcov * mg;
            deps_acc += dvar;
            Xrow[jj] = make_float4(dmI * invN, dmP * invN, dcov * invN, dvar * invN);
          }
        }
      }
    }
    __syncthreads();
  }
  if constexpr (COEF) return;
  // fixed-order workgroup sum of the strip's deps contribution
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) deps_acc += __shfl_xor(deps_acc, off);
  if ((t & 63) == 0) red[t >> 6] = deps_acc;
  __syncthreads();
  if (t == 0) {
    float s = red[0];
#pragma unroll
    for (int k = 1; k < kWideBT / 64; ++k) s += red[k];
    a.eps_part[((size_t)plane * a.pny + by) * a.pnx + bx] = s;
  }
}

// Pass 2: box sums of the first pass's plane.  Backward: the four X
// quantities give dI_l = B0 + 2 B3 g' + B2 p' and dp_l = B1 + B2 g'.
// Coefficients: the two (A, b) quantities, divided by the window's count,
// give Abar and bbar (written to dI_lo and dp_lo).
template <typename TG, typename TP, int MODE>
__device__ __forceinline__ void wide_box_body(const BwdLoArgs& a, const int bx, const int by,
                                              const int plane, const int R) {
  constexpr bool COEF = MODE == kWideCoef;
  constexpr bool X64 = wide_x64<TP, MODE>();
  using XV = typename std::conditional<X64, double4, float4>::type;
  constexpr int kTPR = kWideBT / kWideB;
  extern __shared__ double4 wlds[];
  constexpr int ROW = kWideBT + kWideBT / kWideSeg;
  const WRows CS{reinterpret_cast<double*>(wlds), ROW};  // padded rows of column sums
  const int K = 2 * R + 1, TWo = kWideBT - 2 * R;
  const int t = threadIdx.x;
  const int h = a.h, w = a.w;
  const int j0 = bx * TWo, jl = j0 - R, j = jl + t;
  const bool colin = (unsigned)j < (unsigned)w;
  const int i0 = by * a.TR, i1 = min(i0 + a.TR, h);
  const int x0 = i0 - R, xend = i1 + R;
  const size_t pofs = (size_t)plane * h * w;
  const TG* G = reinterpret_cast<const TG*>(a.I_lo) + pofs;
  const TP* P = reinterpret_cast<const TP*>(a.p_lo) + pofs;
  float cg, cp;
  plane_centre(a, G, P, cg, cp);
  const XV* X4 = reinterpret_cast<const XV*>(a.X) + pofs;
  const float2* X2 = reinterpret_cast<const float2*>(a.X) + pofs;
  const int jcl = min(max(j, 0), w - 1);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  // the plane's entering and leaving rows, one block ahead
  XV qi[kWideB], qo[kWideB];
  auto fetch = [&](int xb) __attribute__((always_inline)) {
#pragma unroll
    for (int d = 0; d < kWideB; ++d) {
      const size_t oi = (size_t)min(max(xb + d, 0), h - 1) * w + jcl;
      const size_t oo = (size_t)min(max(xb + d - K, 0), h - 1) * w + jcl;
      if constexpr (COEF) {
        const float2 vi = X2[oi], vo = X2[oo];
        qi[d] = XV{vi.x, vi.y, 0.f, 0.f};
        qo[d] = XV{vo.x, vo.y, 0.f, 0.f};
      } else {
        qi[d] = X4[oi];
        qo[d] = X4[oo];
      }
    }
  };
  fetch(x0);
  for (int xb = x0; xb < xend; xb += kWideB) {
#pragma unroll
    for (int d = 0; d < kWideB; ++d) {
      const int x = xb + d, xl = x - K;
      if (x < xend) {
        const XV in = qi[d], out = qo[d];
        const bool ok = colin && row_ok(x, h);
        const bool okl = colin && xl >= x0 && row_ok(xl, h);
        if (ok) {
          s0 += (double)in.x;
          s1 += (double)in.y;
          if (!COEF) {
            s2 += (double)in.z;
            s3 += (double)in.w;
          }
        }
        if (okl) {
          s0 -= (double)out.x;
          s1 -= (double)out.y;
          if (!COEF) {
            s2 -= (double)out.z;
            s3 -= (double)out.w;
          }
        }
      }
      if constexpr (COEF)
        CS.put2(0, d, t, make_double2(s0, s1));  // row rx = x - R
      else
        CS.put4(d, t, make_double4(s0, s1, s2, s3));
    }
    fetch(xb + kWideB);
    __syncthreads();
    {
      const int d = t / kTPR, s = t % kTPR;
      const int rx = xb + d - R;
      const int c0 = R + s * kWideSeg;
      if (xb + d < xend && rx >= i0 && rx < i1 && c0 < kWideBT - R) {
        auto get = [&](int c) __attribute__((always_inline)) {
          if constexpr (COEF) {
            const double2 v = CS.get2(0, d, c);
            return make_double4(v.x, v.y, 0.0, 0.0);
          } else {
            return CS.get4(d, c);
          }
        };
        double4 W = get(c0 - R), W2 = make_double4(0.0, 0.0, 0.0, 0.0);
        for (int k = c0 - R + 1; k < c0 + R; k += 2) {
          W = d4add(W, get(k));
          W2 = d4add(W2, get(k + 1));
        }
        W = d4add(W, W2);
        const int nrow = clip_count(rx, R, h);
#pragma unroll
        for (int u = 0; u < kWideSeg; ++u) {
          const int c = c0 + u;
          if (c >= kWideBT - R) break;
          if (u > 0) W = d4sub(d4add(W, get(c + R)), get(c - R - 1));
          const int jj = jl + c;
          if ((unsigned)jj < (unsigned)w) {
            const size_t o = (size_t)rx * w + jj;
            if constexpr (COEF) {
              const float invN = 1.f / (float)(nrow * clip_count(jj, R, w));
              a.dI_lo[pofs + o] = (float)W.x * invN;
              if (a.dp_lo) a.dp_lo[pofs + o] = (float)W.y * invN;
            } else if constexpr (X64) {
              const double g = (double)to_f(G[o]) - (double)cg;
              const double p = (double)to_f(P[o]) - (double)cp;
              if (a.dI_lo) a.dI_lo[pofs + o] = (float)(W.x + 2.0 * W.w * g + W.z * p);
              if (a.dp_lo) a.dp_lo[pofs + o] = (float)(W.y + W.z * g);
            } else {
              const float g = to_f(G[o]) - cg, p = to_f(P[o]) - cp;
              const float B0 = (float)W.x, B1 = (float)W.y, B2 = (float)W.z, B3 = (float)W.w;
              if (a.dI_lo) a.dI_lo[pofs + o] = B0 + 2.f * B3 * g + B2 * p;
              if (a.dp_lo) a.dp_lo[pofs + o] = B1 + B2 * g;
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename TG, typename TP, int MODE>
__global__ __launch_bounds__(kWideBT) void wide_stats_kernel(BwdLoArgs a, int R) {
  wide_stats_body<TG, TP, MODE>(a, blockIdx.x, blockIdx.y, blockIdx.z, R);
}
template <typename TG, typename TP, int MODE>
__global__ __launch_bounds__(kWideBT) void wide_box_kernel(BwdLoArgs a, int R) {
  wide_box_body<TG, TP, MODE>(a, blockIdx.x, blockIdx.y, blockIdx.z, R);
}

// The coefficient passes' arguments from the coefficient walker's: the
// outputs Abar, bbar travel as dI_lo, dp_lo, the (A, b) plane as X.
__device__ __host__ __forceinline__ BwdLoArgs wide_coef_args(const CoefArgs& c) {
  BwdLoArgs a{};
  a.I_lo = c.I_lo;
  a.p_lo = c.p_lo;
  a.eps = c.eps;
  a.eps_count = c.eps_count;
  a.c = c.c;
  a.h = c.h;
  a.w = c.w;
  a.TR = c.TR;
  a.dI_lo = c.abar;
  a.dp_lo = c.bbar;
  a.X = c.X;
  return a;
}
