/*
 * FP64 CPU oracle of the convolutional guided filtering layer (Wu et al.,
 * "Fast End-to-End Trainable Guided Filter", arXiv 1803.05619, Sec. III-E,
 * the layer of the DGF_b^c variant, Sec. IV-B).
 *
 * TEST INFRASTRUCTURE ONLY (like gf_oracle.c): only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark use it; it shares no
 * code, header or table with the HIP library.
 *
 * The paper replaces the mean filter f_mu by dilated convolutions (r is
 * their dilation rate) and the local linear model A = cov / (var + eps) by a
 * block of pointwise convolutions, and drops eps; it gives neither the
 * normalisation of the convolutions nor the block's depth and widths.
 * Reading taken here, per image and channel k (guide channel k filters
 * output channel k):
 *
 *   f_d,k(X)(m) = sum_t D_k[t] X(m + r t) / sum_t D_k[t] [m + r t in image]
 *       a 3x3 depthwise convolution with dilation r (taps t in {-1,0,1}^2,
 *       one learned 3x3 kernel per channel, zero outside the image),
 *       normalised by the same convolution of the all-ones image, so that
 *       uniform weights at r = 1 give the clipped box mean f_mu exactly;
 *   mean_I = f_d(I), mean_p = f_d(p),
 *   cov = f_d(I p) - mean_I mean_p, var = f_d(I I) - mean_I^2
 *       (evaluated in the equal two-pass form sum_t a_t (I_t - mean_I)(...)
 *       with a_t = D_k[t] / N(m));
 *   A = W3 lrelu(W2 lrelu(W1 u)), u = (cov_0..cov_{c-1}, var_0..var_{c-1})
 *       per pixel: the pointwise block (2c -> K -> K -> c, no biases, leaky
 *       ReLU with the given slope; derivative `slope` at y <= 0);
 *   b = mean_p - A mean_I;
 *   Abar = f_d(A), bbar = f_d(b) (mean_ab = 1) or A, b (mean_ab = 0);
 *   q = f_up(Abar) I_h + f_up(bbar) (bilinear, as in gf_oracle.c).
 *
 * The backward differentiates exactly these loops, in scatter form (each
 * loop the transpose of a forward loop), and returns the gradients of
 * <q, dq> with respect to I_l, p_l, I_h and every parameter, plus, per
 * parameter, the sum of the magnitudes of the per-pixel terms it adds up
 * (the rounding scale of a computed parameter gradient).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "gf_oracle.h"

static int cimin(int a, int b) { return a < b ? a : b; }

static double lrelu(double y, double s) { return y > 0.0 ? y : s * y; }
static double lrelu_d(double y, double s) { return y > 0.0 ? 1.0 : s; }

/* bilinear taps (half-pixel or corner-aligned), as in gf_oracle.c */
static void ctap(int d, int D, int S, int ac, int *t0, int *t1, double *wt) {
  double src;
  if (ac) {
    src = (D > 1) ? (double)d * (double)(S - 1) / (double)(D - 1) : 0.0;
  } else {
    src = ((double)d + 0.5) * (double)S / (double)D - 0.5;
    if (src < 0.0) src = 0.0;
  }
  int i0 = (int)floor(src);
  if (i0 > S - 1) i0 = S - 1;
  *t0 = i0;
  *t1 = cimin(i0 + 1, S - 1);
  *wt = src - (double)i0;
}

typedef struct {
  int h, w, r;
} cgeom_t;

/* tap t = 0..8 of pixel (i, j): (ty, tx) = (t / 3 - 1, t % 3 - 1); returns
 * the flat index of the tapped pixel or -1 outside the image */
static long tap_at(const cgeom_t *g, int i, int j, int t) {
  const int u = i + (t / 3 - 1) * g->r, v = j + (t % 3 - 1) * g->r;
  if (u < 0 || u >= g->h || v < 0 || v >= g->w) return -1;
  return (long)u * g->w + v;
}

/* normaliser N(m) = sum of the in-image taps' weights */
static double tap_norm(const cgeom_t *g, const double *Dk, int i, int j) {
  double s = 0.0;
  for (int t = 0; t < 9; ++t)
    if (tap_at(g, i, j, t) >= 0) s += Dk[t];
  return s;
}

/* Y = f_d(X) for one plane */
static void fd_plane(const cgeom_t *g, const double *Dk, const double *X, double *Y) {
  for (int i = 0; i < g->h; ++i)
    for (int j = 0; j < g->w; ++j) {
      double s = 0.0;
      for (int t = 0; t < 9; ++t) {
        const long o = tap_at(g, i, j, t);
        if (o >= 0) s += Dk[t] * X[o];
      }
      Y[(long)i * g->w + j] = s / tap_norm(g, Dk, i, j);
    }
}

/* per-channel statistics of one image: mean_I, mean_p, cov, var [c][P] */
static void conv_stats(const cgeom_t *g, int c, const double *D, const double *I,
                       const double *p, double *mI, double *mP, double *cov, double *var) {
  const long P = (long)g->h * g->w;
  for (int k = 0; k < c; ++k) {
    const double *Dk = D + 9 * k, *Ik = I + k * P, *pk = p + k * P;
    for (int i = 0; i < g->h; ++i)
      for (int j = 0; j < g->w; ++j) {
        const double N = tap_norm(g, Dk, i, j);
        double sI = 0.0, sP = 0.0;
        for (int t = 0; t < 9; ++t) {
          const long o = tap_at(g, i, j, t);
          if (o >= 0) {
            sI += Dk[t] * Ik[o];
            sP += Dk[t] * pk[o];
          }
        }
        const double mi = sI / N, mp = sP / N;
        double sv = 0.0, sc = 0.0;
        for (int t = 0; t < 9; ++t) {
          const long o = tap_at(g, i, j, t);
          if (o >= 0) {
            sv += Dk[t] * (Ik[o] - mi) * (Ik[o] - mi);
            sc += Dk[t] * (Ik[o] - mi) * (pk[o] - mp);
          }
        }
        const long m = (long)i * g->w + j;
        mI[k * P + m] = mi;
        mP[k * P + m] = mp;
        var[k * P + m] = sv / N;
        cov[k * P + m] = sc / N;
      }
  }
}

/* the pointwise block at one pixel: u[2c] -> y1, z1, y2, z2 [K], A[c] */
static void block_fwd(const gfo_conv_t *P, int c, const double *u, double *y1, double *z1,
                      double *y2, double *z2, double *A) {
  const int K = P->hidden;
  for (int a = 0; a < K; ++a) {
    double s = 0.0;
    for (int e = 0; e < 2 * c; ++e) s += P->W1[a * 2 * c + e] * u[e];
    y1[a] = s;
    z1[a] = lrelu(s, P->slope);
  }
  for (int a = 0; a < K; ++a) {
    double s = 0.0;
    for (int e = 0; e < K; ++e) s += P->W2[a * K + e] * z1[e];
    y2[a] = s;
    z2[a] = lrelu(s, P->slope);
  }
  for (int k = 0; k < c; ++k) {
    double s = 0.0;
    for (int e = 0; e < K; ++e) s += P->W3[k * K + e] * z2[e];
    A[k] = s;
  }
}

long gfo_conv_param_count(int c, int hidden) {
  return 9L * c + (long)hidden * 2 * c + (long)hidden * hidden + (long)c * hidden;
}

/* forward of one image: A, b [c][P] and Abar, bbar [c][P] */
static int conv_coeffs(const cgeom_t *g, int c, int mean_ab, const gfo_conv_t *P,
                       const double *I, const double *p, double *A, double *B, double *Ab,
                       double *Bb, double *mI, double *mP, double *cov, double *var) {
  const long Pl = (long)g->h * g->w;
  const int K = P->hidden;
  double *scr = (double *)malloc(sizeof(double) * (size_t)(2 * c + 4 * K + c));
  if (!scr) return -2;
  double *u = scr, *y1 = u + 2 * c, *z1 = y1 + K, *y2 = z1 + K, *z2 = y2 + K, *a = z2 + K;
  conv_stats(g, c, P->D, I, p, mI, mP, cov, var);
  for (long m = 0; m < Pl; ++m) {
    for (int k = 0; k < c; ++k) {
      u[k] = cov[k * Pl + m];
      u[c + k] = var[k * Pl + m];
    }
    block_fwd(P, c, u, y1, z1, y2, z2, a);
    for (int k = 0; k < c; ++k) {
      A[k * Pl + m] = a[k];
      B[k * Pl + m] = mP[k * Pl + m] - a[k] * mI[k * Pl + m];
    }
  }
  for (int k = 0; k < c; ++k) {
    if (mean_ab) {
      fd_plane(g, P->D + 9 * k, A + k * Pl, Ab + k * Pl);
      fd_plane(g, P->D + 9 * k, B + k * Pl, Bb + k * Pl);
    } else {
      memcpy(Ab + k * Pl, A + k * Pl, sizeof(double) * Pl);
      memcpy(Bb + k * Pl, B + k * Pl, sizeof(double) * Pl);
    }
  }
  free(scr);
  return 0;
}

static int conv_check(int n, int c, int h, int w, int H, int W, int r, const gfo_conv_t *P) {
  if (n <= 0 || c <= 0 || h <= 0 || w <= 0 || H < h || W < w || r < 1 || !P ||
      P->hidden <= 0 || !P->D || !P->W1 || !P->W2 || !P->W3)
    return -1;
  return 0;
}

int gfo_conv_forward(int n, int c, int h, int w, int H, int W, int r, int align_corners,
                     int mean_ab, const gfo_conv_t *P, const double *I_lo,
                     const double *p_lo, const double *I_hi, double *q) {
  if (conv_check(n, c, h, w, H, W, r, P)) return -1;
  const cgeom_t g = {h, w, r};
  const long Pl = (long)h * w, Ph = (long)H * W;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < n; ++b) {
    double *buf = (double *)malloc(sizeof(double) * (size_t)c * Pl * 8);
    if (!buf) {
      fail = 1;
      continue;
    }
    double *A = buf, *B = A + c * Pl, *Ab = B + c * Pl, *Bb = Ab + c * Pl;
    double *mI = Bb + c * Pl, *mP = mI + c * Pl, *cov = mP + c * Pl, *var = cov + c * Pl;
    if (conv_coeffs(&g, c, mean_ab, P, I_lo + (long)b * c * Pl, p_lo + (long)b * c * Pl, A, B,
                    Ab, Bb, mI, mP, cov, var)) {
      fail = 1;
      free(buf);
      continue;
    }
    for (int k = 0; k < c; ++k) {
      const double *gh = I_hi + ((long)b * c + k) * Ph;
      double *qq = q + ((long)b * c + k) * Ph;
      for (int y = 0; y < H; ++y) {
        int y0, y1;
        double wy;
        ctap(y, H, h, align_corners, &y0, &y1, &wy);
        for (int x = 0; x < W; ++x) {
          int x0, x1;
          double wx;
          ctap(x, W, w, align_corners, &x0, &x1, &wx);
          const double *La = Ab + k * Pl, *Lb = Bb + k * Pl;
          const double ah = (1 - wy) * ((1 - wx) * La[y0 * w + x0] + wx * La[y0 * w + x1]) +
                            wy * ((1 - wx) * La[y1 * w + x0] + wx * La[y1 * w + x1]);
          const double bh = (1 - wy) * ((1 - wx) * Lb[y0 * w + x0] + wx * Lb[y0 * w + x1]) +
                            wy * ((1 - wx) * Lb[y1 * w + x0] + wx * Lb[y1 * w + x1]);
          qq[(long)y * W + x] = ah * gh[(long)y * W + x] + bh;
        }
      }
    }
    free(buf);
  }
  return fail ? -2 : 0;
}

/* Transposed f_d of one plane: the gradient G of X's f_d output adds
 * D[t] / N(m) G(m) to X(m + r t); the weight gradient of this f_d use adds
 * G(m) (X(m + r t) - Y(m)) / N(m) to dD[t] (Y = f_d(X)). */
static void fd_plane_bwd(const cgeom_t *g, const double *Dk, const double *X, const double *Y,
                         const double *G, double *dX, double *dD, double *dD_abs) {
  for (int i = 0; i < g->h; ++i)
    for (int j = 0; j < g->w; ++j) {
      const long m = (long)i * g->w + j;
      const double N = tap_norm(g, Dk, i, j);
      for (int t = 0; t < 9; ++t) {
        const long o = tap_at(g, i, j, t);
        if (o < 0) continue;
        dX[o] += Dk[t] / N * G[m];
        const double term = G[m] * (X[o] - Y[m]) / N;
        dD[t] += term;
        dD_abs[t] += fabs(term);
      }
    }
}

int gfo_conv_backward(int n, int c, int h, int w, int H, int W, int r, int align_corners,
                      int mean_ab, const gfo_conv_t *P, const double *I_lo,
                      const double *p_lo, const double *I_hi, const double *dq,
                      double *dI_lo, double *dp_lo, double *dI_hi, double *dparams,
                      double *dparams_abs) {
  if (conv_check(n, c, h, w, H, W, r, P)) return -1;
  const cgeom_t g = {h, w, r};
  const long Pl = (long)h * w, Ph = (long)H * W;
  const int K = P->hidden;
  const long NP = gfo_conv_param_count(c, K);
  const long oW1 = 9L * c, oW2 = oW1 + (long)K * 2 * c, oW3 = oW2 + (long)K * K;
  /* per-image parameter gradients, summed over images in a fixed order */
  double *pg = (double *)calloc((size_t)n * NP * 2, sizeof(double));
  if (!pg) return -2;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < n; ++b) {
    double *dp = pg + (long)b * NP * 2, *dpa = dp + NP;
    double *buf = (double *)calloc((size_t)c * Pl * 16, sizeof(double));
    double *scr = (double *)malloc(sizeof(double) * (size_t)(6 * c + 8 * K));
    if (!buf || !scr) {
      fail = 1;
      free(buf);
      free(scr);
      continue;
    }
    double *A = buf, *B = A + c * Pl, *Ab = B + c * Pl, *Bb = Ab + c * Pl;
    double *mI = Bb + c * Pl, *mP = mI + c * Pl, *cov = mP + c * Pl, *var = cov + c * Pl;
    double *dAb = var + c * Pl, *dBb = dAb + c * Pl, *dA = dBb + c * Pl, *dB = dA + c * Pl;
    double *dmI = dB + c * Pl, *dmP = dmI + c * Pl, *dcov = dmP + c * Pl, *dvar = dcov + c * Pl;
    const double *I = I_lo + (long)b * c * Pl, *p = p_lo + (long)b * c * Pl;
    if (conv_coeffs(&g, c, mean_ab, P, I, p, A, B, Ab, Bb, mI, mP, cov, var)) {
      fail = 1;
      free(buf);
      free(scr);
      continue;
    }
    /* high resolution: q = Ah Gh + Bh -> dI_h, and the transposed bilinear */
    for (int k = 0; k < c; ++k) {
      const double *gh = I_hi + ((long)b * c + k) * Ph, *dqq = dq + ((long)b * c + k) * Ph;
      double *dih = dI_hi ? dI_hi + ((long)b * c + k) * Ph : NULL;
      const double *La = Ab + k * Pl;
      double *ga = dAb + k * Pl, *gb = dBb + k * Pl;
      for (int y = 0; y < H; ++y) {
        int y0, y1;
        double wy;
        ctap(y, H, h, align_corners, &y0, &y1, &wy);
        for (int x = 0; x < W; ++x) {
          int x0, x1;
          double wx;
          ctap(x, W, w, align_corners, &x0, &x1, &wx);
          const long o = (long)y * W + x;
          const double w00 = (1 - wy) * (1 - wx), w01 = (1 - wy) * wx, w10 = wy * (1 - wx),
                       w11 = wy * wx;
          if (dih) {
            const double ah = w00 * La[y0 * w + x0] + w01 * La[y0 * w + x1] +
                              w10 * La[y1 * w + x0] + w11 * La[y1 * w + x1];
            dih[o] = dqq[o] * ah;
          }
          const double va = dqq[o] * gh[o], vb = dqq[o];
          ga[y0 * w + x0] += w00 * va;
          ga[y0 * w + x1] += w01 * va;
          ga[y1 * w + x0] += w10 * va;
          ga[y1 * w + x1] += w11 * va;
          gb[y0 * w + x0] += w00 * vb;
          gb[y0 * w + x1] += w01 * vb;
          gb[y1 * w + x0] += w10 * vb;
          gb[y1 * w + x1] += w11 * vb;
        }
      }
      /* through the window mean of A and b */
      if (mean_ab) {
        fd_plane_bwd(&g, P->D + 9 * k, A + k * Pl, Ab + k * Pl, ga, dA + k * Pl, dp + 9 * k,
                     dpa + 9 * k);
        fd_plane_bwd(&g, P->D + 9 * k, B + k * Pl, Bb + k * Pl, gb, dB + k * Pl, dp + 9 * k,
                     dpa + 9 * k);
      } else {
        for (long m = 0; m < Pl; ++m) {
          dA[k * Pl + m] += ga[m];
          dB[k * Pl + m] += gb[m];
        }
      }
    }
    /* b = mean_p - A mean_I, then the pointwise block */
    double *u = scr, *y1 = u + 2 * c, *z1 = y1 + K, *y2 = z1 + K, *z2 = y2 + K, *a = z2 + K;
    double *dz2 = a + c, *dy2 = dz2 + K, *dz1 = dy2 + K, *dy1 = dz1 + K, *du = dy1 + K;
    double *dAt = du + 2 * c;
    for (long m = 0; m < Pl; ++m) {
      for (int k = 0; k < c; ++k) {
        dmP[k * Pl + m] += dB[k * Pl + m];
        dAt[k] = dA[k * Pl + m] - dB[k * Pl + m] * mI[k * Pl + m];
        dmI[k * Pl + m] += -dB[k * Pl + m] * A[k * Pl + m];
        u[k] = cov[k * Pl + m];
        u[c + k] = var[k * Pl + m];
      }
      block_fwd(P, c, u, y1, z1, y2, z2, a);
      for (int e = 0; e < K; ++e) {
        double s = 0.0;
        for (int k = 0; k < c; ++k) {
          s += P->W3[k * K + e] * dAt[k];
          dp[oW3 + k * K + e] += dAt[k] * z2[e];
          dpa[oW3 + k * K + e] += fabs(dAt[k] * z2[e]);
        }
        dz2[e] = s;
        dy2[e] = s * lrelu_d(y2[e], P->slope);
      }
      for (int e = 0; e < K; ++e) {
        double s = 0.0;
        for (int a2 = 0; a2 < K; ++a2) {
          s += P->W2[a2 * K + e] * dy2[a2];
          dp[oW2 + a2 * K + e] += dy2[a2] * z1[e];
          dpa[oW2 + a2 * K + e] += fabs(dy2[a2] * z1[e]);
        }
        dz1[e] = s;
        dy1[e] = s * lrelu_d(y1[e], P->slope);
      }
      for (int e = 0; e < 2 * c; ++e) {
        double s = 0.0;
        for (int a1 = 0; a1 < K; ++a1) {
          s += P->W1[a1 * 2 * c + e] * dy1[a1];
          dp[oW1 + a1 * 2 * c + e] += dy1[a1] * u[e];
          dpa[oW1 + a1 * 2 * c + e] += fabs(dy1[a1] * u[e]);
        }
        du[e] = s;
      }
      for (int k = 0; k < c; ++k) {
        dcov[k * Pl + m] = du[k];
        dvar[k * Pl + m] = du[c + k];
      }
    }
    /* the statistics: mean_I, mean_p, cov, var of every window */
    for (int k = 0; k < c; ++k) {
      const double *Dk = P->D + 9 * k, *Ik = I + k * Pl, *pk = p + k * Pl;
      double *gI = dI_lo ? dI_lo + ((long)b * c + k) * Pl : NULL;
      double *gP = dp_lo ? dp_lo + ((long)b * c + k) * Pl : NULL;
      if (gI) memset(gI, 0, sizeof(double) * Pl);
      if (gP) memset(gP, 0, sizeof(double) * Pl);
      for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
          const long m = (long)i * w + j, km = k * Pl + m;
          const double N = tap_norm(&g, Dk, i, j);
          const double mi = mI[km], mp = mP[km];
          for (int t = 0; t < 9; ++t) {
            const long o = tap_at(&g, i, j, t);
            if (o < 0) continue;
            const double at = Dk[t] / N, di = Ik[o] - mi, dpp = pk[o] - mp;
            if (gI) gI[o] += at * (dmI[km] + dcov[km] * dpp + 2.0 * dvar[km] * di);
            if (gP) gP[o] += at * (dmP[km] + dcov[km] * di);
            const double term = (dmI[km] * di + dmP[km] * dpp +
                                 dcov[km] * (di * dpp - cov[km]) +
                                 dvar[km] * (di * di - var[km])) / N;
            dp[9 * k + t] += term;
            dpa[9 * k + t] += fabs(term);
          }
        }
    }
    free(buf);
    free(scr);
  }
  if (!fail) {
    if (dparams) memset(dparams, 0, sizeof(double) * NP);
    if (dparams_abs) memset(dparams_abs, 0, sizeof(double) * NP);
    for (int b = 0; b < n; ++b)
      for (long e = 0; e < NP; ++e) {
        if (dparams) dparams[e] += pg[(long)b * NP * 2 + e];
        if (dparams_abs) dparams_abs[e] += pg[(long)b * NP * 2 + NP + e];
      }
  }
  free(pg);
  return fail ? -2 : 0;
}
