/*
 * FP64 CPU oracle of the fast guided filtering layer (Wu et al., "Fast
 * End-to-End Trainable Guided Filter", arXiv 1803.05619).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP
 * library.
 *
 * What it computes, per image n and channel c (guide channel c filters
 * output channel c, Sec. III-D):
 *   G_l = F(I_l), G_h = F(I_h)                          (Sec. III-D, Fig. 2)
 *   per low-res pixel k, window w_k = (2r+1)^2 square clipped to the image,
 *   N_k = |w_k| (mean filter f_mu realised as a box filter, Sec. III-C):
 *     mean_I = sum G / N, mean_p = sum p / N
 *     var    = sum (G - mean_I)^2 / N          (two-pass form)
 *     cov    = sum (G - mean_I)(p - mean_p) / N
 *     A = cov / (var + eps), b = mean_p - A mean_I   (local linear model,
 *                                                     Eq. (1); the
 *                                                     closed form implied
 *                                                     by Algorithm 1)
 *   optional window mean of A and b (the guided filter of He et al. that
 *   the layer reformulates; Algorithm 1 omits it) -> Abar, bbar
 *   A_h, b_h = bilinear upsampling of Abar, bbar (f_up, Sec. III-C)
 *   q = A_h * G_h + b_h                                 (Eq. (2))
 *
 * Everything is written as plain loops over windows ("brute force"): no
 * integral images, no separable passes, no running sums.  The backward
 * pass differentiates exactly these loops; its gradients are written in
 * scatter form, each loop the transpose of a forward loop.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - window clipped at the border and normalised by its in-image count;
 *   - population variance (1/N);
 *   - A := 0 (with zero gradient) when var + eps == 0;
 *   - bilinear with half-pixel centres (align_corners = 0) or corner
 *     alignment (align_corners = 1), taps clamped to the image;
 *   - transform F: 1x1 conv (no bias) -> adaptive norm lam*h + mu*BN(h)
 *     with training-mode batch statistics of that call (biased variance)
 *     -> leaky ReLU (derivative `slope` for y <= 0) -> 1x1 conv + bias.
 *
 * Parallelised over planes with OpenMP; within a plane the loops run in
 * a fixed order, so results are deterministic for any thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "gf_oracle.h"

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

/* Bilinear source taps for destination index d of a length-D axis
 * sampled from a length-S axis. */
static void bilinear_tap(int d, int D, int S, int align_corners,
                         int *t0, int *t1, double *wt) {
  double src;
  if (align_corners) {
    src = (D > 1) ? (double)d * (double)(S - 1) / (double)(D - 1) : 0.0;
  } else {
    src = ((double)d + 0.5) * (double)S / (double)D - 0.5;
    if (src < 0.0) src = 0.0;
  }
  int i0 = (int)floor(src);
  if (i0 > S - 1) i0 = S - 1;
  int i1 = imin(i0 + 1, S - 1);
  *t0 = i0;
  *t1 = i1;
  *wt = src - (double)i0;
}

/* ------------------------------------------------------------------ */
/* guidance transform F                                                */
/* ------------------------------------------------------------------ */

/* Branch of the leaky ReLU taken at pre-activation y: the positive branch
 * for y > 0 (derivative 1), the negative one otherwise (derivative slope).
 * With flip_delta > 0 every y with |y| < flip_delta takes the other branch,
 * in the forward and the backward alike: there the branch is not fixed by
 * any finite-precision evaluation of y, and both choices give a valid
 * gradient (of the function that takes that branch), which tests use. */
static int lrelu_positive(const gfo_guide_t *g, double y) {
  int pos = y > 0.0;
  if (g->flip_delta > 0.0 && fabs(y) < g->flip_delta) pos = !pos;
  return pos;
}

/* Saved per-call state of the transform (needed by its backward). */
typedef struct {
  int hidden;
  double *hpre;  /* [n, hidden, P] 1x1 conv output                   */
  double *mean;  /* [hidden] batch mean                               */
  double *rstd;  /* [hidden] 1/sqrt(var + bn_eps)                     */
} guide_state_t;

static void guide_state_free(guide_state_t *s) {
  free(s->hpre);
  free(s->mean);
  free(s->rstd);
  memset(s, 0, sizeof(*s));
}

/* G[n, cout, P] = F(X[n, cin, P]).  mode 0: identity (cin == cout);
 * mode 1: channel mean broadcast to every output channel; mode 2: the
 * trainable transform with batch statistics over (n, P). */
static int guide_forward(int mode, const gfo_guide_t *g, int n, int cin,
                         int cout, long P, const double *X, double *G,
                         guide_state_t *st) {
  memset(st, 0, sizeof(*st));
  if (mode == GFO_GUIDE_IDENTITY) {
    if (cin != cout) return -1;
    memcpy(G, X, sizeof(double) * (size_t)n * cin * P);
    return 0;
  }
  if (mode == GFO_GUIDE_GREY) {
    for (int b = 0; b < n; ++b)
      for (long p = 0; p < P; ++p) {
        double s = 0.0;
        for (int ci = 0; ci < cin; ++ci) s += X[((long)b * cin + ci) * P + p];
        s /= (double)cin;
        for (int co = 0; co < cout; ++co) G[((long)b * cout + co) * P + p] = s;
      }
    return 0;
  }
  if (mode != GFO_GUIDE_TRANSFORM || g == NULL || g->hidden <= 0) return -1;
  const int K = g->hidden;
  st->hidden = K;
  st->hpre = (double *)malloc(sizeof(double) * (size_t)n * K * P);
  st->mean = (double *)calloc((size_t)K, sizeof(double));
  st->rstd = (double *)calloc((size_t)K, sizeof(double));
  if (!st->hpre || !st->mean || !st->rstd) return -2;
  /* first 1x1 convolution, no bias */
  for (int b = 0; b < n; ++b)
    for (int k = 0; k < K; ++k)
      for (long p = 0; p < P; ++p) {
        double s = 0.0;
        for (int ci = 0; ci < cin; ++ci)
          s += g->w1[k * cin + ci] * X[((long)b * cin + ci) * P + p];
        st->hpre[((long)b * K + k) * P + p] = s;
      }
  /* batch statistics, two-pass, biased variance */
  const double cnt = (double)n * (double)P;
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int b = 0; b < n; ++b)
      for (long p = 0; p < P; ++p) s += st->hpre[((long)b * K + k) * P + p];
    double m = s / cnt;
    double v = 0.0;
    for (int b = 0; b < n; ++b)
      for (long p = 0; p < P; ++p) {
        double d = st->hpre[((long)b * K + k) * P + p] - m;
        v += d * d;
      }
    v /= cnt;
    st->mean[k] = m;
    st->rstd[k] = 1.0 / sqrt(v + g->bn_eps);
  }
  /* adaptive norm, leaky ReLU, second 1x1 convolution with bias */
  double *z = (double *)malloc(sizeof(double) * (size_t)K);
  if (!z) return -2;
  for (int b = 0; b < n; ++b)
    for (long p = 0; p < P; ++p) {
      for (int k = 0; k < K; ++k) {
        double h = st->hpre[((long)b * K + k) * P + p];
        double hn = (h - st->mean[k]) * st->rstd[k];
        double y = g->lam * h + g->mu * (g->gamma[k] * hn + g->beta[k]);
        z[k] = lrelu_positive(g, y) ? y : g->slope * y;
      }
      for (int co = 0; co < cout; ++co) {
        double s = g->b2[co];
        for (int k = 0; k < K; ++k) s += g->w2[co * K + k] * z[k];
        G[((long)b * cout + co) * P + p] = s;
      }
    }
  free(z);
  return 0;
}

/* Adjoint of guide_forward.  dX[n, cin, P] is overwritten; parameter
 * gradients are ADDED into dparam (layout of gfo_guide_grad_size), and, when
 * dabs is not NULL, the magnitudes of the per-pixel terms each parameter
 * gradient sums are ADDED into dabs (same layout): the scale of the
 * rounding error any summation order of those terms can make. */
static int guide_backward(int mode, const gfo_guide_t *g, int n, int cin,
                          int cout, long P, const double *X,
                          const guide_state_t *st, const double *dG,
                          double *dX, double *dparam, double *dabs) {
  if (mode == GFO_GUIDE_IDENTITY) {
    memcpy(dX, dG, sizeof(double) * (size_t)n * cin * P);
    return 0;
  }
  if (mode == GFO_GUIDE_GREY) {
    for (int b = 0; b < n; ++b)
      for (long p = 0; p < P; ++p) {
        double s = 0.0;
        for (int co = 0; co < cout; ++co) s += dG[((long)b * cout + co) * P + p];
        for (int ci = 0; ci < cin; ++ci)
          dX[((long)b * cin + ci) * P + p] = s / (double)cin;
      }
    return 0;
  }
  const int K = g->hidden;
  double *scratch_param = NULL;
  if (dparam == NULL) {
    scratch_param = (double *)calloc((size_t)gfo_guide_grad_size(cin, cout, K), sizeof(double));
    if (!scratch_param) return -2;
    dparam = scratch_param;
  }
  double *dw1 = dparam;
  double *dw2 = dw1 + K * cin;
  double *db2 = dw2 + cout * K;
  double *dlam = db2 + cout;
  double *dmu = dlam + 1;
  double *dgam = dmu + 1;
  double *dbet = dgam + K;
  const double cnt = (double)n * (double)P;
  const long nparam = gfo_guide_grad_size(cin, cout, K);
  double *abs_scratch = NULL;
  if (dabs == NULL) {
    abs_scratch = (double *)calloc((size_t)nparam, sizeof(double));
    if (!abs_scratch) {
      free(scratch_param);
      return -2;
    }
    dabs = abs_scratch;
  }
  double *aw1 = dabs;
  double *aw2 = aw1 + K * cin;
  double *ab2 = aw2 + cout * K;
  double *alam = ab2 + cout;
  double *amu = alam + 1;
  double *agam = amu + 1;
  double *abet = agam + K;

  /* pass 1: everything up to d(hn); keep dy and dhn per pixel */
  double *dy = (double *)malloc(sizeof(double) * (size_t)n * K * P);
  double *dhn = (double *)malloc(sizeof(double) * (size_t)n * K * P);
  if (!dy || !dhn) {
    free(dy);
    free(dhn);
    free(scratch_param);
    free(abs_scratch);
    return -2;
  }
  for (int b = 0; b < n; ++b)
    for (long p = 0; p < P; ++p) {
      for (int co = 0; co < cout; ++co) {
        db2[co] += dG[((long)b * cout + co) * P + p];
        ab2[co] += fabs(dG[((long)b * cout + co) * P + p]);
      }
      for (int k = 0; k < K; ++k) {
        long idx = ((long)b * K + k) * P + p;
        double h = st->hpre[idx];
        double hn = (h - st->mean[k]) * st->rstd[k];
        double bn = g->gamma[k] * hn + g->beta[k];
        double y = g->lam * h + g->mu * bn;
        const int pos = lrelu_positive(g, y);
        double z = pos ? y : g->slope * y;
        double dz = 0.0;
        for (int co = 0; co < cout; ++co) {
          double dg = dG[((long)b * cout + co) * P + p];
          dw2[co * K + k] += dg * z;
          aw2[co * K + k] += fabs(dg * z);
          dz += g->w2[co * K + k] * dg;
        }
        double dyv = pos ? dz : g->slope * dz;
        *dlam += dyv * h;
        *dmu += dyv * bn;
        double dbn = g->mu * dyv;
        dgam[k] += dbn * hn;
        dbet[k] += dbn;
        *alam += fabs(dyv * h);
        *amu += fabs(dyv * bn);
        agam[k] += fabs(dbn * hn);
        abet[k] += fabs(dbn);
        dy[idx] = dyv;
        dhn[idx] = g->gamma[k] * dbn;
      }
    }
  /* batch-norm adjoint: needs the batch means of dhn and dhn*hn */
  for (int k = 0; k < K; ++k) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < n; ++b)
      for (long p = 0; p < P; ++p) {
        long idx = ((long)b * K + k) * P + p;
        double hn = (st->hpre[idx] - st->mean[k]) * st->rstd[k];
        s1 += dhn[idx];
        s2 += dhn[idx] * hn;
      }
    s1 /= cnt;
    s2 /= cnt;
    for (int b = 0; b < n; ++b)
      for (long p = 0; p < P; ++p) {
        long idx = ((long)b * K + k) * P + p;
        double hn = (st->hpre[idx] - st->mean[k]) * st->rstd[k];
        double dh = g->lam * dy[idx] + st->rstd[k] * (dhn[idx] - s1 - hn * s2);
        dy[idx] = dh; /* reuse storage: now holds d(hpre) */
      }
  }
  /* first convolution */
  for (int b = 0; b < n; ++b)
    for (int ci = 0; ci < cin; ++ci)
      for (long p = 0; p < P; ++p) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += g->w1[k * cin + ci] * dy[((long)b * K + k) * P + p];
        dX[((long)b * cin + ci) * P + p] = s;
      }
  for (int k = 0; k < K; ++k)
    for (int ci = 0; ci < cin; ++ci) {
      double s = 0.0, sa = 0.0;
      for (int b = 0; b < n; ++b)
        for (long p = 0; p < P; ++p) {
          double t = dy[((long)b * K + k) * P + p] * X[((long)b * cin + ci) * P + p];
          s += t;
          sa += fabs(t);
        }
      dw1[k * cin + ci] += s;
      aw1[k * cin + ci] += sa;
    }
  free(dy);
  free(dhn);
  free(scratch_param);
  free(abs_scratch);
  return 0;
}

/* ------------------------------------------------------------------ */
/* per-plane filter                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
  int h, w, H, W, r, align_corners, mean_ab;
} plane_geom_t;

/* window bounds of low-res pixel (i, j) */
static void window(const plane_geom_t *g, int i, int j, int *i0, int *i1,
                   int *j0, int *j1) {
  *i0 = imax(0, i - g->r);
  *i1 = imin(g->h - 1, i + g->r);
  *j0 = imax(0, j - g->r);
  *j1 = imin(g->w - 1, j + g->r);
}

/* Low-res statistics and coefficients of one plane (all arrays h*w). */
static void plane_coeffs(const plane_geom_t *g, const double *G,
                         const double *p, double eps, double *mI, double *mP,
                         double *var, double *cov, double *A, double *B) {
  const int h = g->h, w = g->w;
  for (int i = 0; i < h; ++i)
    for (int j = 0; j < w; ++j) {
      int a0, a1, c0, c1;
      window(g, i, j, &a0, &a1, &c0, &c1);
      double N = (double)((a1 - a0 + 1) * (c1 - c0 + 1));
      double sG = 0.0, sP = 0.0;
      for (int u = a0; u <= a1; ++u)
        for (int v = c0; v <= c1; ++v) {
          sG += G[u * w + v];
          sP += p[u * w + v];
        }
      double mg = sG / N, mp = sP / N;
      double sv = 0.0, sc = 0.0;
      for (int u = a0; u <= a1; ++u)
        for (int v = c0; v <= c1; ++v) {
          double dg = G[u * w + v] - mg;
          sv += dg * dg;
          sc += dg * (p[u * w + v] - mp);
        }
      double vr = sv / N, cv = sc / N;
      double den = vr + eps;
      double a = (den == 0.0) ? 0.0 : cv / den;
      int k = i * w + j;
      mI[k] = mg;
      mP[k] = mp;
      var[k] = vr;
      cov[k] = cv;
      A[k] = a;
      B[k] = mp - a * mg;
    }
}

/* Window mean of X (h*w) into Y. */
static void plane_box_mean(const plane_geom_t *g, const double *X, double *Y) {
  for (int i = 0; i < g->h; ++i)
    for (int j = 0; j < g->w; ++j) {
      int a0, a1, c0, c1;
      window(g, i, j, &a0, &a1, &c0, &c1);
      double N = (double)((a1 - a0 + 1) * (c1 - c0 + 1));
      double s = 0.0;
      for (int u = a0; u <= a1; ++u)
        for (int v = c0; v <= c1; ++v) s += X[u * g->w + v];
      Y[i * g->w + j] = s / N;
    }
}

/* Bilinear sample of low-res plane L at high-res (y, x). */
static double plane_upsample_at(const plane_geom_t *g, const double *L, int y,
                                int x) {
  int y0, y1, x0, x1;
  double wy, wx;
  bilinear_tap(y, g->H, g->h, g->align_corners, &y0, &y1, &wy);
  bilinear_tap(x, g->W, g->w, g->align_corners, &x0, &x1, &wx);
  double top = (1.0 - wx) * L[y0 * g->w + x0] + wx * L[y0 * g->w + x1];
  double bot = (1.0 - wx) * L[y1 * g->w + x0] + wx * L[y1 * g->w + x1];
  return (1.0 - wy) * top + wy * bot;
}

static int check_args(int n, int c, int h, int w, int H, int W, int r,
                      int eps_count) {
  if (n <= 0 || c <= 0 || h <= 0 || w <= 0 || H <= 0 || W <= 0 || r < 0) return -1;
  if (eps_count != 1 && eps_count != n) return -1;
  return 0;
}

static int guide_cout_ok(int mode, int cin, int c, const gfo_guide_t *gd) {
  if (mode == GFO_GUIDE_IDENTITY) return cin == c;
  if (mode == GFO_GUIDE_GREY) return cin >= 1;
  if (mode == GFO_GUIDE_TRANSFORM) return gd != NULL && gd->hidden > 0;
  return 0;
}

/* ------------------------------------------------------------------ */
/* public entry points                                                 */
/* ------------------------------------------------------------------ */

void gfo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

long gfo_guide_grad_size(int cin, int cout, int hidden) {
  return (long)hidden * cin + (long)cout * hidden + cout + 2 + 2L * hidden;
}

int gfo_guide_apply(int mode, const gfo_guide_t *g, int n, int cin, int cout,
                    long P, const double *X, double *G) {
  guide_state_t st;
  int rc = guide_forward(mode, g, n, cin, cout, P, X, G, &st);
  guide_state_free(&st);
  return rc;
}

/* Pre-activations y = lam h + mu BN(h) of the transform (hidden channels,
 * batch statistics of X), Y[n, hidden, P]: where some y is within rounding
 * of 0 the leaky ReLU's branch is not determined by any finite-precision
 * evaluation, which tests use to tell such pixels apart. */
int gfo_guide_preact(const gfo_guide_t *g, int n, int cin, long P, const double *X,
                     double *Y) {
  if (!g || g->hidden <= 0) return -1;
  const int K = g->hidden;
  double *G = (double *)malloc(sizeof(double) * (size_t)n * 3 * P);
  if (!G) return -2;
  guide_state_t st;
  memset(&st, 0, sizeof(st));
  int rc = guide_forward(GFO_GUIDE_TRANSFORM, g, n, cin, 3, P, X, G, &st);
  if (rc == 0) {
    for (int b = 0; b < n; ++b)
      for (int k = 0; k < K; ++k)
        for (long p = 0; p < P; ++p) {
          const long idx = ((long)b * K + k) * P + p;
          const double h = st.hpre[idx];
          const double hn = (h - st.mean[k]) * st.rstd[k];
          Y[idx] = g->lam * h + g->mu * (g->gamma[k] * hn + g->beta[k]);
        }
  }
  guide_state_free(&st);
  free(G);
  return rc;
}

int gfo_forward(int n, int c, int h, int w, int H, int W, int r,
                int align_corners, int mean_ab, int guide_mode, int cin,
                const gfo_guide_t *gd, const double *I_lo, const double *p_lo,
                const double *I_hi, const double *eps, int eps_count,
                double *q) {
  if (check_args(n, c, h, w, H, W, r, eps_count)) return -1;
  if (!guide_cout_ok(guide_mode, cin, c, gd)) return -1;
  const long Pl = (long)h * w, Ph = (long)H * W;
  double *Gl = (double *)malloc(sizeof(double) * (size_t)n * c * Pl);
  double *Gh = (double *)malloc(sizeof(double) * (size_t)n * c * Ph);
  if (!Gl || !Gh) {
    free(Gl);
    free(Gh);
    return -2;
  }
  guide_state_t sl, sh;
  memset(&sl, 0, sizeof(sl));
  memset(&sh, 0, sizeof(sh));
  int rc = guide_forward(guide_mode, gd, n, cin, c, Pl, I_lo, Gl, &sl);
  if (!rc) rc = guide_forward(guide_mode, gd, n, cin, c, Ph, I_hi, Gh, &sh);
  guide_state_free(&sl);
  guide_state_free(&sh);
  if (rc) {
    free(Gl);
    free(Gh);
    return rc;
  }
  plane_geom_t geo = {h, w, H, W, r, align_corners, mean_ab};
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int pl = 0; pl < n * c; ++pl) {
    const int b = pl / c;
    const double e = eps[eps_count == 1 ? 0 : b];
    double *buf = (double *)malloc(sizeof(double) * (size_t)Pl * 8);
    if (!buf) {
      fail = 1;
      continue;
    }
    double *mI = buf, *mP = buf + Pl, *vr = buf + 2 * Pl, *cv = buf + 3 * Pl;
    double *A = buf + 4 * Pl, *B = buf + 5 * Pl, *Ab = buf + 6 * Pl,
           *Bb = buf + 7 * Pl;
    plane_coeffs(&geo, Gl + pl * Pl, p_lo + pl * Pl, e, mI, mP, vr, cv, A, B);
    if (mean_ab) {
      plane_box_mean(&geo, A, Ab);
      plane_box_mean(&geo, B, Bb);
    } else {
      memcpy(Ab, A, sizeof(double) * Pl);
      memcpy(Bb, B, sizeof(double) * Pl);
    }
    const double *gh = Gh + pl * Ph;
    double *qq = q + pl * Ph;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double ah = plane_upsample_at(&geo, Ab, y, x);
        double bh = plane_upsample_at(&geo, Bb, y, x);
        qq[(long)y * W + x] = ah * gh[(long)y * W + x] + bh;
      }
    free(buf);
  }
  free(Gl);
  free(Gh);
  return fail ? -2 : 0;
}

int gfo_backward(int n, int c, int h, int w, int H, int W, int r,
                 int align_corners, int mean_ab, int guide_mode, int cin,
                 const gfo_guide_t *gd, const double *I_lo,
                 const double *p_lo, const double *I_hi, const double *eps,
                 int eps_count, const double *dq, double *dI_lo,
                 double *dp_lo, double *dI_hi, double *deps,
                 double *deps_abs, double *dguide, double *dguide_abs) {
  if (check_args(n, c, h, w, H, W, r, eps_count)) return -1;
  if (!guide_cout_ok(guide_mode, cin, c, gd)) return -1;
  const long Pl = (long)h * w, Ph = (long)H * W;
  double *Gl = (double *)malloc(sizeof(double) * (size_t)n * c * Pl);
  double *Gh = (double *)malloc(sizeof(double) * (size_t)n * c * Ph);
  double *dGl = (double *)calloc((size_t)n * c * Pl, sizeof(double));
  double *dGh = (double *)calloc((size_t)n * c * Ph, sizeof(double));
  double *dep = (double *)calloc((size_t)n * c * 2, sizeof(double));
  if (!Gl || !Gh || !dGl || !dGh || !dep) {
    free(Gl);
    free(Gh);
    free(dGl);
    free(dGh);
    free(dep);
    return -2;
  }
  guide_state_t sl, sh;
  memset(&sl, 0, sizeof(sl));
  memset(&sh, 0, sizeof(sh));
  int rc = guide_forward(guide_mode, gd, n, cin, c, Pl, I_lo, Gl, &sl);
  if (!rc) rc = guide_forward(guide_mode, gd, n, cin, c, Ph, I_hi, Gh, &sh);
  plane_geom_t geo = {h, w, H, W, r, align_corners, mean_ab};
  int fail = rc ? 1 : 0;
  if (!fail) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int pl = 0; pl < n * c; ++pl) {
      const int b = pl / c;
      const double e = eps[eps_count == 1 ? 0 : b];
      double *buf = (double *)malloc(sizeof(double) * (size_t)Pl * 12);
      if (!buf) {
        fail = 1;
        continue;
      }
      double *mI = buf, *mP = buf + Pl, *vr = buf + 2 * Pl, *cv = buf + 3 * Pl;
      double *A = buf + 4 * Pl, *B = buf + 5 * Pl, *Ab = buf + 6 * Pl,
             *Bb = buf + 7 * Pl;
      double *dAb = buf + 8 * Pl, *dBb = buf + 9 * Pl, *dA = buf + 10 * Pl,
             *dB = buf + 11 * Pl;
      const double *G = Gl + pl * Pl, *p = p_lo + pl * Pl;
      plane_coeffs(&geo, G, p, e, mI, mP, vr, cv, A, B);
      if (mean_ab) {
        plane_box_mean(&geo, A, Ab);
        plane_box_mean(&geo, B, Bb);
      } else {
        memcpy(Ab, A, sizeof(double) * Pl);
        memcpy(Bb, B, sizeof(double) * Pl);
      }
      memset(dAb, 0, sizeof(double) * Pl);
      memset(dBb, 0, sizeof(double) * Pl);
      /* q = A_h G_h + b_h, A_h/b_h bilinear: scatter into the taps */
      const double *gh = Gh + pl * Ph, *dqq = dq + pl * Ph;
      double *dgh = dGh + pl * Ph;
      for (int y = 0; y < H; ++y) {
        int y0, y1;
        double wy;
        bilinear_tap(y, H, h, align_corners, &y0, &y1, &wy);
        for (int x = 0; x < W; ++x) {
          int x0, x1;
          double wx;
          bilinear_tap(x, W, w, align_corners, &x0, &x1, &wx);
          long o = (long)y * W + x;
          double top = (1.0 - wx) * Ab[y0 * w + x0] + wx * Ab[y0 * w + x1];
          double bot = (1.0 - wx) * Ab[y1 * w + x0] + wx * Ab[y1 * w + x1];
          double ah = (1.0 - wy) * top + wy * bot;
          dgh[o] = dqq[o] * ah;
          double ga = dqq[o] * gh[o]; /* d A_h */
          double gb = dqq[o];         /* d b_h */
          double w00 = (1.0 - wy) * (1.0 - wx), w01 = (1.0 - wy) * wx;
          double w10 = wy * (1.0 - wx), w11 = wy * wx;
          dAb[y0 * w + x0] += w00 * ga;
          dAb[y0 * w + x1] += w01 * ga;
          dAb[y1 * w + x0] += w10 * ga;
          dAb[y1 * w + x1] += w11 * ga;
          dBb[y0 * w + x0] += w00 * gb;
          dBb[y0 * w + x1] += w01 * gb;
          dBb[y1 * w + x0] += w10 * gb;
          dBb[y1 * w + x1] += w11 * gb;
        }
      }
      /* window mean of A, b: scatter each window's gradient back */
      if (mean_ab) {
        memset(dA, 0, sizeof(double) * Pl);
        memset(dB, 0, sizeof(double) * Pl);
        for (int i = 0; i < h; ++i)
          for (int j = 0; j < w; ++j) {
            int a0, a1, c0, c1;
            window(&geo, i, j, &a0, &a1, &c0, &c1);
            double N = (double)((a1 - a0 + 1) * (c1 - c0 + 1));
            double ga = dAb[i * w + j] / N, gb = dBb[i * w + j] / N;
            for (int u = a0; u <= a1; ++u)
              for (int v = c0; v <= c1; ++v) {
                dA[u * w + v] += ga;
                dB[u * w + v] += gb;
              }
          }
      } else {
        memcpy(dA, dAb, sizeof(double) * Pl);
        memcpy(dB, dBb, sizeof(double) * Pl);
      }
      /* coefficients -> window statistics -> pixels */
      double *dg = dGl + pl * Pl;
      double *dp = dp_lo ? dp_lo + pl * Pl : NULL;
      if (dp) memset(dp, 0, sizeof(double) * Pl);
      double de = 0.0, dabs = 0.0;
      for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) {
          int k = i * w + j;
          /* b = mean_p - A mean_I */
          double dmP = dB[k];
          double dmI = -dB[k] * A[k];
          double dAk = dA[k] - dB[k] * mI[k];
          /* A = cov / (var + eps) */
          double den = vr[k] + e;
          double dcv = 0.0, dvr = 0.0;
          if (den != 0.0) {
            dcv = dAk / den;
            dvr = -dAk * cv[k] / (den * den);
          }
          de += dvr;
          dabs += fabs(dvr);
          int a0, a1, c0, c1;
          window(&geo, i, j, &a0, &a1, &c0, &c1);
          double N = (double)((a1 - a0 + 1) * (c1 - c0 + 1));
          /* mean_I, mean_p, two-pass var and cov over the window */
          for (int u = a0; u <= a1; ++u)
            for (int v = c0; v <= c1; ++v) {
              int t = u * w + v;
              double cg = G[t] - mI[k], cp = p[t] - mP[k];
              dg[t] += (dmI + 2.0 * dvr * cg + dcv * cp) / N;
              if (dp) dp[t] += (dmP + dcv * cg) / N;
            }
        }
      dep[pl] = de;
      dep[n * c + pl] = dabs;
      free(buf);
    }
  }
  /* per eps entry: the gradient, and the sum of the magnitudes of its
   * terms (a scale for judging the rounding error of the sum) */
  for (int which = 0; which < 2 && !fail; ++which) {
    double *out = which == 0 ? deps : deps_abs;
    const double *src = dep + (size_t)which * n * c;
    if (!out) continue;
    if (eps_count == 1) {
      double s = 0.0;
      for (int pl = 0; pl < n * c; ++pl) s += src[pl];
      out[0] = s;
    } else {
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int ch = 0; ch < c; ++ch) s += src[b * c + ch];
        out[b] = s;
      }
    }
  }
  /* through the guidance transform (shared by both resolutions) */
  if (!fail && dguide && guide_mode == GFO_GUIDE_TRANSFORM)
    memset(dguide, 0, sizeof(double) * (size_t)gfo_guide_grad_size(cin, c, gd->hidden));
  if (!fail && dguide_abs && guide_mode == GFO_GUIDE_TRANSFORM)
    memset(dguide_abs, 0, sizeof(double) * (size_t)gfo_guide_grad_size(cin, c, gd->hidden));
  if (!fail) {
    double *tmp = dI_lo;
    double *own = NULL;
    if (!tmp) tmp = own = (double *)malloc(sizeof(double) * (size_t)n * cin * Pl);
    if (!tmp) fail = 1;
    else if (guide_backward(guide_mode, gd, n, cin, c, Pl, I_lo, &sl, dGl, tmp, dguide,
                            dguide_abs))
      fail = 1;
    free(own);
  }
  if (!fail) {
    double *tmp = dI_hi;
    double *own = NULL;
    if (!tmp) tmp = own = (double *)malloc(sizeof(double) * (size_t)n * cin * Ph);
    if (!tmp) fail = 1;
    else if (guide_backward(guide_mode, gd, n, cin, c, Ph, I_hi, &sh, dGh, tmp, dguide,
                            dguide_abs))
      fail = 1;
    free(own);
  }
  guide_state_free(&sl);
  guide_state_free(&sh);
  free(Gl);
  free(Gh);
  free(dGl);
  free(dGh);
  free(dep);
  return fail ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* downsampling of the DGF framework (Sec. IV, Fig. 3)                 */
/* ------------------------------------------------------------------ */

/* I_l = area downsampling of I_h to (h, w): the paper only says that I_h is
 * downsampled to obtain I_l (Sec. IV).  Reading: each low-res pixel (i, j)
 * is the plain mean of the high-res pixels of its covering rectangle, rows
 * floor(i H / h) .. ceil((i + 1) H / h) - 1 and columns likewise (for an
 * integer factor s = H / h the s x s block mean).  Written as the literal
 * double loop over that rectangle. */
int gfo_area_down(int n, int c, int H, int W, int h, int w, const double *X,
                  double *Y) {
  if (n < 1 || c < 1 || h < 1 || w < 1 || h > H || w > W || !X || !Y) return -1;
  const long planes = (long)n * c;
#pragma omp parallel for schedule(static)
  for (long pl = 0; pl < planes; ++pl) {
    const double *x = X + pl * (long)H * W;
    double *y = Y + pl * (long)h * w;
    for (int i = 0; i < h; ++i) {
      const long r0 = (long)i * H / h, r1 = ((long)(i + 1) * H + h - 1) / h;
      for (int j = 0; j < w; ++j) {
        const long c0 = (long)j * W / w, c1 = ((long)(j + 1) * W + w - 1) / w;
        double s = 0.0;
        for (long yy = r0; yy < r1; ++yy)
          for (long xx = c0; xx < c1; ++xx) s += x[yy * W + xx];
        y[(long)i * w + j] = s / (double)((r1 - r0) * (c1 - c0));
      }
    }
  }
  return 0;
}
