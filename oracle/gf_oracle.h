/*
 * FP64 CPU oracle of the fast guided filtering layer (arXiv 1803.05619,
 * Sec. III and Algorithm 1).  TEST INFRASTRUCTURE ONLY: used by the tests,
 * the smoke check and the CPU-baseline leg of the benchmark; never by the
 * product path.  Independent of the HIP library (no shared code/headers).
 *
 * Layouts: every array is NCHW contiguous, double precision, host memory.
 *   I_lo [n, cin, h, w]   p_lo [n, c, h, w]   I_hi [n, cin, H, W]
 *   q / dq / dI_hi at high resolution, dI_lo / dp_lo at low resolution.
 * eps has eps_count entries: 1 (shared) or n (one per image); deps likewise.
 * Any output pointer of the backward may be NULL (not computed).
 * deps_abs receives, per eps entry, the sum over pixels and channels of
 * |d var| (the magnitudes of the terms deps sums): the scale against which
 * the rounding error of a computed deps is judged.
 * Return 0 on success, -1 on invalid arguments, -2 on allocation failure.
 */
#ifndef GF_ORACLE_H
#define GF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { GFO_GUIDE_IDENTITY = 0, GFO_GUIDE_GREY = 1, GFO_GUIDE_TRANSFORM = 2 };

/* Parameters of the trainable guidance transform F (Sec. III-D, Table I):
 * 1x1 conv cin->hidden (no bias), adaptive norm lam*h + mu*BN(h) with BN
 * affine gamma/beta and batch statistics, leaky ReLU, 1x1 conv hidden->c
 * with bias. */
typedef struct {
  int hidden;
  const double *w1;    /* [hidden * cin]   row k = hidden channel      */
  const double *w2;    /* [c * hidden]                                 */
  const double *b2;    /* [c]                                          */
  double lam, mu;      /* adaptive-norm mix                            */
  const double *gamma; /* [hidden]                                     */
  const double *beta;  /* [hidden]                                     */
  double bn_eps;       /* batch-norm epsilon                           */
  double slope;        /* leaky ReLU negative slope                    */
  double flip_delta;   /* > 0: pre-activations with |y| < flip_delta   */
                       /* take the other leaky-ReLU branch (tests of   */
                       /* branch-ambiguous pixels); 0: off             */
} gfo_guide_t;

/* OpenMP threads of the following calls (n > 0). */
void gfo_set_threads(int n);

/* Length of the flattened guide gradient:
 * dw1 | dw2 | db2 | dlam | dmu | dgamma | dbeta. */
long gfo_guide_grad_size(int cin, int cout, int hidden);

/* G [n, cout, P] = F(X [n, cin, P]) for one call (batch statistics of X). */
int gfo_guide_apply(int mode, const gfo_guide_t *g, int n, int cin, int cout,
                    long P, const double *X, double *G);

int gfo_forward(int n, int c, int h, int w, int H, int W, int r,
                int align_corners, int mean_ab, int guide_mode, int cin,
                const gfo_guide_t *g, const double *I_lo, const double *p_lo,
                const double *I_hi, const double *eps, int eps_count,
                double *q);

int gfo_guide_preact(const gfo_guide_t *g, int n, int cin, long P, const double *X,
                     double *Y);
int gfo_backward(int n, int c, int h, int w, int H, int W, int r,
                 int align_corners, int mean_ab, int guide_mode, int cin,
                 const gfo_guide_t *g, const double *I_lo,
                 const double *p_lo, const double *I_hi, const double *eps,
                 int eps_count, const double *dq, double *dI_lo,
                 double *dp_lo, double *dI_hi, double *deps, double *deps_abs,
                 double *dguide, double *dguide_abs);

/* I_l [n, c, h, w] = area downsampling of I_h [n, c, H, W] (the first
 * step of the DGF framework, Sec. IV): each low-res pixel is the mean of
 * its covering high-res rectangle, rows floor(i H / h) .. ceil((i+1) H / h)
 * - 1, columns likewise; any h <= H, w <= W. */
int gfo_area_down(int n, int c, int H, int W, int h, int w, const double *X,
                  double *Y);

/* ---- convolutional guided filtering layer (Sec. III-E), gf_conv_oracle.c
 * Parameters: D [c][9] (3x3 depthwise taps per channel, row-major over
 * (dy, dx) in {-1, 0, 1}^2, dilation r), W1 [hidden][2c], W2 [hidden]
 * [hidden], W3 [c][hidden]; flat gradient layout D | W1 | W2 | W3. */
typedef struct {
  int hidden;
  const double *D, *W1, *W2, *W3;
  double slope;
} gfo_conv_t;

long gfo_conv_param_count(int c, int hidden);
int gfo_conv_forward(int n, int c, int h, int w, int H, int W, int r, int align_corners,
                     int mean_ab, const gfo_conv_t *P, const double *I_lo,
                     const double *p_lo, const double *I_hi, double *q);
/* dparams / dparams_abs: gfo_conv_param_count entries (may be NULL) */
int gfo_conv_backward(int n, int c, int h, int w, int H, int W, int r, int align_corners,
                      int mean_ab, const gfo_conv_t *P, const double *I_lo,
                      const double *p_lo, const double *I_hi, const double *dq,
                      double *dI_lo, double *dp_lo, double *dI_hi, double *dparams,
                      double *dparams_abs);

#ifdef __cplusplus
}
#endif
#endif
