/*
 * gf.h — C ABI of the MI355X (gfx950) fast guided filtering layer.
 *
 * The operator is the guided filtering layer of Wu et al., "Fast End-to-End
 * Trainable Guided Filter" (arXiv 1803.05619), Sec. III: given a low-res
 * guide I_l, a low-res input p_l (the paper's O_l) and a high-res guide I_h,
 * it returns the high-res output q (the paper's O_h):
 *
 *   G = F(I)                     guidance map (Sec. III-D): the identity, the
 *                                channel mean (grey guide, Sec. IV-B), or the
 *                                trainable transform of gf_guide_t
 *   mean_I, mean_p, var, cov     (2r+1)^2 window means over G_l, p_l, the
 *                                window clipped to the image and normalised
 *                                by its in-image pixel count N (box filter
 *                                f_mu, Sec. III-C)
 *   A = cov / (var + eps)        local linear model, Eq. (1); A := 0 when
 *   b = mean_p - A mean_I        var + eps == 0
 *   Abar, bbar                   window means of A and b (mean_ab = 1, the
 *                                guided filter the layer reformulates) or
 *                                A, b themselves (mean_ab = 0, the form of
 *                                Algorithm 1)
 *   A_h, b_h                     bilinear upsampling f_up, half-pixel centres
 *                                (or corner-aligned, desc.align_corners)
 *   q = A_h * G_h + b_h          Eq. (2)
 *
 * gf_backward is the adjoint (Algorithm 1, extended by the window mean of
 * A and b when mean_ab = 1): gradients of <q, dq> with respect to I_l, p_l,
 * I_h and eps.
 *
 * Conventions shared by every entry point
 *  - Tensor pointers are DEVICE pointers (HIP global memory), NCHW
 *    contiguous, 16-byte aligned.  Shapes:
 *        I_lo, p_lo      [n, c, h_lo, w_lo]   io_dtype
 *        I_hi, q_hi      [n, c, h_hi, w_hi]   io_dtype
 *        dq_hi, dI_hi    [n, c, h_hi, w_hi]   io_dtype
 *        dI_lo, dp_lo    [n, c, h_lo, w_lo]   float32 (any io_dtype)
 *        eps, deps       [eps_count]          float32, eps_count = 1 or n
 *  - Any sizes h_lo <= h_hi, w_lo <= w_hi (the ratio may differ per axis
 *    and need not be an integer; Sec. III-A).  One integer factor
 *    s in {1, 2, 4, 8} on both axes takes kernels with compile-time tap
 *    weights; other ratios take general kernels with exact per-row and
 *    per-column taps (the batched plans take the integer factors only).
 *  - The caller owns all memory.  Scratch memory is passed in as `ws`
 *    (device pointer, ws_bytes long, at least gf_workspace_size(...)).
 *    The library allocates nothing.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and is asynchronous: a return of GF_OK means the arguments were valid
 *    and the kernels were launched.  Faults inside kernels surface at the
 *    next synchronisation, as with any HIP launch.
 *  - Argument checks run on the host before any HIP call; invalid input
 *    returns an error code, never aborts, and launches nothing.
 *  - Gradient outputs are overwritten, never accumulated.  deps with
 *    eps_count = 1 receives the sum over all images.
 *  - Not re-entrant on one workspace: concurrent calls need distinct ws.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { GF_F32 = 0, GF_F16 = 1, GF_BF16 = 2 } gf_dtype_t;

typedef enum {
  GF_OK = 0,
  GF_ERR_INVALID_ARG = 1, /* null pointer, bad size, negative radius/eps ... */
  GF_ERR_UNSUPPORTED = 2, /* valid for the method, not implemented here     */
  GF_ERR_WORKSPACE = 3,   /* ws too small (or NULL with nonzero need)       */
  GF_ERR_HIP = 4          /* a HIP runtime call failed                      */
} gf_status_t;

/* Problem description (host struct, read during the call only). */
typedef struct {
  int32_t n;        /* images                                             */
  int32_t c;        /* channels; guide channel k filters input channel k  */
  int32_t h_lo;     /* low-res height                                     */
  int32_t w_lo;     /* low-res width                                      */
  int32_t h_hi;     /* high-res height >= h_lo                            */
  int32_t w_hi;     /* high-res width  >= w_lo                            */
  int32_t r;        /* box radius, >= 0 (window side 2r + 1)              */
  int32_t mean_ab;  /* 1: window-mean A and b before upsampling; 0: not   */
  int32_t io_dtype; /* gf_dtype_t of I_lo, p_lo, I_hi, q_hi, dq_hi, dI_hi */
  int32_t align_corners; /* 0: half-pixel centres (default); 1: corner   */
                         /* alignment, source y (h_lo-1)/(h_hi-1)        */
  int32_t precise;  /* 0: window statistics of radii 0..4 in two levels in
                       FP32 (faster); 1: FP64 running window sums at every
                       radius, and for FP32 I/O the backward's adjoint
                       quantities in FP64 too: FP32-level accuracy also at
                       tiny eps on nearly flat guides (about 1.7x the time
                       of the low-res passes' share at radius 1).  Radii
                       >= 5 take the FP64 walkers either way.            */
} gf_desc_t;

/* Guidance map G = F(I) (Sec. III-D).  Pass NULL for the identity.
 *
 * GF_GUIDE_GREY: G_k = mean of the c_in input channels, for every output
 *   channel k (the grey guide used when input and output channel counts
 *   differ, Sec. IV-B); c_in in 1..4, c in 1..4.
 * GF_GUIDE_TRANSFORM: the trainable transform of Sec. III-D / Table I,
 *   per pixel x (c_in channels):
 *     h = W1 x                      1x1 convolution, hidden channels, no bias
 *     y = lam h + mu BN(h)          adaptive normalisation; BN with affine
 *                                   gamma, beta and the batch statistics of
 *                                   the call (all images and pixels of I_lo,
 *                                   respectively of I_hi; biased variance)
 *     z = leaky_relu(y, slope)      derivative `slope` for y <= 0
 *     G = W2 z + b2                 1x1 convolution with bias
 *   c_in == c == 3, hidden in 1..16.
 * With a guide, I_lo is [n, c_in, h_lo, w_lo], I_hi [n, c_in, h_hi, w_hi],
 * dI_lo [n, c_in, h_lo, w_lo] (float32) and dI_hi [n, c_in, h_hi, w_hi]. */
typedef enum {
  GF_GUIDE_IDENTITY = 0,
  GF_GUIDE_GREY = 1,
  GF_GUIDE_TRANSFORM = 2
} gf_guide_mode_t;

typedef struct {
  int32_t mode;          /* gf_guide_mode_t                                 */
  int32_t c_in;          /* channels of I_lo / I_hi                         */
  int32_t hidden;        /* transform: hidden channels                      */
  float bn_eps;          /* transform: batch-norm epsilon (e.g. 1e-5)       */
  float slope;           /* transform: leaky-ReLU negative slope (0.2)      */
  const float *params;   /* transform: DEVICE, gf_guide_param_count floats:
                            W1 [hidden][c_in] | W2 [c][hidden] | b2 [c] |
                            lam | mu | gamma [hidden] | beta [hidden]       */
  float *stats;          /* transform, optional DEVICE buffer of
                            gf_guide_stats_count floats: the batch mean and
                            covariance of the I_lo and the I_hi call.
                            gf_forward writes it (if not NULL);
                            gf_backward reads it when use_stats != 0,
                            otherwise recomputes the statistics            */
  int32_t use_stats;
} gf_guide_t;

size_t gf_guide_param_count(int32_t c_in, int32_t c, int32_t hidden);
size_t gf_guide_stats_count(int32_t c_in);

/* Bytes of scratch memory gf_forward (backward = 0), gf_backward
 * (backward = 1) or gf_forward_backward (backward = 2) needs for this
 * problem; 0 for an invalid description. */
size_t gf_workspace_size(const gf_desc_t *desc, const gf_guide_t *guide,
                         int32_t backward);

/* Forward pass (Sec. III-B/C, Eq. (1)-(2)): writes q_hi. */
int32_t gf_forward(const gf_desc_t *desc, const gf_guide_t *guide,
                   const void *I_lo, const void *p_lo, const void *I_hi,
                   const float *eps, int32_t eps_count, void *q_hi, void *ws,
                   size_t ws_bytes, void *stream);

/* Backward pass (Algorithm 1): gradients of sum(q * dq_hi).  Each output
 * pointer may be NULL (that gradient is not computed).  The low-res box
 * statistics and coefficients are recomputed from the inputs, not taken
 * from the forward pass.  dparams (transform guide only, DEVICE,
 * gf_guide_param_count floats, same layout as params) receives the
 * gradient of every transform parameter, summed over the I_lo and I_hi
 * calls of the shared transform. */
int32_t gf_backward(const gf_desc_t *desc, const gf_guide_t *guide,
                    const void *I_lo, const void *p_lo, const void *I_hi,
                    const float *eps, int32_t eps_count, const void *dq_hi,
                    float *dI_lo, float *dp_lo, void *dI_hi, float *deps,
                    float *dparams, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------- convolutional layer
 * The convolutional guided filtering layer (Sec. III-E, the layer of the
 * DGF_b^c variant): the mean filter becomes a learned 3x3 depthwise
 * convolution per channel with dilation desc->r (>= 1), normalised by the
 * same convolution of the all-ones image,
 *   f_d(X)(m) = sum_t D[t] X(m + r t) / sum_t D[t] [m + r t in the image],
 * and the local linear model a bias-free pointwise block on the per-pixel
 * (cov_0..cov_{c-1}, var_0..var_{c-1}) of all channels:
 *   A = W3 lrelu(W2 lrelu(W1 u))     (2c -> hidden -> hidden -> c)
 * with mean_I = f_d(I), mean_p = f_d(p), cov = f_d(I p) - mean_I mean_p,
 * var = f_d(I I) - mean_I^2; eps is dropped.  b = mean_p - A mean_I, the
 * window means Abar = f_d(A), bbar = f_d(b) (desc->mean_ab), bilinear
 * upsampling and q = A_h I_h + b_h as in gf_forward.  The paper fixes
 * neither the normalisation nor the block's depth and widths; this is the
 * library's reading (uniform D at r = 1 is the clipped box mean).
 * desc->c in 1..4 (guide channel k filters output channel k), hidden in
 * 1..16; the sum of each channel's in-image tap weights must be nonzero.
 * Shapes and dtypes as for gf_forward / gf_backward (identity guide, any
 * size ratio); params is a DEVICE float array of gf_conv_param_count
 * entries: D [c][9] (taps row-major over (dy, dx) in {-1, 0, 1}^2) |
 * W1 [hidden][2c] | W2 [hidden][hidden] | W3 [c][hidden]; dparams (nullable)
 * receives the gradient in the same layout. */
typedef struct {
  int32_t hidden;        /* width of the pointwise block's hidden layers   */
  float slope;           /* leaky-ReLU negative slope (derivative at 0)    */
  const float *params;   /* DEVICE, gf_conv_param_count(c, hidden) floats  */
} gf_conv_t;

size_t gf_conv_param_count(int32_t c, int32_t hidden);
size_t gf_conv_workspace_size(const gf_desc_t *desc, const gf_conv_t *conv,
                              int32_t backward);
int32_t gf_conv_forward(const gf_desc_t *desc, const gf_conv_t *conv,
                        const void *I_lo, const void *p_lo, const void *I_hi,
                        void *q_hi, void *ws, size_t ws_bytes, void *stream);
/* Gradients of sum(q * dq_hi); each output may be NULL.  Recomputes the
 * low-res statistics from the inputs. */
int32_t gf_conv_backward(const gf_desc_t *desc, const gf_conv_t *conv,
                         const void *I_lo, const void *p_lo, const void *I_hi,
                         const void *dq_hi, float *dI_lo, float *dp_lo,
                         void *dI_hi, float *dparams, void *ws, size_t ws_bytes,
                         void *stream);

/* Area downsampling, the first step of the deep guided filtering network
 * (Sec. IV, Fig. 3: I_h is downsampled to obtain I_l).  I_lo
 * [n, c, h_lo, w_lo] receives, per pixel (i, j), the mean of its covering
 * rectangle of I_hi [n, c, h_hi, w_hi]: rows floor(i h_hi / h_lo) ..
 * ceil((i + 1) h_hi / h_lo) - 1, columns likewise (the s x s block mean for
 * an integer factor s).  Both tensors have io_dtype; sums run in float32
 * and the result is rounded once.  Any h_lo <= h_hi, w_lo <= w_hi with
 * n * c and h_lo at most 65535 and at most 8191 high-res columns per
 * low-res pixel (GF_ERR_UNSUPPORTED otherwise).  No workspace. */
int32_t gf_downsample(int32_t n, int32_t c, int32_t h_hi, int32_t w_hi,
                      int32_t h_lo, int32_t w_lo, int32_t io_dtype,
                      const void *I_hi, void *I_lo, void *stream);

/* ------------------------------------------------------------- batched
 * Many independent problems of different sizes, factors, radii and eps
 * (identity guide, one io_dtype for all) run as one launch per phase and
 * launch class (the radius for the low-res phases, the factor for the
 * high-res ones) instead of one launch set per problem.  Each item follows
 * gf_forward / gf_backward exactly (same kernels, same results).
 *
 * gf_plan_create validates the items on the host, derives every launch
 * shape, and uploads the per-item launch tables to the current device (it
 * allocates: call it outside stream capture).  The item pointers are
 * stored in the plan: every gf_batched call reads and writes those
 * buffers.  gf_batched allocates nothing and does not synchronise. */
typedef struct {
  gf_desc_t d;          /* the item's problem (d.io_dtype equal for all items) */
  float eps;            /* its eps (>= 0), one for its d.n images              */
  const void *I_lo, *p_lo, *I_hi;   /* inputs, as for gf_forward               */
  void *q_hi;           /* forward output; NULL if the plan runs no forward    */
  const void *dq_hi;    /* backward input; NULL if the plan runs no backward   */
  float *dI_lo, *dp_lo; /* backward outputs, each may be NULL                  */
  void *dI_hi;
  float *deps;          /* one float: d<q, dq>/d eps summed over its images    */
} gf_item_t;

/* gf_batched modes: forward, backward, or both (the coefficients are then
 * computed once); GF_RUN_GRAPH additionally records the launches into a
 * HIP graph on the first call for a (mode, workspace) pair and replays it
 * afterwards (the first such call instantiates the graph on the host). */
enum { GF_RUN_FORWARD = 1, GF_RUN_BACKWARD = 2, GF_RUN_GRAPH = 4 };

typedef struct gf_plan gf_plan_t;

int32_t gf_plan_create(const gf_item_t *items, int32_t count, gf_plan_t **plan);
/* Workspace bytes gf_batched needs (every mode); 0 for NULL. */
size_t gf_plan_workspace_size(const gf_plan_t *plan);
int32_t gf_batched(gf_plan_t *plan, int32_t mode, void *ws, size_t ws_bytes,
                   void *stream);
/* Frees the plan's device tables and graphs (no call may be in flight). */
void gf_plan_destroy(gf_plan_t *plan);

/* ------------------------------------------------------------- autotuner
 * Times the candidate launch shapes of the four filter kernels (rows per
 * low-res walker wave, high-res rows per apply thread, low-res rows per
 * backward high-res wave) on the caller's buffers, `iters` launches each,
 * and keeps the fastest per kernel in a process-wide table keyed by
 * (io_dtype, factor, radius, guide mode, mean_ab).  Later plans for that
 * key (gf_forward, gf_backward, gf_plan_create) use the table.  Arguments
 * as for gf_forward plus gf_backward; every output is overwritten.  Shapes
 * whose workspace exceeds ws_bytes are skipped.  Synchronises the stream;
 * uses the kernel timing of gf_profile_enable (clears its records and
 * leaves it off). */
int32_t gf_autotune(const gf_desc_t *desc, const gf_guide_t *guide,
                    const void *I_lo, const void *p_lo, const void *I_hi,
                    const float *eps, int32_t eps_count, void *q_hi,
                    const void *dq_hi, float *dI_lo, float *dp_lo, void *dI_hi,
                    float *deps, float *dparams, void *ws, size_t ws_bytes,
                    int32_t iters, void *stream);
/* The table as text, one entry per line:
 *   dtype S r guide mean_ab : coef_rows lo_rows apply_rows bwd_rows
 * gf_tune_export writes up to cap bytes (NUL-terminated) and returns the
 * length of the full text; gf_tune_import adds the entries of such a text
 * (GF_ERR_INVALID_ARG on a malformed line, nothing imported then). */
size_t gf_tune_export(char *buf, size_t cap);
int32_t gf_tune_import(const char *text);

/* Forward and backward in one call: q_hi as gf_forward writes it and the
 * gradients as gf_backward writes them, with the guidance maps, the batch
 * statistics (saved to guide->stats if given) and the coefficients
 * computed once for both.  For callers that have dq_hi when they run the
 * forward (e.g. a fused training step or a benchmark of the whole layer).
 * Arguments as for gf_backward plus q_hi (required). */
int32_t gf_forward_backward(const gf_desc_t *desc, const gf_guide_t *guide,
                            const void *I_lo, const void *p_lo,
                            const void *I_hi, const float *eps,
                            int32_t eps_count, const void *dq_hi, void *q_hi,
                            float *dI_lo, float *dp_lo, void *dI_hi,
                            float *deps, float *dparams, void *ws,
                            size_t ws_bytes, void *stream);

/* gf_forward_backward without a caller workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs and errors as for
 * gf_forward_backward, minus ws / ws_bytes: the scratch memory is a static
 * device array of GF_STATIC_SCRATCH_BYTES inside the library (one per GPU,
 * held until the process ends).  A problem whose
 * gf_workspace_size(desc, guide, 2) exceeds it returns GF_ERR_WORKSPACE
 * before touching the device.  The call allocates nothing.  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other host threads) race: order them on one stream. */
#define GF_STATIC_SCRATCH_BYTES ((size_t)96 << 20)
int32_t gf_forward_backward_static(const gf_desc_t *desc,
                                   const gf_guide_t *guide, const void *I_lo,
                                   const void *p_lo, const void *I_hi,
                                   const float *eps, int32_t eps_count,
                                   const void *dq_hi, void *q_hi, float *dI_lo,
                                   float *dp_lo, void *dI_hi, float *deps,
                                   float *dparams, void *stream);

/* Human-readable name of a status code (static string). */
const char *gf_status_string(int32_t status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char *gf_last_error_detail(void);

/* Kernel timing on the launch stream (hipEvents recorded around every
 * kernel the library launches).  gf_profile_enable(1) starts recording
 * (and clears earlier records); gf_profile_read synchronises the events,
 * then fills up to `cap` entries with the kernel name and the summed
 * milliseconds and launch count of each kernel, and returns the number of
 * distinct kernels.  For measurement only: recording adds two event
 * records per launch. */
int32_t gf_profile_enable(int32_t on);
int32_t gf_profile_read(char (*names)[48], double *ms, int32_t *launches,
                        int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* GF_H */
