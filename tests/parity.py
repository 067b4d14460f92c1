"""Error measures and bars shared by the GPU parity tests (HIP path vs the
FP64 oracle, element by element on the same seeded inputs).

Per-pixel outputs
  q                   max |gpu - ref|                               <= TOL[io]
  dI_lo, dp_lo, dI_hi max |gpu - ref| / max(1, max |ref|)           <= TOL[io]
Bars: 1e-4 for FP32 I/O, 2e-2 for BF16/FP16 I/O (q and dI_hi are rounded
once to the I/O type; the low-res gradients are FP32 outputs but inherit
the conditioning of eps = 1e-8 on half-quantised guides).

Sums over pixels (deps: one term d var per channel and low-res pixel;
each transform-parameter gradient: one term per pixel of both calls) pass
when either bound holds, per entry:
  rel     |gpu - ref| <= TOL[io] * scale, scale = |ref| (deps) or the
          largest |ref| of the entry's group (transform parameters: W1, W2,
          lam, mu, gamma, beta): the stated target of the whole fused
          forward + backward for the problem's I/O type;
  sum     |gpu - ref| <= sum_bar(n) * sum |terms|, the terms' magnitude sum
          from the oracle (pinned against torch autograd): the first-order
          rounding bound of an FP32 sum whose terms pass through at most D
          sequential additions (the kernels' fixed reduction order: per-lane
          walks of at most 128 rows or pixels, shuffle and LDS trees,
          strided sums of at most ~100 partials per thread at these sizes;
          D <= 256 + log2 n) and are each formed with at most 16 roundings:
          (D + 16) u, u = 2^-24.
The first is the target; the second is what an FP32 evaluation can deliver
when the sum cancels heavily (sum |terms| / |sum| reaches 5e3 and more for
the transform's parameters and for deps at eps = 1e-8, where 1e-4 relative
to |ref| would ask for more than FP32 resolves).  A wrong term, sign or
factor misses both unless the sum is cancellation noise below FP32
resolution.  The gradient of b2 is zero up to rounding (adding a constant to
G at both resolutions leaves q unchanged), so it has only the sum bound.
Reported per quantity: max over entries of min(err_rel / bar_rel,
err_sum / bar_sum), which must be <= 1, beside both raw errors.

Branch-ambiguous pixels of the transform guide (some hidden pre-activation
|y| < BRANCH_DELTA, from the oracle's own pre-activations): the leaky ReLU's
branch there is not fixed by a finite-precision evaluation of y, and the
input gradient of either branch is valid.  The GPU value must equal the
oracle's normal gradient or the oracle's gradient with those pixels'
branches flipped (oracle option flip_delta), within the same bar.
"""
import math

import numpy as np

import oracle

U32 = 2.0 ** -24
TOL = {"f32": 1e-4, "bf16": 2e-2, "f16": 2e-2}
BRANCH_DELTA = 2e-6
GROUPS = ("w1", "w2", "lam", "mu", "gamma", "beta")


def sum_bar(n_terms: int) -> float:
    depth = 256 + math.ceil(math.log2(max(2, int(n_terms))))
    return (depth + 16) * U32


def branch_ambiguous(X, guide):
    """[n, 1, H, W] mask of pixels with some |y| < BRANCH_DELTA (oracle)."""
    Y = oracle.guide_preact(X, guide)
    return (np.abs(Y) < BRANCH_DELTA).any(axis=1, keepdims=True)


def flipped_reference(args, r, eps, dq, guide, **kw):
    """The oracle's gradients with every branch-ambiguous branch flipped."""
    return oracle.backward(*args, r, eps, dq, guide=dict(guide, flip_delta=BRANCH_DELTA), **kw)


def measure(got, ref, io, *, n_eps_terms=None, n_guide_terms=None, hidden=None, amb=None,
            ref_flip=None):
    """Errors of every output present in `got` (numpy float64 arrays) and the
    bar each must meet: {name: (error, bar)}."""
    tol = TOL[io]
    res = {}
    if "q" in got:
        res["q"] = (float(np.abs(got["q"] - ref["q"]).max()), tol)
    for k in ("dI_lo", "dp_lo", "dI_hi"):
        if k not in got:
            continue
        diff = np.abs(got[k] - ref[k])
        if amb is not None and k in amb and amb[k].any():
            alt = np.abs(got[k] - ref_flip[k])
            diff = np.where(amb[k], np.minimum(diff, alt), diff)
        res[k] = (float(diff.max() / max(1.0, np.abs(ref[k]).max())), tol)
    if "deps" in got:
        d = np.abs(got["deps"] - ref["deps"])
        e_sum = d / np.maximum(ref["deps_abs"], 1e-300)
        e_rel = d / np.maximum(np.abs(ref["deps"]), 1e-300)
        bar_sum = sum_bar(n_eps_terms)
        res["deps"] = (float(np.minimum(e_rel / tol, e_sum / bar_sum).max()), 1.0)
        res["deps_sum(info)"] = (float(e_sum.max()), math.inf)
        res["deps_rel(info)"] = (float(e_rel.max()), math.inf)
    if "dparams" in got:
        d = np.abs(got["dparams"] - ref["dguide"])
        e_sum = d / np.maximum(ref["dguide_abs"], 1e-300)
        bar_sum = sum_bar(n_guide_terms)
        res["dparams_sum(info)"] = (float(e_sum.max()), math.inf)
        dg = oracle.guide_grad_split(d, 3, 3, hidden)
        sg = oracle.guide_grad_split(e_sum, 3, 3, hidden)
        rg = oracle.guide_grad_split(ref["dguide"], 3, 3, hidden)
        for g in GROUPS + ("b2",):
            es = np.asarray(sg[g], dtype=np.float64) / bar_sum
            if g == "b2":
                res["db2"] = (float(es.max()), 1.0)
                continue
            er = np.asarray(dg[g], dtype=np.float64) / max(float(np.abs(rg[g]).max()), 1e-300)
            res[f"d{g}"] = (float(np.minimum(er / tol, es).max()), 1.0)
            res[f"d{g}_rel(info)"] = (float(er.max()), math.inf)
    return res


def check(res, label=""):
    print(f"errors {label}:", {k: f"{e:.3e} (bar {b:.1e})" for k, (e, b) in res.items()},
          flush=True)
    bad = {k: v for k, v in res.items() if not v[0] <= v[1]}
    assert not bad, bad
    return res


# ---------------------------------------------------------------- convolutional layer

CONV_TILE, CONV_BLOCKS, CONV_AB_GRID = 256, 1024, 512


def conv_sum_bar(n_pix: int, h: int, w: int, planes: int) -> float:
    """Rounding bound of the convolutional layer's parameter-gradient sums
    (an upper bound of the kernels' sequential depth: a tile's pixels, a
    workgroup's tiles, the workgroups, and for D the window-mean adjoint's
    per-plane partials), each term formed with at most 32 roundings."""
    tiles = -(-n_pix // CONV_TILE)
    grid = min(tiles, CONV_BLOCKS)
    ab = min(-(-(h * w) // 256), CONV_AB_GRID)
    depth = CONV_TILE + -(-tiles // grid) + grid + planes * ab + 256
    return (depth + 32) * U32


def measure_conv(got, ref, io, n, c, h, w, hidden):
    """Errors and bars of the convolutional layer's outputs: per-pixel ones as
    in measure(); each parameter group (D, W1, W2, W3) entry by entry passes
    when within TOL[io] of the group's largest |ref| or within the rounding
    bound of its sum (reported as the smaller ratio to its bar)."""
    tol = TOL[io]
    res = measure({k: v for k, v in got.items() if k != "dparams"}, ref, io)
    if "dparams" in got:
        d = np.abs(got["dparams"] - ref["dparams"])
        bar = conv_sum_bar(n * h * w, h, w, n * c)
        e_sum = d / np.maximum(ref["dparams_abs"], 1e-300) / bar
        dg = oracle.conv_split(d, c, hidden)
        sg = oracle.conv_split(e_sum, c, hidden)
        rg = oracle.conv_split(ref["dparams"], c, hidden)
        for g in oracle.CONV_GROUPS:
            er = np.asarray(dg[g]) / max(float(np.abs(rg[g]).max()), 1e-300)
            res[f"d{g}"] = (float(np.minimum(er / tol, np.asarray(sg[g])).max()), 1.0)
            res[f"d{g}_rel(info)"] = (float(er.max()), math.inf)
    return res
