"""Error measures and bars shared by the GPU parity tests (HIP path vs the
FP64 oracle, element by element on the same seeded inputs).

Per-pixel outputs
  q                   max |gpu - ref|                               <= TOL[io]
  dI_lo, dp_lo, dI_hi max |gpu - ref| / max(1, max |ref|)           <= TOL[io]
Bars: 1e-4 for FP32 I/O, 2e-2 for BF16/FP16 I/O (q and dI_hi are rounded
once to the I/O type; the low-res gradients are FP32 outputs but inherit
the conditioning of eps = 1e-8 on half-quantised guides).

Sums over pixels (deps: one term d var per channel and low-res pixel;
each transform-parameter gradient: one term per pixel of both calls)
  *_sum   |gpu - ref| <= sum_bar(n) * sum |terms|  per entry, the terms'
          magnitude sum from the oracle (pinned against torch autograd):
          the first-order rounding bound of an FP32 sum whose terms pass
          through at most D sequential additions (the kernels' fixed
          reduction order: per-lane walks of at most 128 rows or pixels,
          shuffle and LDS trees, strided sums of at most ~100 partials per
          thread at these sizes; D <= 256 + log2 n) and are each formed with
          at most 16 roundings: (D + 16) u, u = 2^-24.
  *_rel   |gpu - ref| <= TOL_SUM * max |ref over the group|  (deps: |ref|
          per entry; transform parameters: per group W1, W2, lam, mu,
          gamma, beta).  The gradient of b2 is zero up to rounding (adding
          a constant to G at both resolutions leaves q unchanged), so it has
          only the *_sum check.  TOL_SUM is the FP32-output bar 1e-4: these
          are FP32 results for every I/O type.

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
TOL_SUM = 1e-4
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
        res["deps_sum"] = (float((d / np.maximum(ref["deps_abs"], 1e-300)).max()),
                           sum_bar(n_eps_terms))
        res["deps_rel"] = (float((d / np.maximum(np.abs(ref["deps"]), 1e-300)).max()), TOL_SUM)
    if "dparams" in got:
        d = np.abs(got["dparams"] - ref["dguide"])
        res["dparams_sum"] = (float((d / np.maximum(ref["dguide_abs"], 1e-300)).max()),
                              sum_bar(n_guide_terms))
        dg = oracle.guide_grad_split(d, 3, 3, hidden)
        rg = oracle.guide_grad_split(ref["dguide"], 3, 3, hidden)
        for g in GROUPS:
            scale = float(np.abs(rg[g]).max())
            res[f"d{g}_rel"] = (float(np.max(dg[g])) / max(scale, 1e-300), TOL_SUM)
    return res


def check(res, label=""):
    print(f"errors {label}:", {k: f"{e:.3e} (bar {b:.1e})" for k, (e, b) in res.items()},
          flush=True)
    bad = {k: v for k, v in res.items() if not v[0] <= v[1]}
    assert not bad, bad
    return res
