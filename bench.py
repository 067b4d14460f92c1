"""Benchmark of the fused guided filtering layer on one MI355X.

A step is one forward + one backward of the layer over one batch, with the
inputs already resident in HBM: one gf_forward_backward call (the batched
plan for workload 3), which computes the coefficients and guide maps once
for both directions; `separate_calls` times the same step as gf_forward then
gf_backward.  Workloads (--workload):

  1 (default)  FP32, 4 x 3 x 2048 x 3072 high-res (512 x 768 low-res, s = 4),
               r = 1, eps = 1e-4, dq ~ N(0, 1); gradients to p_l, I_l, I_h, eps
  2            trainable guide (3 -> 15 -> 3, adaptive BN, leaky ReLU 0.2),
               BF16 I/O, 8 x 3 x 1536 x 2048 (s = 4), r = 1, eps = 1e-8;
               gradients to p_l, eps and every guide parameter
  3            64 uneven images (H, W in [512, 3072], s in {2, 4, 8},
               r in {1, 2, 4}, eps in [1e-8, 1e-2]), FP32, one batched plan
               replayed as a HIP graph, launch shapes autotuned first
  4            FP16 I/O precision stress: 2 x 3 x 2160 x 3840 (s = 4) with
               near-constant regions, r = 8 (--radius 1 for the r = 1 run),
               eps = 1e-8

  0            the plain forward only, FP32, 1 x 3 x 256 x 256 from 64 x 64
               (s = 4), r = 1, eps = 1e-2 (latency-bound: reported per call)
  5            the convolutional guided filtering layer (Sec. III-E), FP32,
               the images of workload 1, dilation 1: gf_conv_forward then
               gf_conv_backward, gradients to every input and parameter

Prints ONE JSON line:
  value        high-res Mpixel/s of fwd+bwd (a 3-channel pixel counts once)
  roofline     the dominant kernel: its algorithmic bytes per step / its time
               per step (HIP events around every launch, on the launch
               stream, over a second timed pass of the same steps: events
               add time, so `value` comes from the first, event-free pass),
               against the 8 TB/s HBM peak; `traffic` is the HBM
               bytes per launch measured with rocprofv3 counters (workload 1,
               from the committed summary; null when the kernel changed since)
  timing_ms    per-step median/p10/p90 from HIP events around each step,
               warm (back to back) and cold (a 512 MB buffer written before
               every step, outside its events, to flush L2 and the MALL)
  peak_mem_bytes  torch's peak device allocation over the timed steps
               (inputs, outputs and workspace)
  separate_calls  the step as gf_forward then gf_backward
  autograd_step   the step through the torch.autograd.Function (what a
               training loop calls: gf_forward, then gf_backward)
  plain        the unfused PyTorch composition (autograd) on the same GPU
  cpu_baseline the FP64 CPU oracle on the host cores (bounded sample), the
               host CPU model, and a 1-thread rate on one image
  error_vs_fp64_oracle  errors of this run's outputs on that sample

  --dgf        instead: the deep guided filtering network's inference chain
               (downsampling, C_l, the layer) over 512^2..3072^2 and Table IV's
               I_l sizes: median ms per image, each step's share, peak memory

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload N]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak (256 CUs x 4 SIMDs x 16 lanes x 2 (packed) x 2 (FMA)
# x 2.4 GHz); the library is built without packed FP32, so 78.6 is its cap
FP32_VEC_PEAK_TFLOPS = 157.3
# the sources that define, configure and launch the identity-guide kernels
# whose HBM traffic is profiled (the FP32 instantiation): a traffic figure
# measured on other versions of them is stale
KERNEL_SRCS = tuple(os.path.join(ROOT, p) for p in (
    "include/gf.h", "paper_1803_05619_amd/csrc/gf_internal.h",
    "paper_1803_05619_amd/csrc/gf_kernels.h", "paper_1803_05619_amd/csrc/gf_api.cpp",
    "paper_1803_05619_amd/csrc/gf_f32.hip"))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_fp32_4x3x2048x3072.txt")
METRIC = "high-res Mpixel/s fwd+bwd, fused vs plain at stated max-abs error; % HBM peak"
DATA = "synthetic (seeded photo-like images: smooth field + step edges + noise)"
BYTES = {"f32": 4, "bf16": 2, "f16": 2}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    """sha256[:16] over KERNEL_SRCS, in that order."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        h.update(os.path.basename(path).encode())
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def identity_bytes(n, c, H, W, h, w, b, with_dI=True):
    """Compulsory bytes of each identity-guide kernel per launch (every input
    read once, every output written once; low-res gradients are float32)."""
    hi, lo = n * c * H * W, n * c * h * w
    return {
        "apply": 2 * b * hi,                                  # I_h in, q out
        "bwd_hi": (3 if with_dI else 2) * b * hi,             # dq, I_h in, dI_h out
        "coef": 2 * b * lo,                                   # I_l, p_l in
        "bwd_lo": 2 * b * lo + (8 if with_dI else 4) * lo,    # I_l, p_l in; dI_l, dp_l out
    }


def oracle_errors(got, ref, hidden=None):
    """Errors as in the parity tests: q absolute; per-pixel gradients scaled
    by max(1, max |ref|); deps relative to |ref| and to the sum of the
    magnitudes of its terms; the guide parameters' gradients relative to the
    largest gradient of their group (W1, W2, lam, mu, gamma, beta) and to
    the magnitude sums of their terms."""
    import numpy as np
    err = {}
    if "q" in got:
        err["q_max_abs"] = float(np.abs(got["q"] - ref["q"]).max())
    for k in ("dI_lo", "dp_lo", "dI_hi"):
        if k in got and k in ref:
            err[k + "_scaled"] = float(np.abs(got[k] - ref[k]).max() /
                                       max(1.0, np.abs(ref[k]).max()))
    if "deps" in got:
        d = np.abs(got["deps"] - ref["deps"])
        err["deps_rel"] = float((d / np.maximum(np.abs(ref["deps"]), 1e-300)).max())
        err["deps_sum_scaled"] = float((d / np.maximum(ref["deps_abs"], 1e-300)).max())
    if "dguide" in got:
        import oracle
        d = np.abs(got["dguide"] - ref["dguide"])
        err["dguide_sum_scaled"] = float((d / np.maximum(ref["dguide_abs"], 1e-300)).max())
        dg = oracle.guide_grad_split(d, 3, 3, hidden)
        rg = oracle.guide_grad_split(ref["dguide"], 3, 3, hidden)
        err["dguide_group_rel"] = max(float(np.max(dg[g])) / max(float(np.abs(rg[g]).max()), 1e-300)
                                      for g in ("w1", "w2", "lam", "mu", "gamma", "beta"))
    return err


def merge_max(acc, err):
    for k, v in err.items():
        acc[k] = max(acc.get(k, 0.0), v)
    return acc


# ------------------------------------------------------------------ workloads

def workload_1(args, dev):
    import torch

    from paper_1803_05619_amd import datagen, gf, plain
    log("generating workload 1 (FP32 4x3x2048x3072)")
    prob = datagen.make_config(1)
    return identity_workload(args, dev, prob, "f32",
                             "guided filtering layer fwd+bwd, FP32, 4x3x2048x3072 high-res "
                             "<- 512x768 low-res (s=4), r=1, eps=1e-4, window-mean of A,b, "
                             "grads to p_l, I_l, I_h, eps")


def workload_4(args, dev):
    from paper_1803_05619_amd import datagen
    r = args.radius if args.radius is not None else 8
    log(f"generating workload 4 (FP16 2x3x2160x3840, near-constant regions, r={r})")
    prob = datagen.make_config(4, r=r)
    return identity_workload(args, dev, prob, "f16",
                             f"precision stress fwd+bwd, FP16 I/O + FP32 accumulate, "
                             f"2x3x2160x3840 <- 540x960 (s=4), r={r}, eps=1e-8, near-constant "
                             f"regions 0.5+N(0,1e-4), grads to p_l, I_l, I_h, eps")


def identity_workload(args, dev, prob, dt, name):
    import torch

    from paper_1803_05619_amd import gf, plain
    n, c, H, W, h, w, r = (prob[k] for k in ("n", "c", "H", "W", "h", "w", "r"))
    pr = bool(args.precise)  # FP64 wide walkers at every radius
    if pr:
        name += ", precise walkers (FP64 window sums at every radius)"
    t = {k: prob[k].to(dev) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    eps = torch.tensor(prob["eps"], dtype=torch.float32, device=dev)
    q = torch.empty_like(t["I_hi"])
    outs = (torch.empty(t["I_lo"].shape, dtype=torch.float32, device=dev),
            torch.empty(t["p_lo"].shape, dtype=torch.float32, device=dev),
            torch.empty_like(t["I_hi"]),
            torch.empty(1, dtype=torch.float32, device=dev))
    desc = gf.make_desc(t["I_lo"], t["I_hi"], r, precise=pr)
    ws = torch.empty(gf.gf_workspace_size(desc, None, 2), dtype=torch.uint8, device=dev)

    def step():
        gf.forward_backward(t["I_lo"], t["p_lo"], t["I_hi"], eps, t["dq"], r, ws=ws,
                            outs=(q,) + outs, precise=pr)

    def separate_step():
        gf.forward(t["I_lo"], t["p_lo"], t["I_hi"], eps, r, out=q, ws=ws, precise=pr)
        gf.backward(t["I_lo"], t["p_lo"], t["I_hi"], eps, t["dq"], r, ws=ws, outs=outs,
                    precise=pr)

    kb = identity_bytes(n, c, H, W, h, w, BYTES[dt])
    # one gf_forward_backward call: the coefficient pass, one fused high-res
    # pass (I_h, dq in; q, dI_h out), the low-res backward, the eps sum
    per_step = {"gf_fwd_bwd_hi": kb["apply"] + kb["bwd_hi"] - BYTES[dt] * n * c * H * W,
                "gf_coef": kb["coef"], "gf_bwd_lo": kb["bwd_lo"], "gf_eps_reduce": 0}
    step_bytes = per_step["gf_fwd_bwd_hi"] + kb["coef"] + kb["bwd_lo"]

    I_lo = t["I_lo"].clone().requires_grad_(True)
    p_lo = t["p_lo"].clone().requires_grad_(True)
    I_hi = t["I_hi"].clone().requires_grad_(True)
    eps_p = eps.clone().requires_grad_(True)

    def plain_step():
        for x in (I_lo, p_lo, I_hi, eps_p):
            x.grad = None
        plain.guided_filter(I_lo, p_lo, I_hi, r, eps_p).backward(t["dq"].float())

    def cpu_sample():
        import oracle
        args_np = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        dq_np = prob["dq"].double().numpy()
        reps, t0 = 0, time.perf_counter()
        while True:
            ref = {"q": oracle.forward(*args_np, r, prob["eps"])}
            ref.update(oracle.backward(*args_np, r, prob["eps"], dq_np))
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or reps >= 20:
                break
        torch.cuda.synchronize()
        got = {"q": q.double().cpu().numpy(), "dI_lo": outs[0].double().cpu().numpy(),
               "dp_lo": outs[1].double().cpu().numpy(), "dI_hi": outs[2].double().cpu().numpy(),
               "deps": outs[3].double().cpu().numpy()}
        return (n * H * W / 1e6 * reps, el,
                f"the full {n}-image batch, fwd+bwd, repeated {reps}x ({el:.1f} s); parallel "
                f"over the {n * c} image planes", n * c, oracle_errors(got, ref))

    def cpu_one():
        import oracle
        args1 = [prob[k][:1].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        t0 = time.perf_counter()
        oracle.forward(*args1, r, prob["eps"][:1])
        oracle.backward(*args1, r, prob["eps"][:1], prob["dq"][:1].double().numpy())
        return H * W / 1e6, time.perf_counter() - t0, "image 0 of the batch, fwd+bwd once"

    def tune():
        gf.autotune(t["I_lo"], t["p_lo"], t["I_hi"], eps, t["dq"], r=r, iters=5, precise=pr)

    # the layer as a training step would call it: the autograd function's
    # forward (gf_forward) and backward (gf_backward, recomputing the
    # coefficients), gradients to every input
    leaves = [t[k].clone().requires_grad_(True) for k in ("I_lo", "p_lo", "I_hi")]
    eps_leaf = eps.clone().requires_grad_(True)

    def autograd_step():
        for x in leaves + [eps_leaf]:
            x.grad = None
        gf.guided_filter(*leaves, r=r, eps=eps_leaf, precise=pr).backward(t["dq"])

    return dict(step=step, separate_step=separate_step, plain_step=plain_step,
                cpu_sample=cpu_sample, cpu_one=cpu_one, autograd_step=autograd_step,
                mpx=n * H * W / 1e6, tune=tune,
                per_step=per_step, step_bytes=step_bytes, dtype=dt,
                config={"workload": name, "n": n, "c": c, "H": H, "W": W, "s": prob["s"], "r": r,
                        "eps": float(prob["eps"][0]), **({"precise": True} if pr else {})},
                traffic_ok=(dt == "f32" and n == 4 and H == 2048 and W == 3072 and not pr))


def workload_2(args, dev):
    import numpy as np
    import torch

    from paper_1803_05619_amd import datagen, gf, plain
    log("generating workload 2 (BF16 8x3x1536x2048, trainable guide)")
    prob = datagen.make_config(2)
    n, c, H, W, h, w, r = (prob[k] for k in ("n", "c", "H", "W", "h", "w", "r"))
    gp = prob["guide"]
    K = np.asarray(gp["w1"]).shape[0]
    t = {k: prob[k].to(dev) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    eps = torch.tensor(prob["eps"], dtype=torch.float32, device=dev)
    params = gf.pack_transform_params(gp["w1"], gp["w2"], gp["b2"], gp["lam"], gp["mu"],
                                      gp["gamma"], gp["beta"], device=dev)
    stats = torch.empty(gf.gf_guide_stats_count(3), dtype=torch.float32, device=dev)
    g_fwd = gf.Guide(gf.GF_GUIDE_TRANSFORM, 3, K, params, gp["bn_eps"], gp["slope"], stats, False)
    g_bwd = gf.Guide(gf.GF_GUIDE_TRANSFORM, 3, K, params, gp["bn_eps"], gp["slope"], stats, True)
    q = torch.empty_like(t["I_hi"])
    f32 = dict(dtype=torch.float32, device=dev)
    dp_lo = torch.empty(t["p_lo"].shape, **f32)
    deps = torch.empty(1, **f32)
    dparams = torch.empty(gf.gf_guide_param_count(3, 3, K), **f32)
    desc = gf.make_desc(t["I_lo"], t["I_hi"], r)
    ws = torch.empty(gf.gf_workspace_size(desc, g_fwd.struct(), 2), dtype=torch.uint8,
                     device=dev)

    def step():
        gf.forward_backward(t["I_lo"], t["p_lo"], t["I_hi"], eps, t["dq"], r, ws=ws, guide=g_fwd,
                            outs=(q, None, dp_lo, None, deps, dparams))

    def separate_step():
        gf.forward(t["I_lo"], t["p_lo"], t["I_hi"], eps, r, out=q, ws=ws, guide=g_fwd)
        gf.backward(t["I_lo"], t["p_lo"], t["I_hi"], eps, t["dq"], r, ws=ws, guide=g_bwd,
                    outs=(None, dp_lo, None, deps, dparams))

    b = 2
    hi, lo = n * c * H * W, n * c * h * w
    hpx, lpx = n * H * W, n * h * w
    # each kernel's own compulsory I/O per step (G planes are float32)
    per_step = {
        "gf_guide_moments": 3 * b * (hpx + lpx),
        "gf_guide_map": (3 * b + 12) * (hpx + lpx),
        "gf_coef": (4 + b) * lo,
        "gf_fwd_bwd_hi": (4 + b + b + 4) * hi,     # G_h, dq in; q, dG_h out
        "gf_bwd_lo": (4 + b + 4 + 4) * lo,
        "gf_guide_bwd": (3 * b + 12) * (hpx + lpx),
    }
    # the step's compulsory bytes: inputs read once per pass, outputs once
    step_bytes = 2 * b * hi + 2 * b * lo + 2 * b * hi + 2 * b * lo + 4 * lo

    w1, w2, b2, gam, bet = (torch.tensor(np.asarray(gp[k]), **f32)
                            for k in ("w1", "w2", "b2", "gamma", "beta"))
    leaves = [x.clone().requires_grad_(True) for x in (w1, w2, b2, gam, bet)]
    lam_t = torch.tensor(float(gp["lam"]), **f32).requires_grad_(True)
    mu_t = torch.tensor(float(gp["mu"]), **f32).requires_grad_(True)
    p_lo = t["p_lo"].clone().requires_grad_(True)
    eps_p = eps.clone().requires_grad_(True)

    def plain_step():
        for x in leaves + [lam_t, mu_t, p_lo, eps_p]:
            x.grad = None
        G_lo = plain.guide_transform(t["I_lo"], leaves[0], leaves[1], leaves[2], lam_t, mu_t,
                                     leaves[3], leaves[4], gp["bn_eps"], gp["slope"])
        G_hi = plain.guide_transform(t["I_hi"], leaves[0], leaves[1], leaves[2], lam_t, mu_t,
                                     leaves[3], leaves[4], gp["bn_eps"], gp["slope"])
        plain.guided_filter(G_lo, p_lo, G_hi, r, eps_p).backward(t["dq"].float())

    def cpu_sample():
        import oracle
        args_np = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        dq_np = prob["dq"].double().numpy()
        reps, t0 = 0, time.perf_counter()
        while True:
            ref = {"q": oracle.forward(*args_np, r, prob["eps"], guide=gp)}
            ref.update(oracle.backward(*args_np, r, prob["eps"], dq_np, guide=gp))
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or reps >= 20:
                break
        torch.cuda.synchronize()
        got = {"q": q.double().cpu().numpy(), "dp_lo": dp_lo.double().cpu().numpy(),
               "deps": deps.double().cpu().numpy(), "dguide": dparams.double().cpu().numpy()}
        return (n * H * W / 1e6 * reps, el,
                f"the full {n}-image batch, fwd+bwd with the guide, repeated {reps}x "
                f"({el:.1f} s); parallel over the {n * c} image planes", n * c,
                oracle_errors(got, ref, K))

    def tune():
        gf.autotune(t["I_lo"], t["p_lo"], t["I_hi"], eps, t["dq"], r=r, iters=5, guide=g_fwd)

    def cpu_one():
        import oracle
        args1 = [prob[k][:1].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        t0 = time.perf_counter()
        oracle.forward(*args1, r, prob["eps"], guide=gp)
        oracle.backward(*args1, r, prob["eps"], prob["dq"][:1].double().numpy(), guide=gp)
        return (H * W / 1e6, time.perf_counter() - t0,
                "image 0 alone (its own batch statistics), fwd+bwd with the guide once")

    # autograd step: gradients to p_l, eps and the guide parameters
    params_leaf = params.clone().requires_grad_(True)
    p_leaf = t["p_lo"].clone().requires_grad_(True)
    eps_leaf = eps.clone().requires_grad_(True)
    g_ag = gf.Guide(gf.GF_GUIDE_TRANSFORM, 3, K, params_leaf, gp["bn_eps"], gp["slope"])

    def autograd_step():
        for x in (params_leaf, p_leaf, eps_leaf):
            x.grad = None
        gf.guided_filter(t["I_lo"], p_leaf, t["I_hi"], r=r, eps=eps_leaf,
                         guide=g_ag).backward(t["dq"])

    # the guide backward is arithmetic-bound: per pixel and hidden unit the
    # pre-activation (6 flops), its branch (1), the W2 gradient sums (6),
    # dz = W2^T dG (5), dy (1), the sums of dy and of dy (x - mean) (1 + 6);
    # per pixel the sums of dG and the centred input (6); both calls
    flops = {"gf_guide_bwd": (n * H * W + n * h * w) * (26 * K + 6)}
    return dict(step=step, separate_step=separate_step, plain_step=plain_step,
                cpu_sample=cpu_sample, cpu_one=cpu_one, autograd_step=autograd_step,
                mpx=n * H * W / 1e6, tune=tune, flops=flops,
                per_step=per_step, step_bytes=step_bytes, dtype="bf16",
                config={"workload": "trainable-guide guided filtering fwd+bwd, BF16 I/O + FP32 "
                                    "accumulate, 8x3x1536x2048 <- 384x512 (s=4), r=1, eps=1e-8, "
                                    "guide 3->15->3 with adaptive BN and leaky ReLU 0.2, grads "
                                    "to p_l, eps and the guide parameters",
                        "n": n, "c": c, "H": H, "W": W, "s": prob["s"], "r": r, "eps": 1e-8,
                        "hidden": K},
                traffic_ok=False)


def workload_3(args, dev):
    from concurrent.futures import ThreadPoolExecutor

    import torch

    from paper_1803_05619_amd import datagen, gf, plain
    specs = datagen.batched_specs(args.items)
    log(f"generating workload 3 ({len(specs)} uneven images)")
    probs = [None] * len(specs)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    # threads in this process (numpy and torch release the GIL in the bulk
    # work): no child processes, which a profiler would attach to as well
    with ThreadPoolExecutor(workers) as pool:
        for k, p in enumerate(pool.map(datagen.batched_item, specs)):
            probs[k] = p
            if (k + 1) % 8 == 0:
                log(f"  {k + 1}/{len(specs)} images")
    items = []
    f32 = dict(dtype=torch.float32, device=dev)
    for p in probs:
        it = {k: p[k].to(dev) for k in ("I_lo", "p_lo", "I_hi", "dq")}
        it.update(r=p["r"], eps=float(p["eps"][0]), mean_ab=True)
        it["q"] = torch.empty_like(it["I_hi"])
        it["dI_hi"] = torch.empty_like(it["I_hi"])
        it["dI_lo"] = torch.empty(it["I_lo"].shape, **f32)
        it["dp_lo"] = torch.empty(it["p_lo"].shape, **f32)
        it["deps"] = torch.empty(1, **f32)
        items.append(it)
    if args.autotune != 0:
        log(f"autotuned {gf.autotune_batch(items)} launch-shape keys")
    log("tuned shapes: " + gf.gf_tune_export().strip().replace("\n", "; "))
    plan = gf.BatchPlan(items)

    def step():
        plan.run(gf.GF_RUN_FORWARD | gf.GF_RUN_BACKWARD, graph=True)

    # kernel records are per launch class: radius (low-res) or factor (high-res)
    per_step = {"gf_eps_multi": 0}
    step_bytes = 0
    mpx = 0.0
    for p in probs:
        kb = identity_bytes(1, 3, p["H"], p["W"], p["h"], p["w"], 4)
        # forward+backward plan: the high-res pass is fused (I_h, dq in; q,
        # dI_h out)
        fused_hi = kb["apply"] + kb["bwd_hi"] - 4 * 3 * p["H"] * p["W"]
        for name, nbytes in ((f"gf_coef_multi_r{p['r']}", kb["coef"]),
                             (f"gf_bwd_hi_multi_s{p['s']}", fused_hi),
                             (f"gf_bwd_lo_multi_r{p['r']}", kb["bwd_lo"])):
            per_step[name] = per_step.get(name, 0) + nbytes
        step_bytes += fused_hi + kb["coef"] + kb["bwd_lo"]
        mpx += p["H"] * p["W"] / 1e6

    leaves = [{k: it[k].clone().requires_grad_(True) for k in ("I_lo", "p_lo", "I_hi")}
              for it in items]
    eps_t = [torch.tensor([it["eps"]], **f32).requires_grad_(True) for it in items]

    def plain_step():
        for lv, e, it in zip(leaves, eps_t, items):
            for x in list(lv.values()) + [e]:
                x.grad = None
            plain.guided_filter(lv["I_lo"], lv["p_lo"], lv["I_hi"], it["r"], e).backward(it["dq"])

    def cpu_sample():
        import oracle
        err, done, t0, k = {}, 0.0, time.perf_counter(), 0
        torch.cuda.synchronize()
        while k < len(probs):
            p, it = probs[k], items[k]
            args_np = [p[x].double().numpy() for x in ("I_lo", "p_lo", "I_hi")]
            ref = {"q": oracle.forward(*args_np, p["r"], p["eps"])}
            ref.update(oracle.backward(*args_np, p["r"], p["eps"], p["dq"].double().numpy()))
            got = {x: it[x].double().cpu().numpy() for x in ("q", "dI_lo", "dp_lo", "dI_hi",
                                                             "deps")}
            merge_max(err, oracle_errors(got, ref))
            done += p["H"] * p["W"] / 1e6
            k += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        return (done, el, f"the first {k} of the {len(probs)} images, fwd+bwd each once "
                          f"({el:.1f} s); parallel over each image's 3 planes", 3, err)

    def eager_step():
        plan.run(gf.GF_RUN_FORWARD | gf.GF_RUN_BACKWARD, graph=False)

    def cpu_one():
        import oracle
        p = probs[0]
        args_np = [p[x].double().numpy() for x in ("I_lo", "p_lo", "I_hi")]
        t0 = time.perf_counter()
        oracle.forward(*args_np, p["r"], p["eps"])
        oracle.backward(*args_np, p["r"], p["eps"], p["dq"].double().numpy())
        return (p["H"] * p["W"] / 1e6, time.perf_counter() - t0,
                f"image 0 ({p['H']}x{p['W']}, s={p['s']}, r={p['r']}), fwd+bwd once")

    return dict(step=step, eager_step=eager_step, plain_step=plain_step, cpu_sample=cpu_sample,
                cpu_one=cpu_one,
                mpx=mpx, per_step=per_step, step_bytes=step_bytes, dtype="f32",
                config={"workload": f"batched uneven guided filtering fwd+bwd, FP32, "
                                    f"{len(probs)} images H,W in [512,3072], s in {{2,4,8}}, "
                                    f"r in {{1,2,4}}, eps in [1e-8,1e-2]; one plan replayed as "
                                    f"a HIP graph, autotuned launch shapes",
                        "images": len(probs), "Mpx_per_step": round(mpx, 2)},
                traffic_ok=False, keep=plan)


def workload_0(args, dev):
    """Forward only, 1 x 3 x 256 x 256 from 64 x 64: one gf_forward call per
    step (a few microseconds: launch-latency bound)."""
    import torch

    from paper_1803_05619_amd import datagen, gf, plain
    prob = datagen.make_config(0, with_dq=False)
    n, c, H, W, h, w, r = (prob[k] for k in ("n", "c", "H", "W", "h", "w", "r"))
    t = {k: prob[k].to(dev) for k in ("I_lo", "p_lo", "I_hi")}
    eps = torch.tensor(prob["eps"], dtype=torch.float32, device=dev)
    q = torch.empty_like(t["I_hi"])
    desc = gf.make_desc(t["I_lo"], t["I_hi"], r)
    ws = torch.empty(gf.gf_workspace_size(desc, None, 0), dtype=torch.uint8, device=dev)

    def step():
        gf.forward(t["I_lo"], t["p_lo"], t["I_hi"], eps, r, out=q, ws=ws)

    kb = identity_bytes(n, c, H, W, h, w, 4)

    def plain_step():
        with torch.no_grad():
            plain.guided_filter(t["I_lo"], t["p_lo"], t["I_hi"], r, eps)

    def cpu_sample():
        import oracle
        args_np = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        reps, t0 = 0, time.perf_counter()
        while True:
            ref = {"q": oracle.forward(*args_np, r, prob["eps"])}
            reps += 1
            el = time.perf_counter() - t0
            if el >= min(args.cpu_seconds, 2.0) or reps >= 200:
                break
        torch.cuda.synchronize()
        return (n * H * W / 1e6 * reps, el,
                f"the 1-image forward repeated {reps}x ({el:.2f} s)", n * c,
                oracle_errors({"q": q.double().cpu().numpy()}, ref))

    def cpu_one():
        import oracle
        args_np = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 1.0:
            oracle.forward(*args_np, r, prob["eps"])
            reps += 1
        return n * H * W / 1e6 * reps, time.perf_counter() - t0, f"the forward, {reps}x"

    return dict(step=step, plain_step=plain_step, cpu_sample=cpu_sample, cpu_one=cpu_one,
                mpx=n * H * W / 1e6,
                per_step={"gf_coef": kb["coef"], "gf_apply": kb["apply"]},
                step_bytes=kb["coef"] + kb["apply"], dtype="f32",
                config={"workload": "guided filtering layer forward only, FP32, 1x3x256x256 <- "
                                    "64x64 (s=4), r=1, eps=1e-2 (launch-latency bound)",
                        "n": n, "c": c, "H": H, "W": W, "s": prob["s"], "r": r, "eps": 1e-2},
                traffic_ok=False)


def conv_params_np(seed, c=3, K=16):
    """Random parameters of the convolutional layer at the scale of photo
    statistics (positive taps; W1 large enough that the hidden units leave
    zero on cov, var ~ 1e-3 .. 1e-2)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return {"D": rng.uniform(0.2, 1.0, size=(c, 3, 3)), "W1": rng.normal(0, 40.0, size=(K, 2 * c)),
            "W2": rng.normal(0, 0.4, size=(K, K)), "W3": rng.normal(0, 0.4, size=(c, K)),
            "slope": 0.2}


def workload_5(args, dev):
    """The convolutional guided filtering layer (Sec. III-E), forward then
    backward (gradients to p_l, I_l, I_h and the 427 parameters), FP32, on the
    4 x 3 x 2048 x 3072 images of workload 1, dilation r = 1."""
    import torch

    from paper_1803_05619_amd import datagen, gf, plain
    log("generating workload 5 (FP32 4x3x2048x3072, convolutional layer)")
    prob = datagen.make_config(1)
    n, c, H, W, h, w = (prob[k] for k in ("n", "c", "H", "W", "h", "w"))
    r, K = 1, 16
    P = conv_params_np(225)
    t = {k: prob[k].to(dev) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    params = gf.pack_conv_params(P["D"], P["W1"], P["W2"], P["W3"], device=dev)
    desc = gf.make_desc(t["I_lo"], t["I_hi"], r)
    cv = gf.gf_conv_t(K, P["slope"], params.data_ptr())
    ws = torch.empty(gf.gf_conv_workspace_size(desc, cv, 1), dtype=torch.uint8, device=dev)
    outs = {}

    def step():
        outs["q"] = gf.conv_forward(t["I_lo"], t["p_lo"], t["I_hi"], params, r, K, ws=ws)
        outs["g"] = gf.conv_backward(t["I_lo"], t["p_lo"], t["I_hi"], params, t["dq"], r, K,
                                     ws=ws)

    kb = identity_bytes(n, c, H, W, h, w, 4)
    # the statistics kernel runs in both calls (the backward recomputes them)
    per_step = {"gf_apply": kb["apply"], "gf_bwd_hi": kb["bwd_hi"],
                "gf_conv_stats": 2 * kb["coef"], "gf_conv_inputs_grad": kb["bwd_lo"]}
    step_bytes = kb["apply"] + kb["bwd_hi"] + 2 * kb["coef"] + kb["bwd_lo"]
    # the block kernel is arithmetic-bound: per low-res pixel the pointwise
    # block's forward (recomputed) and backward products (2 x (2cK + K^2 + cK)
    # FMA), the weight gradients' outer products (2cK + K^2 + cK FMA) and the
    # 9c dilated-conv weight terms (8 flops each)
    blk = 2 * c * K + K * K + c * K
    flops = {"gf_conv_bwd_block": n * h * w * (3 * 2 * blk + 8 * 9 * c)}
    tp = {k: torch.tensor(P[k], dtype=torch.float32, device=dev, requires_grad=True)
          for k in ("D", "W1", "W2", "W3")}
    leaves = [t[k].clone().requires_grad_(True) for k in ("I_lo", "p_lo", "I_hi")]

    def plain_step():
        for x in leaves + list(tp.values()):
            x.grad = None
        plain.conv_guided_filter(*leaves, r, tp["D"], tp["W1"], tp["W2"], tp["W3"]).backward(
            t["dq"])

    def cpu_sample():
        import oracle
        args_np = [prob[k][:1].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        dq_np = prob["dq"][:1].double().numpy()
        reps, t0 = 0, time.perf_counter()
        while True:
            ref = {"q": oracle.conv_forward(*args_np, r, P)}
            ref.update(oracle.conv_backward(*args_np, r, P, dq_np))
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or reps >= 20:
                break
        torch.cuda.synchronize()
        got = {"q": outs["q"][:1].double().cpu().numpy(),
               "dI_lo": outs["g"][0][:1].double().cpu().numpy(),
               "dp_lo": outs["g"][1][:1].double().cpu().numpy(),
               "dI_hi": outs["g"][2][:1].double().cpu().numpy()}
        return (H * W / 1e6 * reps, el,
                f"image 0 of the batch, fwd+bwd, repeated {reps}x ({el:.1f} s); parallel over "
                f"its images (1)", 1, oracle_errors(got, ref))

    return dict(step=step, plain_step=plain_step, cpu_sample=cpu_sample,
                mpx=n * H * W / 1e6, per_step=per_step, step_bytes=step_bytes, dtype="f32",
                config={"workload": "convolutional guided filtering layer fwd+bwd (Sec. III-E), "
                                    "FP32, 4x3x2048x3072 <- 512x768 (s=4), dilation 1, block "
                                    "6->16->16->3, grads to p_l, I_l, I_h and the parameters",
                        "n": n, "c": c, "H": H, "W": W, "s": 4, "r": r, "hidden": K},
                traffic_ok=False, flops=flops)


WORKLOADS = {0: workload_0, 1: workload_1, 2: workload_2, 3: workload_3, 4: workload_4,
             5: workload_5}


def dgf_sweep(args, dev):
    """The deep guided filtering network's inference chain (Sec. IV, Fig. 3):
    area downsampling to I_l (short side 64), the low-res network C_l (the
    context aggregation network of Table I with random weights, PyTorch
    convolutions) and the guided filtering layer (r = 1, eps = 1e-8), over
    square images 512^2 .. 3072^2 as in the paper's running-time figure
    (Sec. V-D), and over I_l sizes 32 .. 512 at 2048^2 as in Table IV.  Per
    size: median ms of the chain (eager, and replayed as a HIP graph), the
    share of each step, and the peak device memory."""
    import torch

    from paper_1803_05619_amd import datagen, dgf, gf

    net = dgf.CAN(seed=0).to(dev).eval()
    iters = max(5, args.timing_iters)

    def median_ms(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(iters)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) for a, b in ev)
        return ts[len(ts) // 2]

    def one(S, lo):
        rng = datagen.rng_for(5, S)
        x = datagen.quantize(datagen.photo(rng, 3, S, S, noise=0.02)[None], "f32").to(dev)
        h, w = dgf.low_res_size(S, S, lo)
        ws = torch.empty(gf.gf_workspace_size(gf.make_desc(torch.empty(1, 3, h, w), x, 1), None,
                                              0), dtype=torch.uint8, device=dev)
        eps = torch.full((1,), 1e-8, dtype=torch.float32, device=dev)
        with torch.no_grad():
            I_lo = gf.downsample(x, h, w)
            p_lo = net(I_lo).contiguous()
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated(dev)
        torch.cuda.reset_peak_memory_stats(dev)
        chain_ms = median_ms(lambda: dgf.dgf_forward(x, net, lo=lo, eps=eps, ws=ws))
        peak = torch.cuda.max_memory_allocated(dev)
        rec = {"H": S, "W": S, "h": h, "w": w, "ms": round(chain_ms, 4),
               "downsample_ms": round(median_ms(lambda: gf.downsample(x, h, w)), 4),
               "can_ms": round(median_ms(lambda: net(I_lo)), 4),
               "gf_layer_ms": round(median_ms(lambda: gf.forward(I_lo, p_lo, x, eps, 1, ws=ws)),
                                    4),
               "peak_mem_bytes": int(peak), "input_bytes": int(x.numel() * 4),
               "peak_mem_beyond_resident_bytes": int(peak - base)}
        rec["gf_layer_share"] = round(rec["gf_layer_ms"] / chain_ms, 3)
        # the chain replayed as one HIP graph (eps a device tensor: no host
        # copy during capture), compared replay by replay with eager runs
        try:
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                for _ in range(2):
                    out = dgf.dgf_forward(x, net, lo=lo, eps=eps, ws=ws)
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                out = dgf.dgf_forward(x, net, lo=lo, eps=eps, ws=ws)
            torch.cuda.synchronize()
            rec["graph_ms"] = round(median_ms(g.replay), 4)
            ref = dgf.dgf_forward(x, net, lo=lo, eps=eps, ws=ws)
            for _ in range(3):  # every replay, with eager work between
                g.replay()
                torch.cuda.synchronize()
                rec["graph_matches_eager"] = bool(torch.equal(out, ref))
                if not rec["graph_matches_eager"]:
                    break
                ref = dgf.dgf_forward(x, net, lo=lo, eps=eps, ws=ws)
            del g
        except Exception as e:
            rec["graph_ms"] = None
            rec["graph_error"] = f"{type(e).__name__}: {e}"[:200]
        log(f"DGF {S}^2 <- {h}x{w}: {rec}")
        del x, ws, I_lo, p_lo
        torch.cuda.empty_cache()
        return rec

    sweep = [one(S, 64) for S in (512, 1024, 1536, 2048, 2560, 3072)]
    table4 = [one(2048, lo) for lo in (32, 64, 96, 128, 256, 512)]
    at2048 = next(r for r in sweep if r["H"] == 2048)
    best = lambda r: min(v for v in (r["ms"], r.get("graph_ms")) if v is not None)
    out = {
        "metric": "deep guided filtering network inference (area downsampling + C_l + guided "
                  "filtering layer), ms per 2048x2048 image",
        "value": round(best(at2048), 4), "unit": "ms", "n_gpus": 1, "steps": iters,
        "warmup": 3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": DATA + "; C_l with random weights",
        "config": {"workload": "DGF_b inference, 1x3xSxS FP32, I_l short side 64, C_l = CAN "
                               "(Table I, 24 channels, dilations 1,1,2,4,8,16,1), r=1, "
                               "eps=1e-8"},
        "sweep_512_to_3072": sweep, "table4_low_res_sweep_at_2048": table4,
        "paper_context": {"hardware": "Nvidia Titan X (Pascal), Intel E5-2650 2.20GHz",
                          "DGF_b_ms_at_2048": 6, "DGF_b_under_ms_512_to_3072": 10,
                          "CAN_full_res_ms_at_2048": 160, "DGF_b_peak_mem_GB_at_3072": "< 1",
                          "table4_ms": {"32": 6, "64": 6, "96": 6, "128": 7, "256": 7, "512": 19},
                          "table4_mem_GB": {"32": 0.67, "64": 0.68, "96": 0.70, "128": 0.73,
                                            "256": 0.87, "512": 1.41}},
    }
    print(json.dumps(out), flush=True)


def flush_buffer(dev):
    import torch
    return torch.empty(512 << 20, dtype=torch.uint8, device=dev)


def step_stats(step, iters, flush):
    """Median, p10 and p90 (ms) of `iters` steps, each between two HIP events
    recorded on the current stream (the stream the library launches on);
    with `flush`, that buffer is written before each step, outside its
    events."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(iters)]
    for k, (a, b) in enumerate(ev):
        if flush is not None:
            flush.fill_(k & 255)
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)

    def pct(q):
        return round(ts[min(len(ts) - 1, int(q * (len(ts) - 1) + 0.5))], 4)
    return {"median": pct(0.5), "p10": pct(0.1), "p90": pct(0.9), "iters": iters}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", type=int, default=1, choices=sorted(WORKLOADS))
    ap.add_argument("--radius", type=int, default=None, help="workload 4: radius (default 8)")
    ap.add_argument("--items", type=int, default=64, help="workload 3: images")
    ap.add_argument("--precise", action="store_true",
                    help="workloads 1 and 4: the precise option (FP64 wide walkers at every "
                         "radius)")
    ap.add_argument("--autotune", type=int, default=-1,
                    help="1: run the autotuner on the workload before timing (untimed); "
                         "0: the planner's default shapes; default: 1 for workload 3 (the "
                         "uneven batch), 0 otherwise (the defaults are the tuned shapes of "
                         "workload 1)")
    ap.add_argument("--timing-iters", type=int, default=50,
                    help="steps per event-timed pass (warm, and cold after a 512 MB flush)")
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain PyTorch leg")
    ap.add_argument("--dgf", action="store_true",
                    help="time the deep guided filtering network's inference chain over "
                         "512^2..3072^2 and the I_l sizes of Table IV instead of a workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one 1 GiB device copy (torch copy_) as a known-size "
                         "reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the layer "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1803_05619_amd import gf

    dev = torch.device("cuda:0")
    if args.dgf:
        dgf_sweep(args, dev)
        return
    if args.copy_probe:
        src = torch.ones(256 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
        del src, dst
    wl = WORKLOADS[args.workload](args, dev)
    step = wl["step"]
    if args.autotune < 0:
        args.autotune = 1 if args.workload == 3 else 0
    if args.autotune and "tune" in wl:
        log("autotuning the launch shapes (untimed)")
        wl["tune"]()
        log("tuned shapes: " + gf.gf_tune_export().strip().replace("\n", "; "))

    log(f"warmup {args.warmup} steps")
    torch.cuda.reset_peak_memory_stats(dev)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    value = wl["mpx"] * args.steps / sec
    ms_per_step = 1e3 * sec / args.steps
    peak_mem = torch.cuda.max_memory_allocated(dev)
    log(f"fused: {ms_per_step:.4f} ms/step, {value:.1f} Mpx/s")
    # per-step times: HIP events around each step on the launch stream, warm
    # (steps back to back) and cold (a 512 MB buffer written before each
    # step, outside the events, so the 256 MB MALL and the L2s hold none of
    # the step's data)
    timing = {"warm": step_stats(step, args.timing_iters, None),
              "cold": step_stats(step, args.timing_iters, flush_buffer(dev))}
    log(f"per-step ms: warm {timing['warm']}, cold (flushed) {timing['cold']}")
    # a step is its own launch sequence; per call in microseconds as well
    us_per_step = 1e3 * ms_per_step
    # the kernel breakdown: the same steps again with a HIP event pair
    # around every launch (recording events adds host and device time, so
    # this pass is not the one `value` comes from)
    gf.gf_profile_enable(True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof_ms_per_step = 1e3 * (time.perf_counter() - p0) / args.steps
    prof = gf.gf_profile_read(64)
    gf.gf_profile_enable(False)
    log(f"profiled pass: {prof_ms_per_step:.4f} ms/step")

    prof_steps = args.steps
    if not prof and "eager_step" in wl:
        # graph replays record no per-kernel events: a separate eager pass
        # (same launches, not timed as the step) gives the kernel breakdown
        prof_steps = min(args.steps, 10)
        gf.gf_profile_enable(True)
        for _ in range(prof_steps):
            wl["eager_step"]()
        torch.cuda.synchronize()
        prof = gf.gf_profile_read(64)
        gf.gf_profile_enable(False)
    kernels = {}
    for name, (ms, cnt) in prof.items():
        b = wl["per_step"].get(name, 0)
        step_s = ms / prof_steps * 1e-3
        kernels[name] = {"avg_us": round(1e3 * ms / max(cnt, 1), 3), "launches": cnt,
                         "us_per_step": round(1e6 * step_s, 3), "algo_bytes_per_step": b,
                         "algo_GBs": round(b / step_s / 1e9, 1) if step_s > 0 else None}
        fl = wl.get("flops", {}).get(name, 0)
        if fl and step_s > 0:
            kernels[name]["algo_TFLOPs"] = round(fl / step_s / 1e12, 3)
    # graph replays record no per-kernel events: fall back to the whole step
    if prof:
        dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
        dom_s = prof[dom][0] / prof_steps * 1e-3
        dom_bytes = wl["per_step"].get(dom, 0)
    else:
        dom, dom_s, dom_bytes = "step (graph replay)", ms_per_step * 1e-3, wl["step_bytes"]
    dom_flops = wl.get("flops", {}).get(dom, 0)
    achieved = dom_bytes / dom_s / 1e9
    traffic = None
    if wl.get("traffic_ok") and os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_src_sha256_16") == kernel_hash() and dom in rec.get("kernels", {}):
            traffic = rec["kernels"][dom]["hbm_bytes_per_launch"]
    launches = prof[dom][1] / prof_steps if prof else 1
    tf = dom_flops / dom_s / 1e12 if dom_flops else 0.0
    if dom_flops and tf / FP32_VEC_PEAK_TFLOPS > achieved / HBM_PEAK_GBS:
        # the arithmetic roofline binds: algorithmic FP32 flops over the
        # kernel's time, against the FP32 vector peak
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(tf, 3),
                    "peak": FP32_VEC_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / FP32_VEC_PEAK_TFLOPS, 4), "traffic": None,
                    "algo_flops_per_launch": int(dom_flops / max(launches, 1)),
                    "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)}
    else:
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "algo_bytes_per_launch": int(dom_bytes / max(launches, 1))}
    step_gbs = wl["step_bytes"] / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"],
        "us_per_step": round(us_per_step, 2),
        "data": DATA, "config": wl["config"], "roofline": roofline,
        "timing_ms": timing, "peak_mem_bytes": int(peak_mem),
        "step_algo_GBs": round(step_gbs, 1), "kernels": kernels,
        "profiled_pass_ms_per_step": round(prof_ms_per_step, 4),
    }
    if "autograd_step" in wl:
        # the layer through its torch.autograd.Function: gf_forward, then
        # gf_backward when autograd reaches it
        for _ in range(3):
            wl["autograd_step"]()
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(args.steps):
            wl["autograd_step"]()
        torch.cuda.synchronize()
        ag_ms = 1e3 * (time.perf_counter() - a0) / args.steps
        out["autograd_step"] = {"ms_per_step": round(ag_ms, 4),
                                "value": round(wl["mpx"] / (ag_ms * 1e-3), 1),
                                "warm_ms": step_stats(wl["autograd_step"], args.timing_iters,
                                                      None)}
        log(f"autograd step: {ag_ms:.4f} ms/step")
    if "separate_step" in wl:
        # the same step as separate gf_forward and gf_backward calls (the
        # backward recomputing the coefficients), for comparison
        sep = max(10, args.steps // 4)
        for _ in range(3):
            wl["separate_step"]()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(sep):
            wl["separate_step"]()
        torch.cuda.synchronize()
        sep_ms = 1e3 * (time.perf_counter() - s0) / sep
        out["separate_calls"] = {"ms_per_step": round(sep_ms, 4),
                                 "value": round(wl["mpx"] / (sep_ms * 1e-3), 1),
                                 "steps": sep}
        log(f"separate gf_forward + gf_backward: {sep_ms:.4f} ms/step")
    if not args.no_plain:
        out["plain"] = plain_leg(args, wl, value)
    if not args.no_cpu:
        out["cpu_baseline"], out["error_vs_fp64_oracle"] = cpu_leg(args, wl)
    print(json.dumps(out), flush=True)


def plain_leg(args, wl, value):
    """The unfused PyTorch composition (autograd) on the same GPU and inputs."""
    import torch
    log(f"timing the plain PyTorch composition ({args.plain_steps} steps)")
    for _ in range(2):
        wl["plain_step"]()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for _ in range(args.plain_steps):
        wl["plain_step"]()
    torch.cuda.synchronize()
    plain_ms = 1e3 * (time.perf_counter() - p0) / args.plain_steps
    plain_val = wl["mpx"] / (plain_ms * 1e-3)
    torch.cuda.empty_cache()
    log(f"plain: {plain_ms:.3f} ms/step, {plain_val:.1f} Mpx/s")
    return {"value": round(plain_val, 1), "unit": "Mpixel/s", "ms_per_step": round(plain_ms, 3),
            "speedup_fused_vs_plain": round(value / plain_val, 2)}


def cpu_leg(args, wl):
    """The FP64 oracle on the host cores over a bounded sample, and the
    error of the timed run's final outputs on that sample."""
    import oracle
    log("CPU oracle leg (FP64, host cores)")
    mpx, el, sample, planes, err = wl["cpu_sample"]()
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    cores = min(threads, planes)
    cpu = {"value": round(mpx / el, 3), "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
           "sample": f"{sample}; OpenMP over planes ({threads} threads available)",
           "cpu_model": cpu_model(), "nproc": len(os.sched_getaffinity(0))}
    if "cpu_one" in wl:
        oracle.set_threads(1)
        try:
            mpx1, el1, sample1 = wl["cpu_one"]()
        finally:
            oracle.set_threads(threads)
        cpu["one_core"] = {"value": round(mpx1 / el1, 3), "unit": "Mpixel/s",
                           "sample": f"{sample1} ({el1:.1f} s) on 1 thread"}
    log(f"cpu oracle: {cpu['value']} Mpx/s; errors {err}")
    return cpu, {k: float(f"{v:.3e}") for k, v in err.items()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
