"""Full-size GPU parity: the trainable-guide BF16 workload, the FP16 stress
workload (r = 8 and r = 1) and the uneven batch, each at its full size and in
the launch configuration bench.py times (one gf_forward_backward call; the
batch as an autotuned plan replayed as a HIP graph), against the FP64 oracle.
Error measures and bars: tests/parity.py.  The uneven batch is compared on
a sample of its images (every fourth); the others on every output."""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_1803_05619_amd import datagen
from tests import parity

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _gf():
    from paper_1803_05619_amd import gf
    return gf


def test_config2_full_size():
    """8 x 3 x 1536 x 2048 BF16 with the 3-15-3 transform guide, r=1,
    eps=1e-8: q, dp_l, dI_l, dI_h, deps and every guide parameter gradient."""
    gf = _gf()
    prob = datagen.make_config(2)
    g = prob["guide"]
    print("case config 2 full size", flush=True)
    d = {k: prob[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    params = gf.pack_transform_params(g["w1"], g["w2"], g["b2"], g["lam"], g["mu"], g["gamma"],
                                      g["beta"], device=DEV)
    guide = gf.Guide(gf.GF_GUIDE_TRANSFORM, 3, np.asarray(g["w1"]).shape[0], params,
                     g["bn_eps"], g["slope"])
    out = gf.forward_backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], prob["r"],
                              guide=guide)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in
           zip(("q", "dI_lo", "dp_lo", "dI_hi", "deps", "dparams"), out)}
    del d, out
    torch.cuda.empty_cache()
    args = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
    ref = {"q": oracle.forward(*args, prob["r"], prob["eps"], guide=g)}
    ref.update(oracle.backward(*args, prob["r"], prob["eps"], prob["dq"].double().numpy(),
                               guide=g))
    amb = {"dI_lo": parity.branch_ambiguous(args[0], g),
           "dI_hi": parity.branch_ambiguous(args[2], g)}
    print("branch-ambiguous pixels:", {k: int(v.sum()) for k, v in amb.items()}, flush=True)
    ref_flip = parity.flipped_reference(args, prob["r"], prob["eps"],
                                        prob["dq"].double().numpy(), g)
    n, h, w, H, W = prob["n"], prob["h"], prob["w"], prob["H"], prob["W"]
    parity.check(parity.measure(got, ref, "bf16", n_eps_terms=n * 3 * h * w,
                                n_guide_terms=n * (h * w + H * W),
                                hidden=np.asarray(g["w1"]).shape[0], amb=amb, ref_flip=ref_flip),
                 "config 2 full size")


@pytest.mark.parametrize("r", [8, 1])
def test_config4_full_size(r):
    """2 x 3 x 2160 x 3840 FP16 with near-constant patches, eps=1e-8."""
    gf = _gf()
    prob = datagen.make_config(4, r=r)
    print(f"case config 4 full size r={r}", flush=True)
    d = {k: prob[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    out = gf.forward_backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], r)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in
           zip(("q", "dI_lo", "dp_lo", "dI_hi", "deps"), out[:5])}
    args = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
    ref = {"q": oracle.forward(*args, r, prob["eps"])}
    ref.update(oracle.backward(*args, r, prob["eps"], prob["dq"].double().numpy()))
    parity.check(parity.measure(got, ref, "f16",
                                n_eps_terms=prob["n"] * 3 * prob["h"] * prob["w"]),
                 f"config 4 full size r={r}")


def test_config3_full_size():
    """The 64 uneven images (H, W in [512, 3072], s in {2, 4, 8}, r in
    {1, 2, 4}, eps in [1e-8, 1e-2]), FP32: one autotuned batched plan,
    forward and backward replayed as a HIP graph twice; every fourth image
    compared with the oracle, every image bit-identical across replays."""
    gf = _gf()
    specs = datagen.batched_specs(64)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as pool:  # numpy releases the GIL in the bulk work
        probs = list(pool.map(datagen.batched_item, specs))
    print(f"case config 3 full size: {len(probs)} images", flush=True)
    f32 = dict(dtype=torch.float32, device=DEV)
    items = []
    for p in probs:
        it = {k: p[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
        it.update(r=p["r"], eps=float(p["eps"][0]), mean_ab=True)
        it["q"] = torch.empty_like(it["I_hi"])
        it["dI_hi"] = torch.empty_like(it["I_hi"])
        it["dI_lo"] = torch.empty(it["I_lo"].shape, **f32)
        it["dp_lo"] = torch.empty(it["p_lo"].shape, **f32)
        it["deps"] = torch.empty(1, **f32)
        items.append(it)
    gf.autotune_batch(items)
    plan = gf.BatchPlan(items)
    plan.run(graph=True)
    torch.cuda.synchronize()
    first = [{k: it[k].clone() for k in ("q", "dI_lo", "dp_lo", "dI_hi", "deps")}
             for it in items]
    plan.run(graph=True)
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        for name, v in first[k].items():
            assert torch.equal(v, it[name]), (k, name)
    del first
    worst = {}
    for k in range(0, len(probs), 4):
        p, it = probs[k], items[k]
        args = [p[x].double().numpy() for x in ("I_lo", "p_lo", "I_hi")]
        ref = {"q": oracle.forward(*args, p["r"], p["eps"])}
        ref.update(oracle.backward(*args, p["r"], p["eps"], p["dq"].double().numpy()))
        got = {x: it[x].double().cpu().numpy() for x in ("q", "dI_lo", "dp_lo", "dI_hi", "deps")}
        res = parity.measure(got, ref, "f32", n_eps_terms=3 * p["h"] * p["w"])
        print(f"image {k}: H={p['H']} W={p['W']} s={p['s']} r={p['r']}", flush=True)
        for name, (e, bar) in res.items():
            # informational entries (infinite bar) keep their largest error
            if name not in worst or (e / bar if math.isfinite(bar) else e) > \
                    (worst[name][0] / bar if math.isfinite(bar) else worst[name][0]):
                worst[name] = (e, bar)
    plan.close()
    parity.check(worst, "config 3 sampled images (worst)")
