"""Batched plans on the GPU (gf_plan_create / gf_batched): every item of an
uneven batch must equal the single-problem calls bit for bit (same kernels,
same launch shapes), in every mode, as a persistent grid-stride launch and
as a replayed HIP graph; sampled items are also checked against the FP64
oracle (bars as in test_gpu_parity.py)."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1803_05619_amd import datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TOL = {"f32": 1e-4, "bf16": 2e-2, "f16": 2e-2}


def _gf():
    from paper_1803_05619_amd import gf
    return gf


def uneven_items(count, div, io_dtype="f32", extra=True):
    """The uneven-batch recipe at reduced size, plus edge items: a width that
    forces the scalar high-res path, Algorithm 1's form (no window mean of
    A and b), s = 1, two images in one item, and radii that take the wide
    low-res backward (a low-res width over one 256-column strip; a low-res
    image smaller than its windows)."""
    probs = datagen.batched_items(count, div=div, io_dtype=io_dtype)
    for p in probs:
        p["mean_ab"] = True
    if extra:
        e1 = datagen.make_problem(1, 3, 2 * 40, 2 * 37, 2, 1, 1e-3, io_dtype, config=140)
        e2 = datagen.make_problem(1, 3, 4 * 30, 4 * 44, 4, 2, 1e-2, io_dtype, config=141)
        e3 = datagen.make_problem(1, 3, 96, 64, 1, 3, 1e-4, io_dtype, config=142)
        e4 = datagen.make_problem(2, 3, 8 * 16, 8 * 20, 8, 1, 1e-3, io_dtype, config=143)
        e5 = datagen.make_problem(1, 3, 4 * 24, 4 * 36, 4, 1, 1e-3, io_dtype, config=144)
        e1["mean_ab"], e2["mean_ab"], e3["mean_ab"], e4["mean_ab"] = True, False, True, True
        e5["mean_ab"], e5["align_corners"] = True, True
        e6 = datagen.make_problem(1, 3, 4 * 70, 4 * 300, 4, 6, 1e-3, io_dtype, config=145)
        e7 = datagen.make_problem(1, 3, 2 * 9, 2 * 11, 2, 5, 1e-2, io_dtype, config=146)
        e6["mean_ab"], e7["mean_ab"] = True, False
        probs += [e1, e2, e3, e4, e5, e6, e7]
    return probs


def device_items(probs):
    items = []
    for p in probs:
        it = {k: p[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
        it.update(r=p["r"], eps=float(np.atleast_1d(p["eps"])[0]), mean_ab=p["mean_ab"],
                  align_corners=p.get("align_corners", False), precise=p.get("precise", False))
        it["q"] = torch.empty_like(it["I_hi"])
        it["dI_hi"] = torch.empty_like(it["I_hi"])
        it["dI_lo"] = torch.empty(it["I_lo"].shape, dtype=torch.float32, device=DEV)
        it["dp_lo"] = torch.empty(it["p_lo"].shape, dtype=torch.float32, device=DEV)
        it["deps"] = torch.empty(1, dtype=torch.float32, device=DEV)
        items.append(it)
    return items


def singles(gf, it):
    ac, pr = it.get("align_corners", False), it.get("precise", False)
    q = gf.forward(it["I_lo"], it["p_lo"], it["I_hi"], it["eps"], it["r"], it["mean_ab"],
                   align_corners=ac, precise=pr)
    g = gf.backward(it["I_lo"], it["p_lo"], it["I_hi"], it["eps"], it["dq"], it["r"],
                    it["mean_ab"], align_corners=ac, precise=pr)
    return {"q": q, "dI_lo": g[0], "dp_lo": g[1], "dI_hi": g[2], "deps": g[3]}


def assert_equal_to_singles(gf, items, keys=("q", "dI_lo", "dp_lo", "dI_hi", "deps")):
    for k, it in enumerate(items):
        ref = singles(gf, it)
        torch.cuda.synchronize()
        for name in keys:
            assert torch.equal(it[name], ref[name]), (k, name)


def print_case(probs):
    desc = [(tuple(p["I_hi"].shape), p["s"] if "s" in p else None, p["r"]) for p in probs]
    print("batch:", len(probs), "items", desc[:6], "...", flush=True)


def test_batched_equals_single_calls():
    gf = _gf()
    probs = uneven_items(10, div=6)
    print_case(probs)
    items = device_items(probs)
    plan = gf.BatchPlan(items)
    plan.run(gf.GF_RUN_FORWARD | gf.GF_RUN_BACKWARD)
    torch.cuda.synchronize()
    assert_equal_to_singles(gf, items)
    plan.close()


def test_batched_precise_items():
    """Precise and default items of the same radius run in separate launch
    classes (FP64 wide walkers and column walkers); each equals its single
    calls bit for bit."""
    gf = _gf()
    probs = uneven_items(8, div=6, extra=False)
    for k, p in enumerate(probs):
        p["precise"] = k % 2 == 0
    print_case(probs)
    items = device_items(probs)
    plan = gf.BatchPlan(items)
    plan.run(gf.GF_RUN_FORWARD | gf.GF_RUN_BACKWARD)
    torch.cuda.synchronize()
    assert_equal_to_singles(gf, items)
    plan.close()


def test_batched_modes_separately():
    gf = _gf()
    probs = uneven_items(5, div=8)
    items = device_items(probs)
    plan = gf.BatchPlan(items)
    plan.run(gf.GF_RUN_FORWARD)
    plan.run(gf.GF_RUN_BACKWARD)
    torch.cuda.synchronize()
    assert_equal_to_singles(gf, items)
    plan.close()


def test_batched_persistent_grid(monkeypatch):
    """A grid much smaller than the tile count: every workgroup walks many
    tiles of many items."""
    gf = _gf()
    monkeypatch.setenv("GF_BATCH_WGS", "7")
    probs = uneven_items(6, div=8)
    items = device_items(probs)
    plan = gf.BatchPlan(items)
    plan.run()
    torch.cuda.synchronize()
    monkeypatch.delenv("GF_BATCH_WGS")
    assert_equal_to_singles(gf, items)
    plan.close()


def test_batched_graph_replays():
    """The graph reads the items' buffers at each replay: new inputs between
    replays give the new results, every replay equal to the eager run."""
    gf = _gf()
    probs = uneven_items(6, div=8)
    items = device_items(probs)
    plan = gf.BatchPlan(items)
    gen = torch.Generator(device="cpu").manual_seed(5)
    for rep in range(3):
        for it in items:
            noise = torch.rand(it["dq"].shape, generator=gen).to(DEV, it["dq"].dtype)
            it["dq"].copy_(noise - 0.5)
        torch.cuda.synchronize()
        plan.run(graph=True)
        torch.cuda.synchronize()
        graph_out = [{k: it[k].clone() for k in ("q", "dI_lo", "dp_lo", "dI_hi", "deps")}
                     for it in items]
        plan.run(graph=False)
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            for name, v in graph_out[k].items():
                assert torch.equal(v, it[name]), (rep, k, name)
    plan.close()


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_batched_against_oracle(dt):
    gf = _gf()
    probs = uneven_items(4, div=8, io_dtype=dt)
    items = device_items(probs)
    plan = gf.BatchPlan(items)
    plan.run()
    torch.cuda.synchronize()
    for p, it in zip(probs, items):
        args = [p[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        eps = float(np.atleast_1d(p["eps"])[0])
        ac = p.get("align_corners", False)
        q = oracle.forward(*args, p["r"], eps, mean_ab=p["mean_ab"], align_corners=ac)
        g = oracle.backward(*args, p["r"], eps, p["dq"].double().numpy(), mean_ab=p["mean_ab"],
                            align_corners=ac)
        err = {"q": float(np.abs(it["q"].double().cpu().numpy() - q).max())}
        for k in ("dI_lo", "dp_lo", "dI_hi"):
            ref = g[k]
            err[k] = float(np.abs(it[k].double().cpu().numpy() - ref).max() /
                           max(1.0, np.abs(ref).max()))
        err["deps"] = float(abs(it["deps"].item() - g["deps"].sum()) /
                            max(1.0, g["deps_abs"].sum()))
        print(tuple(p["I_hi"].shape), p["r"], {k: f"{v:.2e}" for k, v in err.items()},
              flush=True)
        for k, v in err.items():
            assert v <= TOL[dt], (k, v)
    plan.close()


def test_batched_optional_outputs():
    """Items without backward outputs (and without deps) leave them alone."""
    gf = _gf()
    probs = uneven_items(3, div=8, extra=False)
    items = device_items(probs)
    items[1]["dI_lo"] = None
    items[1]["dI_hi"] = None
    items[2]["deps"] = None
    plan = gf.BatchPlan(items)
    plan.run()
    torch.cuda.synchronize()
    ref = singles(gf, items[0])
    torch.cuda.synchronize()
    assert torch.equal(items[0]["dI_hi"], ref["dI_hi"])
    ref1 = singles(gf, items[1])
    torch.cuda.synchronize()
    assert torch.equal(items[1]["dp_lo"], ref1["dp_lo"])
    plan.close()


def test_autotune_then_parity():
    gf = _gf()
    prob = datagen.make_config(1, div=8, n=2)
    d = {k: prob[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    gf.autotune(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], r=1, iters=2)
    text = gf.gf_tune_export()
    print("tuned:", text.strip(), flush=True)
    assert any(line.startswith("0 4 1 0 1 :") for line in text.splitlines())
    q = gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], 1)
    g = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], 1)
    torch.cuda.synchronize()
    args = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
    qr = oracle.forward(*args, 1, prob["eps"])
    gr = oracle.backward(*args, 1, prob["eps"], prob["dq"].double().numpy())
    assert np.abs(q.double().cpu().numpy() - qr).max() <= 1e-4
    for k, v in zip(("dI_lo", "dp_lo", "dI_hi"), g[:3]):
        assert np.abs(v.double().cpu().numpy() - gr[k]).max() / max(1.0, np.abs(gr[k]).max()) \
            <= 1e-4
    # leave the default shapes for later tests in this process
    assert gf.gf_tune_import("0 4 1 0 1 : 16 24 8 2\n") == gf.GF_OK
