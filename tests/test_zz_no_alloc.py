"""gf_forward_backward_static (the library's static scratch instead of a
caller workspace) against gf_forward_backward with a torch-allocated
workspace, through the C ABI: two calls in a row, the second with a smaller
problem (the scratch then holds the first call's contents), each output
compared bit for bit (same kernels, same workspace layout).  Also: a
problem whose workspace exceeds the static scratch is rejected on the host.
"""
import pytest
import torch

from paper_1803_05619_amd import datagen

pytestmark = pytest.mark.gpu


def _gf():
    from paper_1803_05619_amd import gf
    return gf


def _outputs(gf, prob, dev):
    t = {k: prob[k].to(dev) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    f32 = dict(dtype=torch.float32, device=dev)
    outs = {"q": torch.full_like(t["I_hi"], float("nan")),
            "dI_lo": torch.full(t["I_lo"].shape, float("nan"), **f32),
            "dp_lo": torch.full(t["p_lo"].shape, float("nan"), **f32),
            "dI_hi": torch.full_like(t["I_hi"], float("nan")),
            "deps": torch.full((len(prob["eps"]),), float("nan"), **f32)}
    return t, outs


def _run(gf, prob, static):
    dev = torch.device("cuda:0")
    t, o = _outputs(gf, prob, dev)
    eps = torch.tensor(prob["eps"], dtype=torch.float32, device=dev)
    desc = gf.make_desc(t["I_lo"], t["I_hi"], prob["r"])
    stream = torch.cuda.current_stream(dev).cuda_stream
    args = (desc, None, t["I_lo"].data_ptr(), t["p_lo"].data_ptr(), t["I_hi"].data_ptr(),
            eps.data_ptr(), eps.numel(), t["dq"].data_ptr(), o["q"].data_ptr(),
            o["dI_lo"].data_ptr(), o["dp_lo"].data_ptr(), o["dI_hi"].data_ptr(),
            o["deps"].data_ptr(), None)
    if static:
        st = gf.gf_forward_backward_static(*args, stream)
    else:
        need = gf.gf_workspace_size(desc, None, 2)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        st = gf.gf_forward_backward(*args, ws.data_ptr(), ws.numel(), stream)
    assert st == gf.GF_OK, gf.gf_last_error_detail()
    torch.cuda.synchronize()
    return {k: v.cpu() for k, v in o.items()}


def test_static_scratch_equals_workspace_call():
    gf = _gf()
    cases = [
        # a larger problem first (several tiles, ragged column strip), then a
        # smaller one with another radius and eps per image
        datagen.make_problem(2, 3, 384, 648, 4, 1, [1e-4, 1e-2], "f32", config=1, noise=0.02),
        datagen.make_problem(1, 3, 136, 200, 2, 2, [1e-3], "f32", config=1, noise=0.02),
    ]
    for prob in cases:
        print(f"case n={prob['n']} H={prob['H']} W={prob['W']} s={prob['s']} r={prob['r']}",
              flush=True)
        got = _run(gf, prob, static=True)
        ref = _run(gf, prob, static=False)
        for k in ref:
            assert torch.isfinite(got[k]).all(), k
            assert torch.equal(got[k], ref[k]), (k, float((got[k] - ref[k]).abs().max()))


def test_static_scratch_rejects_oversized_problem():
    gf = _gf()
    dev = torch.device("cuda:0")
    # the FP32 4x3x2048x3072 workload fits; 8 images of it do not
    small = gf.gf_desc_t(4, 3, 512, 768, 2048, 3072, 1, 1, gf.GF_F32, 0)
    big = gf.gf_desc_t(8, 3, 512, 768, 2048, 3072, 1, 1, gf.GF_F32, 0)
    assert gf.gf_workspace_size(small, None, 2) <= 96 << 20 < gf.gf_workspace_size(big, None, 2)
    x = torch.zeros(16, device=dev)
    p = x.data_ptr()
    st = gf.gf_forward_backward_static(big, None, p, p, p, p, 1, p, p, p, p, p, p, None,
                                       torch.cuda.current_stream(dev).cuda_stream)
    assert st == gf.GF_ERR_WORKSPACE
    assert "static scratch" in gf.gf_last_error_detail()
