"""GPU parity of the convolutional guided filtering layer (Sec. III-E)
against its FP64 oracle, through the C ABI: forward and every gradient
(inputs and the parameters D, W1, W2, W3), for several dilations, both
window-mean forms and alignments, integer and other size ratios, half I/O,
and at the full size of the FP32 4 x 3 x 2048 x 3072 workload."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_05619_amd import datagen
from tests import parity

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
K = 16


def _gf():
    from paper_1803_05619_amd import gf
    return gf


def conv_params(seed, c=3, K=K):
    """Random parameters at the scale of photo statistics (cov, var ~ 1e-3 ..
    1e-2): positive taps, W1 large enough that the hidden units leave zero."""
    rng = np.random.default_rng(seed)
    return {"D": rng.uniform(0.2, 1.0, size=(c, 3, 3)),
            "W1": rng.normal(0, 40.0, size=(K, 2 * c)),
            "W2": rng.normal(0, 0.4, size=(K, K)),
            "W3": rng.normal(0, 0.4, size=(c, K)), "slope": 0.2}


def run(prob, P, r, mean_ab=True, ac=False, backward=True):
    gf = _gf()
    d = {k: prob[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    params = gf.pack_conv_params(P["D"], P["W1"], P["W2"], P["W3"], device=DEV)
    print(f"case conv n={prob['n']} H={prob['H']} W={prob['W']} h={prob['h']} w={prob['w']} "
          f"r={r} mean_ab={mean_ab} ac={ac} dtype={prob['io_dtype']}", flush=True)
    q = gf.conv_forward(d["I_lo"], d["p_lo"], d["I_hi"], params, r, K, P["slope"], mean_ab,
                        align_corners=ac)
    out = {"q": q}
    if backward:
        dI_lo, dp_lo, dI_hi, dparams = gf.conv_backward(
            d["I_lo"], d["p_lo"], d["I_hi"], params, d["dq"], r, K, P["slope"], mean_ab,
            align_corners=ac)
        out.update(dI_lo=dI_lo, dp_lo=dp_lo, dI_hi=dI_hi, dparams=dparams)
    torch.cuda.synchronize()
    out = {k: v.double().cpu().numpy() for k, v in out.items()}
    args = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
    ref = {"q": oracle.conv_forward(*args, r, P, mean_ab=mean_ab, align_corners=ac)}
    if backward:
        ref.update(oracle.conv_backward(*args, r, P, prob["dq"].double().numpy(),
                                        mean_ab=mean_ab, align_corners=ac))
    return out, ref


def check(prob, P, r, **kw):
    out, ref = run(prob, P, r, **kw)
    return parity.check(parity.measure_conv(out, ref, prob["io_dtype"], prob["n"], prob["c"],
                                            prob["h"], prob["w"], K))


@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("mean_ab", [True, False])
def test_conv_dilations(r, mean_ab):
    prob = datagen.make_problem(2, 3, 4 * 40, 4 * 52, 4, r, 0.0, "f32", config=210, noise=0.02)
    check(prob, conv_params(211 + r), r, mean_ab=mean_ab)


@pytest.mark.parametrize("r", [8, 9])
def test_conv_tiled_gathers_edge(r):
    """Low-res 70 x 150: the LDS-tiled gathers' 16 x 64 tiles, three across
    and five down with ragged last ones, at their largest dilation (8) and
    the per-pixel kernels' first (9)."""
    prob = datagen.make_problem(1, 3, 2 * 70, 2 * 150, 2, r, 0.0, "f32", config=220, noise=0.02)
    check(prob, conv_params(221), r)


def test_conv_align_corners_and_any_ratio():
    prob = datagen.make_problem(2, 3, 2 * 48, 2 * 56, 2, 1, 0.0, "f32", config=212, noise=0.02)
    check(prob, conv_params(213), 1, ac=True)
    prob = datagen.make_problem_sizes(2, 3, 250, 300, 64, 96, 2, 0.0, "f32", config=214,
                                      noise=0.02)
    check(prob, conv_params(215), 2)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_conv_half_io(dt):
    prob = datagen.make_problem(2, 3, 4 * 48, 4 * 64, 4, 1, 0.0, dt, config=216, noise=0.02)
    check(prob, conv_params(217), 1)


def test_conv_small_images_large_dilation():
    """Taps beyond the image on most pixels (dilation above the image side)."""
    for (H, W, s, r) in ((8, 12, 2, 5), (16, 40, 8, 3)):
        prob = datagen.make_problem(1, 3, H, W, s, r, 0.0, "f32", config=218, noise=0.02)
        check(prob, conv_params(219), r)


def test_conv_one_pixel_low_res():
    """A 1x1 low-res image: every window is the pixel itself, so cov = var =
    0, A = 0, q is p upsampled (constant) and every parameter gradient is
    exactly zero; the GPU's may only differ from zero by rounding (the
    normalised single-tap mean D x / D need not equal x exactly)."""
    prob = datagen.make_problem(1, 3, 4, 4, 4, 1, 0.0, "f32", config=218, noise=0.02)
    out, ref = run(prob, conv_params(219), 1)
    parity.check(parity.measure({k: v for k, v in out.items() if k != "dparams"}, ref, "f32"))
    assert float(np.abs(ref["dparams"]).max()) <= 1e-12
    assert float(np.abs(out["dparams"]).max()) <= 1e-10


def test_conv_channels():
    for c in (1, 2, 4):
        prob = datagen.make_problem(2, c, 4 * 24, 4 * 36, 4, 1, 0.0, "f32", config=220 + c,
                                    noise=0.02)
        gf = _gf()
        P = conv_params(221 + c, c=c)
        d = {k: prob[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
        params = gf.pack_conv_params(P["D"], P["W1"], P["W2"], P["W3"], device=DEV)
        q = gf.conv_forward(d["I_lo"], d["p_lo"], d["I_hi"], params, 1, K)
        g = gf.conv_backward(d["I_lo"], d["p_lo"], d["I_hi"], params, d["dq"], 1, K)
        torch.cuda.synchronize()
        args = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
        ref = {"q": oracle.conv_forward(*args, 1, P)}
        ref.update(oracle.conv_backward(*args, 1, P, prob["dq"].double().numpy()))
        got = {"q": q.double().cpu().numpy(), "dI_lo": g[0].double().cpu().numpy(),
               "dp_lo": g[1].double().cpu().numpy(), "dI_hi": g[2].double().cpu().numpy()}
        parity.check(parity.measure(got, ref, "f32"), f"c={c}")
        d_err = np.abs(g[3].double().cpu().numpy() - ref["dparams"])
        assert float((d_err / (parity.conv_sum_bar(2 * 24 * 36, 24, 36, 2 * c) *
                               np.maximum(ref["dparams_abs"], 1e-300))).max()) <= 1.0


def test_conv_deterministic_and_autograd():
    gf = _gf()
    prob = datagen.make_problem(2, 3, 4 * 32, 4 * 40, 4, 2, 0.0, "f32", config=223, noise=0.02)
    P = conv_params(224)
    d = {k: prob[k].to(DEV) for k in ("I_lo", "p_lo", "I_hi", "dq")}
    params = gf.pack_conv_params(P["D"], P["W1"], P["W2"], P["W3"], device=DEV)
    runs = [gf.conv_backward(d["I_lo"], d["p_lo"], d["I_hi"], params, d["dq"], 2, K)
            for _ in range(2)]
    leaves = [d[k].clone().requires_grad_(True) for k in ("I_lo", "p_lo", "I_hi")]
    pl = params.clone().requires_grad_(True)
    q = gf.conv_guided_filter(*leaves, pl, r=2, hidden=K)
    q.backward(d["dq"])
    torch.cuda.synchronize()
    for a, b in zip(*runs):
        assert torch.equal(a, b)
    for got, want in zip((leaves[0].grad, leaves[1].grad, leaves[2].grad, pl.grad), runs[0]):
        assert torch.equal(got, want)


def test_conv_full_size():
    """The FP32 4 x 3 x 2048 x 3072 workload (512 x 768 low-res, r = 1):
    the benchmarked launch shapes, every output against the oracle."""
    prob = datagen.make_config(1)
    check(prob, conv_params(225), 1)
