"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element.  Error measures and bars: see
tests/parity.py.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_05619_amd import datagen
from tests import parity

pytestmark = pytest.mark.gpu


def _gf():
    from paper_1803_05619_amd import gf
    return gf


def to_dev(prob):
    dev = torch.device("cuda:0")
    return {k: (prob[k].to(dev) if isinstance(prob.get(k), torch.Tensor) else prob.get(k))
            for k in ("I_lo", "p_lo", "I_hi", "dq")}


def run_both(prob, mean_ab=True, eps=None, backward=True, align_corners=False, precise=False):
    gf = _gf()
    d = to_dev(prob)
    eps = prob["eps"] if eps is None else eps
    print(f"case n={prob['n']} c={prob['c']} H={prob['H']} W={prob['W']} s={prob['s']} "
          f"r={prob['r']} dtype={prob['io_dtype']} mean_ab={mean_ab} ac={align_corners} "
          f"precise={precise}", flush=True)
    q = gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], eps, prob["r"], mean_ab,
                   align_corners=align_corners, precise=precise)
    out = {"q": q}
    if backward:
        dI_lo, dp_lo, dI_hi, deps, _ = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], eps, d["dq"],
                                                   prob["r"], mean_ab,
                                                   align_corners=align_corners, precise=precise)
        out.update(dI_lo=dI_lo, dp_lo=dp_lo, dI_hi=dI_hi, deps=deps)
    torch.cuda.synchronize()
    out = {k: v.double().cpu().numpy() for k, v in out.items()}
    args = [prob[k].double().numpy() for k in ("I_lo", "p_lo", "I_hi")]
    ref = {"q": oracle.forward(*args, prob["r"], eps, mean_ab=mean_ab,
                               align_corners=align_corners)}
    if backward:
        ref.update(oracle.backward(*args, prob["r"], eps, prob["dq"].double().numpy(),
                                   mean_ab=mean_ab, align_corners=align_corners))
    return out, ref


def measure(prob, out, ref):
    return parity.measure(out, ref, prob["io_dtype"],
                          n_eps_terms=prob["n"] * prob["c"] * prob["h"] * prob["w"])


def check(prob, **kw):
    out, ref = run_both(prob, **kw)
    return parity.check(measure(prob, out, ref))


# ------------------------------------------------------------ configurations

def test_config0_forward_exact_size():
    """64x64 -> 256x256, r=1, eps=1e-2, FP32, forward only."""
    check(datagen.make_config(0, with_dq=False), backward=False)


def test_config1_reduced():
    """The fwd+bwd FP32 workload at 1/8 size (256x384, s=4): several tiles,
    ragged column tile."""
    check(datagen.make_config(1, div=8))


@pytest.mark.parametrize("mean_ab", [False, True])
def test_config1_reduced_mean_ab(mean_ab):
    check(datagen.make_config(1, div=16, n=2), mean_ab=mean_ab)


def test_config2_bf16_reduced():
    """BF16 I/O with FP32 accumulation (identity guide)."""
    check(datagen.make_config(2, div=8, n=2))


@pytest.mark.parametrize("r", [1, 8])
def test_config4_fp16_reduced(r):
    """FP16 I/O, eps=1e-8, near-constant patches (variance cancellation)."""
    check(datagen.make_config(4, div=8, r=r))


# ------------------------------------------------------------ shapes and edge cases

@pytest.mark.parametrize("mean_ab", [True, False])
@pytest.mark.parametrize("io", ["f32", "f16"])
@pytest.mark.parametrize("r", [0, 1, 2, 4])
def test_precise_walkers(r, io, mean_ab):
    """The precise descriptor: FP64 wide walkers at radii 0..4, over several
    256-column strips with a ragged last one and row tiles with a ragged
    tail.  With the A/b window mean (the layer's form) the second image has
    eps = 1e-8 and near-constant patches.  Without it the upstream dA, db of
    each window are the high-res pass's FP32 partial sums themselves, which
    dcov = dA_t / (var + eps) amplifies at eps = 1e-8 beyond the bars of
    either walker (the window mean averages that rounding away), so that
    form runs at eps = 1e-4 here."""
    eps = [1e-3, 1e-8] if mean_ab else [1e-3, 1e-4]
    prob = datagen.make_problem(2, 3, 4 * 37, 4 * 300, 4, r, eps, io, config=91, flat_rects=2)
    check(prob, mean_ab=mean_ab, precise=True)


@pytest.mark.parametrize("io", ["f32", "f16"])
def test_radius0_tiny_eps(io):
    """Radius 0 (one-pixel windows: A = 0, dI_l = 0, dp_l = dbbar exactly)
    at eps = 1e-8 through the default column walkers."""
    prob = datagen.make_problem(2, 3, 4 * 37, 4 * 300, 4, 0, [1e-3, 1e-8], io, config=92,
                                flat_rects=2)
    check(prob)


@pytest.mark.parametrize("s", [1, 2, 4, 8])
@pytest.mark.parametrize("r", [0, 1, 3])
def test_factors_and_radii(s, r):
    prob = datagen.make_problem(2, 3, 8 * 13, 8 * 21, s, r, [1e-3, 3e-2], "f32", config=90)
    check(prob)


@pytest.mark.parametrize("r, mean_ab, dt", [(5, True, "f32"), (6, False, "f32"), (10, True, "f32"),
                                          (8, True, "f16"), (7, False, "bf16")])
def test_wide_backward_radii(r, mean_ab, dt):
    """The wide low-res backward (large radii): low-res 77 x 530 spans three
    256-column strips with a ragged last one and three 32-row tiles with a
    ragged last one; two images."""
    prob = datagen.make_problem(2, 3, 4 * 77, 4 * 530, 4, r, [1e-4, 1e-2], dt, config=91)
    check(prob, mean_ab=mean_ab)


def test_scalar_path_odd_width():
    """W not a multiple of 4: the element-wise (VEC = 1) kernels."""
    prob = datagen.make_problem(1, 2, 2 * 37, 2 * 49, 2, 2, 1e-3, "f32", config=91)
    check(prob)


def test_tiny_images_and_huge_radius():
    for (H, W, s, r) in ((4, 4, 4, 1), (8, 40, 8, 2), (16, 16, 4, 7), (2, 6, 2, 5)):
        prob = datagen.make_problem(1, 3, H, W, s, r, 1e-2, "f32", config=92)
        check(prob)


def test_many_images_per_image_eps():
    prob = datagen.make_problem(5, 3, 96, 128, 4, 2, [1e-4, 1e-3, 1e-2, 1e-1, 1.0], "f32",
                                config=93)
    check(prob)


def test_optional_outputs_are_optional():
    gf = _gf()
    prob = datagen.make_config(1, div=16, n=1)
    d = to_dev(prob)
    full = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], 1)
    part = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], 1,
                       need_dI_lo=False, need_dI_hi=False, need_deps=False)
    torch.cuda.synchronize()
    assert part[0] is None and part[2] is None and part[3] is None
    assert torch.equal(full[1], part[1])


def test_bitwise_deterministic():
    gf = _gf()
    prob = datagen.make_config(1, div=8, n=2)
    d = to_dev(prob)
    runs = []
    for _ in range(2):
        q = gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], 1)
        g = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], 1)
        runs.append([q, *g])
    torch.cuda.synchronize()
    for a, b in zip(*runs):
        assert (a is None and b is None) or torch.equal(a, b)


def test_outputs_stay_in_bounds():
    """Canary bands around every output must be untouched."""
    gf = _gf()
    prob = datagen.make_problem(1, 3, 4 * 19, 4 * 23, 4, 1, 1e-2, "f32", config=94)
    d = to_dev(prob)
    pad = 1024

    def canary(shape, dtype):
        numel = int(np.prod(shape))
        buf = torch.full((numel + 2 * pad,), 12345.0, dtype=dtype, device="cuda:0")
        return buf, buf[pad:pad + numel].view(shape)

    qb, q = canary(d["I_hi"].shape, torch.float32)
    gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], 1, out=q)
    b1, dI_lo = canary(d["I_lo"].shape, torch.float32)
    b2, dp_lo = canary(d["p_lo"].shape, torch.float32)
    b3, dI_hi = canary(d["I_hi"].shape, torch.float32)
    b4, deps = canary((1,), torch.float32)
    gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], 1,
                outs=(dI_lo, dp_lo, dI_hi, deps))
    torch.cuda.synchronize()
    for buf in (qb, b1, b2, b3, b4):
        assert torch.all(buf[:pad] == 12345.0) and torch.all(buf[-pad:] == 12345.0)


def test_autograd_function():
    gf = _gf()
    prob = datagen.make_config(1, div=16, n=1)
    d = to_dev(prob)
    I_lo = d["I_lo"].clone().requires_grad_(True)
    p_lo = d["p_lo"].clone().requires_grad_(True)
    I_hi = d["I_hi"].clone().requires_grad_(True)
    eps = torch.tensor(prob["eps"], dtype=torch.float32, device="cuda:0", requires_grad=True)
    q = gf.guided_filter(I_lo, p_lo, I_hi, r=1, eps=eps)
    (q * d["dq"]).sum().backward()
    ref = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], eps.detach(), d["dq"], 1)
    torch.cuda.synchronize()
    for got, want in zip((I_lo.grad, p_lo.grad, I_hi.grad, eps.grad), ref):
        assert torch.equal(got, want)


# ------------------------------------------------------------ full size

def test_config1_full_size():
    """4 x 3 x 2048 x 3072 FP32, r=1, eps=1e-4: the benchmarked launch shapes,
    every output compared with the full oracle."""
    check(datagen.make_config(1))


@pytest.mark.parametrize("cfg, dt", [(1, "f32"), (2, "bf16"), (4, "f16")])
def test_forward_backward_equals_separate_calls(cfg, dt):
    """One gf_forward_backward call gives bit for bit what gf_forward then
    gf_backward give (the backward recomputes the same coefficients)."""
    gf = _gf()
    prob = datagen.make_config(cfg, div=16, n=2)
    d = to_dev(prob)
    print(f"case config={cfg} dtype={dt}", flush=True)
    q = gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], prob["r"])
    g = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], prob["r"])
    fb = gf.forward_backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], prob["r"])
    torch.cuda.synchronize()
    assert torch.equal(fb[0], q)
    for a, b in zip(fb[1:5], g[:4]):
        assert torch.equal(a, b)


def test_forward_backward_five_images():
    """Five images with per-image eps, twice in a row: the fused call gives
    bit for bit the separate calls' results, and the oracle's."""
    gf = _gf()
    prob = datagen.make_problem(5, 3, 4 * 40, 4 * 56, 4, 1, [1e-4, 1e-3, 1e-2, 1e-5, 1e-6], "f32",
                                config=170, noise=0.02)
    print("case 5 images, per-image eps, fused call", flush=True)
    d = to_dev(prob)
    q = gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], prob["r"])
    g = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], prob["r"])
    for _ in range(2):
        fb = gf.forward_backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"],
                                 prob["r"])
        torch.cuda.synchronize()
        assert torch.equal(fb[0], q)
        for a, b in zip(fb[1:5], g[:4]):
            assert torch.equal(a, b)
    check(prob)


# ------------------------------------------------------------ corner alignment

@pytest.mark.parametrize("s, r, mean_ab", [(1, 1, True), (2, 2, True), (4, 1, True), (4, 3, False),
                                           (8, 1, True), (8, 2, False)])
def test_align_corners(s, r, mean_ab):
    """Corner-aligned bilinear (align_corners = 1): per-column and per-row
    taps at run time, the backward's row sums flushed through LDS."""
    prob = datagen.make_problem(2, 3, 16 * s + 8 * s, 24 * s + 8 * s, s, r, 1e-3, "f32",
                                config=160 + s, noise=0.02)
    check(prob, mean_ab=mean_ab, align_corners=True)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_align_corners_half_io(dt):
    prob = datagen.make_problem(2, 3, 4 * 40, 4 * 52, 4, 2, 1e-4, dt, config=170, noise=0.02)
    check(prob, align_corners=True)


def test_align_corners_scalar_width():
    """A width that is not a multiple of 4 (one column per lane)."""
    prob = datagen.make_problem(1, 3, 2 * 30, 2 * 37, 2, 1, 1e-3, "f32", config=171, noise=0.02)
    check(prob, align_corners=True)


# ------------------------------------------------------------ degenerate cases

def _const_guide(prob, value=0.375):
    """The same problem with a constant guide (exactly representable)."""
    out = dict(prob)
    out["I_lo"] = torch.full_like(prob["I_lo"], value)
    out["I_hi"] = torch.full_like(prob["I_hi"], value)
    return out


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_constant_guide(eps):
    """var = 0 in every window: with eps = 0 the rule A := 0 applies (q is
    the upsampled window mean of p); with eps > 0 A = 0 / eps = 0."""
    prob = _const_guide(datagen.make_problem(2, 3, 4 * 20, 4 * 28, 4, 1, eps, "f32", config=180))
    check(prob)


def test_zero_eps_textured_guide():
    """eps = 0 with a textured guide (noise keeps every window's variance
    positive)."""
    prob = datagen.make_problem(1, 3, 4 * 24, 4 * 24, 4, 1, 0.0, "f32", config=181, noise=0.05)
    check(prob)


@pytest.mark.parametrize("h, w, s", [(1, 1, 4), (1, 17, 2), (13, 1, 8), (2, 3, 1)])
def test_degenerate_shapes(h, w, s):
    """One-pixel, one-row and one-column low-res images."""
    prob = datagen.make_problem(2, 3, s * h, s * w, s, 1, 1e-2, "f32", config=182, noise=0.02)
    check(prob)


# ------------------------------------------------------------ any size ratio

# (h, w, H, W): non-integer ratios, ratios that differ per axis, integer
# factors outside {1, 2, 4, 8}, one-pixel low-res axes
ANY_RATIO = [
    (5, 7, 13, 10),
    (64, 96, 250, 300),
    (32, 48, 64, 192),      # factor 2 vertically, 4 horizontally
    (48, 64, 144, 192),     # factor 3
    (30, 40, 480, 640),     # factor 16
    (20, 30, 960, 1440),    # factor 48 (a 64-pixel I_l under a large I_h)
    (1, 9, 7, 37),
    (9, 1, 40, 3),
]


@pytest.mark.parametrize("h, w, H, W", ANY_RATIO)
@pytest.mark.parametrize("ac", [False, True])
def test_any_ratio(h, w, H, W, ac):
    """Sizes the problem statement allows (any h <= H, w <= W): the general
    high-res kernels, forward and backward, against the oracle."""
    prob = datagen.make_problem_sizes(2, 3, H, W, h, w, 1 + (h * w) % 2, [1e-3, 1e-2], "f32",
                                      config=190, noise=0.02)
    check(prob, align_corners=ac)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_any_ratio_half_io(dt):
    prob = datagen.make_problem_sizes(2, 3, 250, 300, 64, 96, 2, 1e-4, dt, config=191,
                                      noise=0.02)
    check(prob)


def test_any_ratio_without_ab_mean_and_scalar_width():
    """Algorithm 1's form (no window mean of A, b) and a width that is not a
    multiple of 4."""
    prob = datagen.make_problem_sizes(1, 3, 101, 203, 40, 70, 1, 1e-3, "f32", config=192,
                                      noise=0.02)
    check(prob, mean_ab=False)


def test_any_ratio_forward_backward_equals_separate_calls():
    gf = _gf()
    prob = datagen.make_problem_sizes(2, 3, 250, 300, 64, 96, 1, [1e-4, 1e-2], "f32",
                                      config=193, noise=0.02)
    d = to_dev(prob)
    print("case any-ratio fused call 64x96 -> 250x300", flush=True)
    q = gf.forward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], prob["r"])
    g = gf.backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], prob["r"])
    fb = gf.forward_backward(d["I_lo"], d["p_lo"], d["I_hi"], prob["eps"], d["dq"], prob["r"])
    torch.cuda.synchronize()
    assert torch.equal(fb[0], q)
    for a, b in zip(fb[1:5], g[:4]):
        assert torch.equal(a, b)
