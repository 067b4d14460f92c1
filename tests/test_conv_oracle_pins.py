"""Pins of the FP64 oracle of the convolutional guided filtering layer
(Sec. III-E; oracle/gf_conv_oracle.c) against things other than itself: the
box filter that uniform weights at dilation 1 reduce to, the closed form of
a constant guide, an independent float64 PyTorch composition of library
operators (forward and autograd), central finite differences, and the
magnitude sums of the parameter gradients' terms taken from autograd.
"""
import numpy as np
import pytest
import torch

import oracle
from tests import ref_torch as R


def conv_params(rng, c=3, K=16, uniform=False, slope=0.2):
    D = np.full((c, 3, 3), 1.0 / 9.0) if uniform else rng.uniform(0.2, 1.0, size=(c, 3, 3))
    return {"D": D, "W1": rng.normal(0, 0.5, size=(K, 2 * c)),
            "W2": rng.normal(0, 0.3, size=(K, K)), "W3": rng.normal(0, 0.3, size=(c, K)),
            "slope": slope}


def torch_params(P, grad=False):
    out = {k: torch.tensor(np.asarray(P[k], dtype=np.float64), requires_grad=grad)
           for k in oracle.CONV_GROUPS}
    out["slope"] = P["slope"]
    return out


def inputs(rng, n, c, h, w, H, W):
    return rng.random((n, c, h, w)), rng.random((n, c, h, w)), rng.random((n, c, H, W))


def test_constant_guide_uniform_weights_is_double_box_mean():
    """A constant guide makes cov = var = 0, so the bias-free block gives
    A = 0 and q = f_up(f_d(f_d(p))); with uniform weights at r = 1, f_d is
    the clipped box mean, so q = upsampled double box mean of p (avg_pool2d
    and interpolate)."""
    rng = np.random.default_rng(1)
    P = conv_params(rng, uniform=True)
    _, p, _ = inputs(rng, 2, 3, 7, 9, 28, 36)
    I = np.full((2, 3, 7, 9), 0.375)
    Ih = np.full((2, 3, 28, 36), 0.375)
    q = oracle.conv_forward(I, p, Ih, 1, P)
    tp = torch.from_numpy(p)
    ref = R.up(R.box(R.box(tp, 1), 1), 28, 36, False).numpy()
    np.testing.assert_allclose(q, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("mean_ab, ac", [(True, False), (False, False), (True, True)])
def test_forward_equals_torch_composition(r, mean_ab, ac):
    rng = np.random.default_rng(10 * r + mean_ab)
    P = conv_params(rng)
    I, p, Ih = inputs(rng, 2, 3, 8, 11, 21, 40)
    q = oracle.conv_forward(I, p, Ih, r, P, mean_ab=mean_ab, align_corners=ac)
    ref = R.conv_guided_filter(torch.from_numpy(I), torch.from_numpy(p), torch.from_numpy(Ih),
                               r, torch_params(P), mean_ab=mean_ab, align_corners=ac)
    np.testing.assert_allclose(q, ref.numpy(), rtol=0, atol=1e-12)


def _autograd(I, p, Ih, dq, r, P, mean_ab=True, ac=False):
    tI, tp, tIh = (torch.tensor(x, requires_grad=True) for x in (I, p, Ih))
    tP = torch_params(P, grad=True)
    keep = {}
    q = R.conv_guided_filter(tI, tp, tIh, r, tP, mean_ab=mean_ab, align_corners=ac, keep=keep)
    (q * torch.from_numpy(dq)).sum().backward()
    grads = {"dI_lo": tI.grad.numpy(), "dp_lo": tp.grad.numpy(), "dI_hi": tIh.grad.numpy(),
             "dparams": np.concatenate([tP[k].grad.numpy().ravel()
                                        for k in oracle.CONV_GROUPS])}
    return grads, keep, tP, (tI, tp)


@pytest.mark.parametrize("r, mean_ab, ac", [(1, True, False), (2, False, False),
                                            (3, True, True)])
def test_backward_equals_autograd(r, mean_ab, ac):
    rng = np.random.default_rng(20 + r)
    P = conv_params(rng)
    I, p, Ih = inputs(rng, 2, 3, 9, 8, 30, 19)
    dq = rng.normal(size=Ih.shape)
    got = oracle.conv_backward(I, p, Ih, r, P, dq, mean_ab=mean_ab, align_corners=ac)
    ref, _, _, _ = _autograd(I, p, Ih, dq, r, P, mean_ab, ac)
    for k in ("dI_lo", "dp_lo", "dI_hi", "dparams"):
        np.testing.assert_allclose(got[k], ref[k], rtol=0,
                                   atol=1e-11 * max(1.0, np.abs(ref[k]).max()), err_msg=k)


def test_backward_finite_differences():
    """Central differences of <q, dq> for a sample of inputs and of every
    parameter group."""
    rng = np.random.default_rng(30)
    P = conv_params(rng, K=5)
    I, p, Ih = inputs(rng, 1, 3, 5, 6, 11, 13)
    dq = rng.normal(size=Ih.shape)
    r = 1
    got = oracle.conv_backward(I, p, Ih, r, P, dq)

    def loss(I_, p_, Ih_, P_):
        return float((oracle.conv_forward(I_, p_, Ih_, r, P_) * dq).sum())

    eps = 1e-6
    for name, arr, key in (("I", I, "dI_lo"), ("p", p, "dp_lo"), ("Ih", Ih, "dI_hi")):
        for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(4)]:
            a, b = arr.copy(), arr.copy()
            a[idx] += eps
            b[idx] -= eps
            args = {"I": (I, p, Ih), "p": (I, p, Ih), "Ih": (I, p, Ih)}[name]
            la = loss(*[a if x is arr else x for x in args], P)
            lb = loss(*[b if x is arr else x for x in args], P)
            fd = (la - lb) / (2 * eps)
            assert abs(fd - got[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
    flat = got["dparams"]
    split = oracle.conv_split(flat, 3, 5)
    for g in oracle.CONV_GROUPS:
        arr = np.asarray(P[g], dtype=np.float64)
        for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(3)]:
            a, b = dict(P), dict(P)
            a[g], b[g] = arr.copy(), arr.copy()
            a[g][idx] += eps
            b[g][idx] -= eps
            fd = (loss(I, p, Ih, a) - loss(I, p, Ih, b)) / (2 * eps)
            assert abs(fd - split[g][idx]) <= 1e-6 * max(1.0, abs(fd)), (g, idx)


def test_parameter_gradient_magnitude_sums():
    """dparams_abs (the error scale of each parameter gradient) equals the
    sum over pixels of |term| built from autograd's intermediate gradients:
    W1: |dy1 u|, W2: |dy2 z1|, W3: |dA z2| (dA the gradient reaching the
    block's output), D: per tap |(g / N)(x at tap - f_d(x))| for the window
    means of A and b, and for the statistics the four f_d uses' terms summed
    at each pixel and tap (the oracle's two-pass statistics form one term)."""
    rng = np.random.default_rng(40)
    P = conv_params(rng, K=6)
    I, p, Ih = inputs(rng, 2, 3, 6, 7, 17, 25)
    dq = rng.normal(size=Ih.shape)
    r = 2
    got = oracle.conv_backward(I, p, Ih, r, P, dq)
    _, kp, tP, (tI, tp) = _autograd(I, p, Ih, dq, r, P)
    D = tP["D"].detach()
    with torch.no_grad():
        def outer_abs(a, b):
            return torch.einsum("nahw,nehw->ae", a.abs(), b.abs()).numpy()

        w1 = outer_abs(kp["y1"].grad, kp["u"])
        w2 = outer_abs(kp["y2"].grad, kp["z1"])
        w3 = outer_abs(kp["A"].grad, kp["z2"])
        Id, pd = tI.detach(), tp.detach()
        stats = sum(R.conv_fd_weight_terms(kp[k].grad, x, kp[k], D, r)
                    for k, x in (("mI", Id), ("mP", pd), ("fIp", Id * pd), ("fII", Id * Id)))
        dab = R.conv_fd_weight_terms(kp["Ab"].grad, kp["A"], kp["Ab"], D, r)
        dbb = R.conv_fd_weight_terms(kp["bb"].grad, kp["b"], kp["bb"], D, r)
        d_abs = sum(t.abs().sum(dim=(0, 3, 4)) for t in (stats, dab, dbb)).numpy()
    want = np.concatenate([d_abs.ravel(), w1.ravel(), w2.ravel(), w3.ravel()])
    np.testing.assert_allclose(got["dparams_abs"], want, rtol=1e-10, atol=0)
    # and the plain sums of those terms are the gradients
    np.testing.assert_allclose(oracle.conv_split(got["dparams"], 3, 6)["D"].reshape(3, 9),
                               sum(t.sum(dim=(0, 3, 4)) for t in (stats, dab, dbb)).numpy(),
                               rtol=0, atol=1e-11)
