"""The deep guided filtering network's inference chain (Sec. IV, Fig. 3) as
a timing analog of the paper's running-time measurements (Sec. V-D):

    I_l = downsample(I_h)          gf_downsample (this library's kernel)
    O_l = C_l(I_l)                 the low-res network: a context aggregation
                                   network with random weights (Table I),
                                   PyTorch convolutions
    O_h = GF(I_l, O_l, I_h)        gf_forward (this library's layer)

The low-res network is not this library's hot path and runs as plain
PyTorch convolutions (MIOpen); its weights are random (no trained weights
exist here), so the chain measures speed and memory, not quality.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

from . import gf

# Table I, the low-res network C_l: seven 3x3 convolutions of 24 channels
# with dilations 1, 1, 2, 4, 8, 16, 1, no bias, each followed by adaptive
# normalisation and leaky ReLU (slope 0.2), then a 1x1 convolution to 3
# channels with bias.
CAN_DILATIONS = (1, 1, 2, 4, 8, 16, 1)
CAN_WIDTH = 24
SLOPE = 0.2


class CAN(torch.nn.Module):
    """C_l of Table I at inference.  Adaptive normalisation lam x +
    mu BN(x) uses the batch-norm running statistics at inference, so it is
    a per-channel affine map, folded into one scale and shift per layer;
    here at its initial mix lam = 1, mu = 0 (the identity) with random BN
    parameters.  Convolution weights ~ N(0, 2 / fan_in), so activations stay
    of order one through the seven layers."""

    def __init__(self, c_in: int = 3, c_out: int = 3, seed: int = 0):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        ws, scales, shifts = [], [], []
        cin = c_in
        for _ in CAN_DILATIONS:
            ws.append(torch.randn(CAN_WIDTH, cin, 3, 3, generator=g) * (2.0 / (9 * cin)) ** 0.5)
            lam, mu = 1.0, 0.0
            gamma = 1.0 + 0.1 * torch.randn(CAN_WIDTH, generator=g)
            beta = 0.1 * torch.randn(CAN_WIDTH, generator=g)
            # running mean 0, running variance 1, batch-norm eps 1e-5
            bn_scale = gamma / (1.0 + 1e-5) ** 0.5
            scales.append(lam + mu * bn_scale)
            shifts.append(mu * beta)
            cin = CAN_WIDTH
        self.weights = torch.nn.ParameterList([torch.nn.Parameter(w) for w in ws])
        self.register_buffer("scales", torch.stack(scales))
        self.register_buffer("shifts", torch.stack(shifts))
        self.head_w = torch.nn.Parameter(
            torch.randn(c_out, CAN_WIDTH, 1, 1, generator=g) * (1.0 / CAN_WIDTH) ** 0.5)
        self.head_b = torch.nn.Parameter(0.1 * torch.randn(c_out, generator=g))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        for k, d in enumerate(CAN_DILATIONS):
            x = F.conv2d(x, self.weights[k], padding=d, dilation=d)
            x = x * self.scales[k].view(1, -1, 1, 1) + self.shifts[k].view(1, -1, 1, 1)
            x = F.leaky_relu(x, SLOPE)
        return F.conv2d(x, self.head_w, self.head_b)


def low_res_size(H: int, W: int, lo: int) -> tuple:
    """I_l's size: the short side `lo` pixels, the aspect ratio kept (the
    paper's 64s setting, Sec. V-B)."""
    if H <= W:
        return lo, max(1, round(W * lo / H))
    return max(1, round(H * lo / W)), lo


def dgf_forward(I_hi: torch.Tensor, net: torch.nn.Module, lo: int = 64, r: int = 1,
                eps=1e-8, ws: torch.Tensor | None = None, return_all: bool = False):
    """O_h of the DGF framework for the high-res input I_hi [n, 3, H, W]:
    downsampling and the guided filtering layer run in this library's
    kernels, C_l in PyTorch.  eps: a float, or a float32 device tensor (no
    host-to-device copy inside the call: what stream capture needs)."""
    H, W = I_hi.shape[-2:]
    h, w = low_res_size(H, W, lo)
    with torch.no_grad():  # inference: no autograd graph through C_l
        I_lo = gf.downsample(I_hi, h, w)
        p_lo = net(I_lo).contiguous()
        q = gf.forward(I_lo, p_lo, I_hi, eps, r, ws=ws)
    if return_all:
        return q, I_lo, p_lo
    return q
