"""Plain, unfused PyTorch composition of the guided filtering layer.

The layer as a graph of framework operators, the way the paper describes it
(Sec. III-C: a box filter, the local linear model's elementwise operators,
bilinear upsampling and a final linear layer), differentiated by autograd.
It is the "plain" baseline the fused HIP path is timed against; it computes
in float32 (half-precision inputs are up-converted inside the call).
"""
import torch
import torch.nn.functional as F


def _box(x, r):
    return F.avg_pool2d(x, 2 * r + 1, stride=1, padding=r, count_include_pad=False)


def guided_filter(I_lo, p_lo, I_hi, r, eps, mean_ab=True):
    I_lo, p_lo, I_hi = I_lo.float(), p_lo.float(), I_hi.float()
    if isinstance(eps, torch.Tensor) and eps.numel() > 1:
        eps = eps.view(-1, 1, 1, 1)
    mI = _box(I_lo, r)
    mP = _box(p_lo, r)
    var = _box(I_lo * I_lo, r) - mI * mI
    cov = _box(I_lo * p_lo, r) - mI * mP
    A = cov / (var + eps)
    b = mP - A * mI
    if mean_ab:
        A, b = _box(A, r), _box(b, r)
    size = I_hi.shape[-2:]
    A_h = F.interpolate(A, size=size, mode="bilinear", align_corners=False)
    b_h = F.interpolate(b, size=size, mode="bilinear", align_corners=False)
    return A_h * I_hi + b_h


def guide_transform(x, w1, w2, b2, lam, mu, gamma, beta, bn_eps=1e-5, slope=0.2):
    """The trainable guidance map as framework operators (float32): 1x1
    convolution, adaptive normalisation lam*h + mu*BN(h) with the batch
    statistics of x (train-mode batch norm), leaky ReLU, 1x1 convolution."""
    x = x.float()
    h = F.conv2d(x, w1[:, :, None, None])
    m = h.mean(dim=(0, 2, 3), keepdim=True)
    v = ((h - m) ** 2).mean(dim=(0, 2, 3), keepdim=True)
    bn = gamma.view(1, -1, 1, 1) * (h - m) / torch.sqrt(v + bn_eps) + beta.view(1, -1, 1, 1)
    y = lam * h + mu * bn
    return F.conv2d(F.leaky_relu(y, slope), w2[:, :, None, None], b2)


def _conv_fd(x, D, r):
    c = x.shape[1]
    Dw = D.reshape(c, 1, 3, 3)
    num = F.conv2d(x, Dw, padding=r, dilation=r, groups=c)
    den = F.conv2d(torch.ones_like(x[:1]), Dw, padding=r, dilation=r, groups=c)
    return num / den


def conv_guided_filter(I_lo, p_lo, I_hi, r, D, W1, W2, W3, slope=0.2, mean_ab=True):
    """The convolutional guided filtering layer (Sec. III-E) as framework
    operators in float32: normalised dilated depthwise convolutions for the
    window means, a pointwise block of 1x1 convolutions on (cov, var),
    bilinear upsampling."""
    I_lo, p_lo, I_hi = I_lo.float(), p_lo.float(), I_hi.float()
    mI, mP = _conv_fd(I_lo, D, r), _conv_fd(p_lo, D, r)
    cov = _conv_fd(I_lo * p_lo, D, r) - mI * mP
    var = _conv_fd(I_lo * I_lo, D, r) - mI * mI
    z = F.leaky_relu(F.conv2d(torch.cat([cov, var], 1), W1[:, :, None, None]), slope)
    z = F.leaky_relu(F.conv2d(z, W2[:, :, None, None]), slope)
    A = F.conv2d(z, W3[:, :, None, None])
    b = mP - A * mI
    if mean_ab:
        A, b = _conv_fd(A, D, r), _conv_fd(b, D, r)
    size = I_hi.shape[-2:]
    A_h = F.interpolate(A, size=size, mode="bilinear", align_corners=False)
    b_h = F.interpolate(b, size=size, mode="bilinear", align_corners=False)
    return A_h * I_hi + b_h
