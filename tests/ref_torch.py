"""Independent float64 PyTorch compositions used to pin the oracle.

Built from library primitives (avg_pool2d with count_include_pad=False for
the clipped box mean, F.interpolate for bilinear upsampling, conv2d and
batch_norm for the guidance transform) and the one-pass statistics form
that Algorithm 1's adjoint terms imply, so that an error in the oracle's
brute-force loops or in its hand-written adjoint shows up as a mismatch.
"""
import torch
import torch.nn.functional as F


def box(x, r):
    return F.avg_pool2d(x, 2 * r + 1, stride=1, padding=r, count_include_pad=False)


def up(x, H, W, align_corners):
    return F.interpolate(x, size=(H, W), mode="bilinear", align_corners=bool(align_corners))


def transform(x, g):
    """F(I): 1x1 conv -> lam*h + mu*BN_train(h) -> leaky ReLU -> 1x1 conv + bias."""
    w1 = torch.as_tensor(g["w1"], dtype=x.dtype)
    w2 = torch.as_tensor(g["w2"], dtype=x.dtype)
    b2 = torch.as_tensor(g["b2"], dtype=x.dtype)
    gamma = torch.as_tensor(g["gamma"], dtype=x.dtype)
    beta = torch.as_tensor(g["beta"], dtype=x.dtype)
    return transform_params(x, w1, w2, b2, g["lam"], g["mu"], gamma, beta,
                            g.get("bn_eps", 1e-5), g.get("slope", 0.2))


def transform_params(x, w1, w2, b2, lam, mu, gamma, beta, bn_eps=1e-5, slope=0.2):
    h = F.conv2d(x, w1[:, :, None, None])
    bn = F.batch_norm(h, None, None, gamma, beta, training=True, eps=bn_eps)
    y = lam * h + mu * bn
    z = F.leaky_relu(y, slope)
    return F.conv2d(z, w2[:, :, None, None], b2)


def transform_parts(x, w1, w2, b2, lam, mu, gamma, beta, bn_eps=1e-5, slope=0.2):
    """F(I) with its intermediates exposed (each retains its gradient):
    h = W1 x, hn = (h - m) / sqrt(v + bn_eps) (batch statistics), bn =
    gamma hn + beta, y = lam h + mu bn, z = leaky_relu(y), G = W2 z + b2."""
    h = F.conv2d(x, w1[:, :, None, None])
    m = h.mean(dim=(0, 2, 3), keepdim=True)
    v = ((h - m) ** 2).mean(dim=(0, 2, 3), keepdim=True)
    hn = (h - m) / torch.sqrt(v + bn_eps)
    bn = gamma.view(1, -1, 1, 1) * hn + beta.view(1, -1, 1, 1)
    y = lam * h + mu * bn
    z = F.leaky_relu(y, slope)
    G = F.conv2d(z, w2[:, :, None, None], b2)
    parts = dict(h=h, hn=hn, bn=bn, y=y, z=z, G=G)
    for t in (h, bn, y, G):
        if t.requires_grad:
            t.retain_grad()
    return parts


def guided_filter(G_lo, p_lo, G_hi, r, eps, mean_ab=True, align_corners=False, keep=None):
    """q from guides already transformed (G = F(I)); eps: scalar or [n].
    `keep` (a dict), if given, receives the window variance `var` (which
    retains its gradient)."""
    eps = torch.as_tensor(eps, dtype=G_lo.dtype)
    if eps.ndim == 1 and eps.numel() > 1:
        eps = eps.view(-1, 1, 1, 1)
    mI = box(G_lo, r)
    mP = box(p_lo, r)
    var = box(G_lo * G_lo, r) - mI * mI
    if keep is not None and var.requires_grad:
        var.retain_grad()
        keep["var"] = var
    cov = box(G_lo * p_lo, r) - mI * mP
    A = cov / (var + eps)
    b = mP - A * mI
    if mean_ab:
        A, b = box(A, r), box(b, r)
    H, W = G_hi.shape[-2:]
    return up(A, H, W, align_corners) * G_hi + up(b, H, W, align_corners)


# ---------------------------------------------------------------- convolutional layer

def conv_fd(x, D, r):
    """Dilated 3x3 depthwise convolution (weights D [c, 3, 3], dilation r,
    zero padding) normalised by the same convolution of the ones image."""
    c = x.shape[1]
    Dw = D.reshape(c, 1, 3, 3)
    num = F.conv2d(x, Dw, padding=r, dilation=r, groups=c)
    den = F.conv2d(torch.ones_like(x[:1]), Dw, padding=r, dilation=r, groups=c)
    return num / den


def conv_guided_filter(I_lo, p_lo, I_hi, r, P, mean_ab=True, align_corners=False, keep=None):
    """The convolutional layer as a composition of library ops; P holds
    tensors D, W1, W2, W3 and the slope.  `keep` receives the intermediates
    (each retaining its gradient when it has one)."""
    D, W1, W2, W3 = (P[k] for k in ("D", "W1", "W2", "W3"))
    s = P.get("slope", 0.2)
    mI, mP = conv_fd(I_lo, D, r), conv_fd(p_lo, D, r)
    fIp, fII = conv_fd(I_lo * p_lo, D, r), conv_fd(I_lo * I_lo, D, r)
    cov = fIp - mI * mP
    var = fII - mI * mI
    u = torch.cat([cov, var], dim=1)
    y1 = F.conv2d(u, W1[:, :, None, None])
    z1 = F.leaky_relu(y1, s)
    y2 = F.conv2d(z1, W2[:, :, None, None])
    z2 = F.leaky_relu(y2, s)
    A = F.conv2d(z2, W3[:, :, None, None])
    b = mP - A * mI
    Ab, bb = (conv_fd(A, D, r), conv_fd(b, D, r)) if mean_ab else (A, b)
    if keep is not None:
        parts = dict(mI=mI, mP=mP, fIp=fIp, fII=fII, u=u, y1=y1, z1=z1, y2=y2, z2=z2, A=A, b=b,
                     Ab=Ab, bb=bb)
        for t in parts.values():
            if t.requires_grad:
                t.retain_grad()
        keep.update(parts)
    H, W = I_hi.shape[-2:]
    return up(Ab, H, W, align_corners) * I_hi + up(bb, H, W, align_corners)


def conv_taps(x, r):
    """[n, c, 9, h, w]: x at the 9 dilated taps of every pixel (0 outside)."""
    n, c, h, w = x.shape
    cols = F.unfold(x.reshape(n * c, 1, h, w), 3, dilation=r, padding=r)
    return cols.reshape(n, c, 9, h, w)


def conv_fd_weight_terms(g, x, y, D, r):
    """Per (pixel, tap) terms of the gradient of sum(g * f_d(x)) with respect
    to D: g (x at the tap - y) / N, zero where the tap leaves the image
    (y = f_d(x)).  Shape [n, c, 9, h, w]."""
    c = x.shape[1]
    ones = torch.ones_like(x[:1])
    inside = conv_taps(ones, r)
    N = F.conv2d(ones, D.reshape(c, 1, 3, 3), padding=r, dilation=r, groups=c)
    return (g / N).unsqueeze(2) * (conv_taps(x, r) - y.unsqueeze(2)) * inside
