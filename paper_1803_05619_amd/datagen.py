"""Seeded synthetic inputs for the guided filtering layer.

This module only draws data: it holds none of the filter's arithmetic and
is the one piece shared by the CPU oracle's tests and the GPU path.

The paper times and evaluates on high-resolution photographs (MIT-Adobe
FiveK, 512^2..3072^2; Sec. V-C and the timing paragraph of Sec. V-D) which
are not available here.  Synthetic "photo-like" images stand in for them:

* a smooth random field: white noise on a coarse grid (about 1/32 of the
  image side), bicubically upsampled, normalised to zero mean / unit std;
  each channel is 0.7 x a shared field + 0.3 x its own; the image is
  0.5 + 0.15 x field;
* K = 8 random step edges: half-planes through a uniform point at a uniform
  angle, each adding a per-channel step drawn from U(-0.25, 0.25);
* clipped to [0, 1]; optional N(0, sigma) noise, clipped again;
* optional near-constant rectangles (value 0.5 + N(0, 1e-4)) to stress the
  variance cancellation regime;
* the low-resolution guide is the s x s area mean of the quantised
  high-resolution guide (the paper downsamples I_h to obtain I_l, Sec. IV);
* the low-resolution input is p = clip(0.8 I_l + 0.1 n, 0, 1), n ~ N(0, 0.05);
* the upstream gradient is N(0, 1).

Every array is quantised once to the I/O dtype (round to nearest even).
Seeds: numpy default_rng(1803_05619 + 1000 * config + image).
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

SEED_BASE = 1803_05619

TORCH_DTYPES = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def rng_for(config: int, image: int = 0, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 1000 * config + image + 7919 * salt)


def quantize(x, io_dtype: str) -> torch.Tensor:
    """Round a float64 array/tensor to the I/O dtype (RNE), as a CPU tensor."""
    t = torch.as_tensor(np.asarray(x, dtype=np.float64))
    return t.to(TORCH_DTYPES[io_dtype]).contiguous()


def smooth_field(rng: np.random.Generator, C: int, H: int, W: int) -> np.ndarray:
    gh = max(4, int(math.ceil(H / 32)) + 1)
    gw = max(4, int(math.ceil(W / 32)) + 1)
    base = torch.from_numpy(rng.standard_normal((1, C + 1, gh, gw)))
    up = F.interpolate(base, size=(H, W), mode="bicubic", align_corners=False)[0].numpy()
    up = (up - up.mean(axis=(1, 2), keepdims=True)) / (up.std(axis=(1, 2), keepdims=True) + 1e-12)
    shared = up[C]
    return 0.7 * shared[None] + 0.3 * up[:C]


def photo(rng: np.random.Generator, C: int, H: int, W: int, noise: float = 0.0,
          edges: int = 8, flat_rects: int = 0) -> np.ndarray:
    """One photo-like image [C, H, W] in [0, 1], float64."""
    img = 0.5 + 0.15 * smooth_field(rng, C, H, W)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    for _ in range(edges):
        py, px = rng.uniform(0, H), rng.uniform(0, W)
        ang = rng.uniform(0, math.pi)
        side = (np.cos(ang) * (xx - px) + np.sin(ang) * (yy - py)) > 0
        step = rng.uniform(-0.25, 0.25, size=C)
        img += side[None] * step[:, None, None]
    img = np.clip(img, 0.0, 1.0)
    if noise > 0:
        img = np.clip(img + rng.normal(0.0, noise, size=img.shape), 0.0, 1.0)
    for _ in range(flat_rects):
        rh = max(1, int(rng.uniform(0.10, 0.25) * H))
        rw = max(1, int(rng.uniform(0.10, 0.25) * W))
        y0 = int(rng.integers(0, H - rh + 1))
        x0 = int(rng.integers(0, W - rw + 1))
        img[:, y0:y0 + rh, x0:x0 + rw] = 0.5 + rng.normal(0.0, 1e-4, size=(C, rh, rw))
    return img


def area_down(x: np.ndarray, sy: int, sx: int) -> np.ndarray:
    """s x s area mean over the last two axes (H, W multiples of s)."""
    *lead, H, W = x.shape
    return x.reshape(*lead, H // sy, sy, W // sx, sx).mean(axis=(-3, -1))


def area_resize(x: np.ndarray, h: int, w: int) -> np.ndarray:
    """Area mean to (h, w) for any size ratio over the last two axes: output
    pixel i covers input rows [floor(i H / h), ceil((i + 1) H / h)), likewise
    columns (the s x s mean when H = s h).  Input generation only."""
    *lead, H, W = x.shape
    rows = [(i * H // h, -(-(i + 1) * H // h)) for i in range(h)]
    cols = [(j * W // w, -(-(j + 1) * W // w)) for j in range(w)]
    tmp = np.stack([x[..., a:b, :].mean(axis=-2) for a, b in rows], axis=-2)
    return np.stack([tmp[..., a:b].mean(axis=-1) for a, b in cols], axis=-1)


def make_problem_sizes(n: int, c: int, H: int, W: int, h: int, w: int, r: int, eps,
                       io_dtype: str, config: int, noise: float = 0.0,
                       with_dq: bool = True) -> dict:
    """Like make_problem, for any low-res size h <= H, w <= W (the size
    ratio need not be an integer, nor the same on both axes): I_l is the
    area mean of the quantised I_h."""
    I_hi = torch.empty((n, c, H, W), dtype=TORCH_DTYPES[io_dtype])
    I_lo = torch.empty((n, c, h, w), dtype=TORCH_DTYPES[io_dtype])
    p_lo = torch.empty((n, c, h, w), dtype=TORCH_DTYPES[io_dtype])
    dq = torch.empty((n, c, H, W), dtype=TORCH_DTYPES[io_dtype]) if with_dq else None
    for b in range(n):
        rng = rng_for(config, b, salt=3)
        ih = quantize(photo(rng, c, H, W, noise=noise), io_dtype)
        il = quantize(area_resize(ih.double().numpy(), h, w), io_dtype)
        pl = np.clip(0.8 * il.double().numpy() + 0.1 * rng.normal(0.0, 0.05, size=(c, h, w)),
                     0.0, 1.0)
        I_hi[b] = ih
        I_lo[b] = il
        p_lo[b] = quantize(pl, io_dtype)
        if with_dq:
            dq[b] = quantize(rng.standard_normal((c, H, W)), io_dtype)
    eps_arr = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    return {"I_lo": I_lo, "p_lo": p_lo, "I_hi": I_hi, "dq": dq, "r": int(r),
            "eps": eps_arr.astype(np.float32).astype(np.float64), "s": None, "sx": None,
            "io_dtype": io_dtype, "n": n, "c": c, "H": H, "W": W, "h": h, "w": w}


def guide_params(rng: np.random.Generator, cin: int = 3, cout: int = 3, hidden: int = 15) -> dict:
    """Random parameters of the 3 -> hidden -> 3 guidance transform."""
    return {
        "w1": rng.normal(0.0, 0.1, size=(hidden, cin)),
        "w2": rng.normal(0.0, 0.1, size=(cout, hidden)),
        "b2": rng.normal(0.0, 0.1, size=(cout,)),
        "lam": 1.0,
        "mu": 0.5,
        "gamma": 1.0 + rng.normal(0.0, 0.1, size=(hidden,)),
        "beta": rng.normal(0.0, 0.1, size=(hidden,)),
        "bn_eps": 1e-5,
        "slope": 0.2,
    }


def make_problem(n: int, c: int, H: int, W: int, s: int, r: int, eps, io_dtype: str,
                 config: int, noise: float = 0.0, flat_rects: int = 0, with_dq: bool = True,
                 sx: int | None = None, image_offset: int = 0) -> dict:
    """One batch of n images: quantised CPU tensors plus the problem scalars.

    H and W must be multiples of the downsample factors (s vertically, sx
    horizontally; sx defaults to s).
    """
    sx = s if sx is None else sx
    if H % s or W % sx:
        raise ValueError("H, W must be multiples of the downsample factor")
    h, w = H // s, W // sx
    I_hi = torch.empty((n, c, H, W), dtype=TORCH_DTYPES[io_dtype])
    I_lo = torch.empty((n, c, h, w), dtype=TORCH_DTYPES[io_dtype])
    p_lo = torch.empty((n, c, h, w), dtype=TORCH_DTYPES[io_dtype])
    dq = torch.empty((n, c, H, W), dtype=TORCH_DTYPES[io_dtype]) if with_dq else None
    for b in range(n):
        rng = rng_for(config, image_offset + b)
        ih = quantize(photo(rng, c, H, W, noise=noise, flat_rects=flat_rects), io_dtype)
        il = quantize(area_down(ih.double().numpy(), s, sx), io_dtype)
        pl = np.clip(0.8 * il.double().numpy() + 0.1 * rng.normal(0.0, 0.05, size=(c, h, w)),
                     0.0, 1.0)
        I_hi[b] = ih
        I_lo[b] = il
        p_lo[b] = quantize(pl, io_dtype)
        if with_dq:
            dq[b] = quantize(rng.standard_normal((c, H, W)), io_dtype)
    eps_arr = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    return {"I_lo": I_lo, "p_lo": p_lo, "I_hi": I_hi, "dq": dq, "r": int(r),
            "eps": eps_arr.astype(np.float32).astype(np.float64), "s": s, "sx": sx,
            "io_dtype": io_dtype, "n": n, "c": c, "H": H, "W": W, "h": h, "w": w}


# Workloads of the benchmark/parity configurations (sizes from the
# problem statement of each configuration).
CONFIGS = {
    0: dict(n=1, c=3, H=256, W=256, s=4, r=1, eps=1e-2, io_dtype="f32", noise=0.0),
    1: dict(n=4, c=3, H=2048, W=3072, s=4, r=1, eps=1e-4, io_dtype="f32", noise=0.02),
    2: dict(n=8, c=3, H=1536, W=2048, s=4, r=1, eps=1e-8, io_dtype="bf16", noise=0.02),
    4: dict(n=2, c=3, H=2160, W=3840, s=4, r=8, eps=1e-8, io_dtype="f16", noise=0.0,
            flat_rects=6),
}


def make_config(i: int, *, div: int = 1, r: int | None = None, with_dq: bool = True,
                n: int | None = None) -> dict:
    """Problem of configuration i; `div` shrinks H and W (keeping s)."""
    cfg = dict(CONFIGS[i])
    s = cfg.pop("s")
    H, W = cfg.pop("H") // div, cfg.pop("W") // div
    H, W = max(s, H - H % s), max(s, W - W % s)
    if r is not None:
        cfg["r"] = r
    if n is not None:
        cfg["n"] = n
    prob = make_problem(cfg.pop("n"), cfg.pop("c"), H, W, s, cfg.pop("r"), cfg.pop("eps"),
                        cfg.pop("io_dtype"), config=i, with_dq=with_dq, **cfg)
    if i == 2:
        prob["guide"] = guide_params(rng_for(2, 0, salt=1))
    return prob


def batched_specs(count: int = 64, *, div: int = 1, seed_config: int = 3) -> list:
    """Per-image (H, W, s, r, eps) of the uneven batch, drawn from the stated
    ranges: H, W = 8 * floor(U[512, 3072] / 8) (divided by `div`, kept a
    multiple of 8), s in {2, 4, 8}, r in {1, 2, 4}, eps = 10^U(-8, -2)."""
    rng = rng_for(seed_config, 0, salt=2)
    specs = []
    for k in range(count):
        H = 8 * int(rng.uniform(512, 3072) // 8)
        W = 8 * int(rng.uniform(512, 3072) // 8)
        s = int(rng.choice([2, 4, 8]))
        r = int(rng.choice([1, 2, 4]))
        eps = float(10.0 ** rng.uniform(-8, -2))
        H = max(8, (H // div) // 8 * 8)
        W = max(8, (W // div) // 8 * 8)
        specs.append({"k": k, "H": H, "W": W, "s": s, "r": r, "eps": eps})
    return specs


def batched_item(spec: dict, io_dtype: str = "f32", seed_config: int = 3) -> dict:
    """Image k of the uneven batch (3 channels, noise 0.02)."""
    return make_problem(1, 3, spec["H"], spec["W"], spec["s"], spec["r"], spec["eps"], io_dtype,
                        config=seed_config, noise=0.02, image_offset=spec["k"])


def batched_items(count: int = 64, *, div: int = 1, seed_config: int = 3,
                  io_dtype: str = "f32") -> list:
    """The uneven batch (see batched_specs), one problem per image."""
    return [batched_item(sp, io_dtype, seed_config)
            for sp in batched_specs(count, div=div, seed_config=seed_config)]
