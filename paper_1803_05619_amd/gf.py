"""Python binding of libgf.so, the HIP guided filtering layer (gfx950).

Thin ctypes marshalling over the C ABI declared in include/gf.h: the raw
entry points keep their C names (gf_forward, gf_backward, ...), and
`forward` / `backward` / `guided_filter` wrap them for torch tensors that
live on the GPU.  Every step of the filter runs in the library's kernels;
there is no fallback: importing this module fails if libgf.so is missing.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "gf.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")

lib = ctypes.CDLL(LIB_PATH)

GF_OK, GF_ERR_INVALID_ARG, GF_ERR_UNSUPPORTED, GF_ERR_WORKSPACE, GF_ERR_HIP = range(5)
GF_F32, GF_F16, GF_BF16 = 0, 1, 2
DTYPE_CODES = {torch.float32: GF_F32, torch.float16: GF_F16, torch.bfloat16: GF_BF16}


class gf_desc_t(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("n", "c", "h_lo", "w_lo", "h_hi", "w_hi", "r", "mean_ab", "io_dtype",
                 "align_corners", "precise")]


GF_GUIDE_IDENTITY, GF_GUIDE_GREY, GF_GUIDE_TRANSFORM = 0, 1, 2


class gf_guide_t(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("c_in", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("bn_eps", ctypes.c_float), ("slope", ctypes.c_float),
                ("params", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("use_stats", ctypes.c_int32)]


_vp = ctypes.c_void_p
_fp = ctypes.c_void_p  # float* passed as raw addresses
_dp = ctypes.POINTER(gf_desc_t)
_gp = ctypes.POINTER(gf_guide_t)
lib.gf_guide_param_count.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
lib.gf_guide_param_count.restype = ctypes.c_size_t
lib.gf_guide_stats_count.argtypes = [ctypes.c_int32]
lib.gf_guide_stats_count.restype = ctypes.c_size_t
lib.gf_workspace_size.argtypes = [_dp, _gp, ctypes.c_int32]
lib.gf_workspace_size.restype = ctypes.c_size_t
lib.gf_forward.argtypes = [_dp, _gp, _vp, _vp, _vp, _fp, ctypes.c_int32, _vp, _vp,
                           ctypes.c_size_t, _vp]
lib.gf_forward.restype = ctypes.c_int32
lib.gf_backward.argtypes = [_dp, _gp, _vp, _vp, _vp, _fp, ctypes.c_int32, _vp, _fp, _fp, _vp,
                            _fp, _fp, _vp, ctypes.c_size_t, _vp]
lib.gf_backward.restype = ctypes.c_int32
lib.gf_forward_backward.argtypes = [_dp, _gp, _vp, _vp, _vp, _fp, ctypes.c_int32, _vp, _vp, _fp,
                                    _fp, _vp, _fp, _fp, _vp, ctypes.c_size_t, _vp]
lib.gf_forward_backward.restype = ctypes.c_int32
lib.gf_forward_backward_static.argtypes = [_dp, _gp, _vp, _vp, _vp, _fp, ctypes.c_int32, _vp,
                                           _vp, _fp, _fp, _vp, _fp, _fp, _vp]
lib.gf_forward_backward_static.restype = ctypes.c_int32
lib.gf_downsample.argtypes = [ctypes.c_int32] * 7 + [_vp, _vp, _vp]
lib.gf_downsample.restype = ctypes.c_int32


class gf_conv_t(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("slope", ctypes.c_float), ("params", ctypes.c_void_p)]


_cp = ctypes.POINTER(gf_conv_t)
lib.gf_conv_param_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
lib.gf_conv_param_count.restype = ctypes.c_size_t
lib.gf_conv_workspace_size.argtypes = [_dp, _cp, ctypes.c_int32]
lib.gf_conv_workspace_size.restype = ctypes.c_size_t
lib.gf_conv_forward.argtypes = [_dp, _cp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
lib.gf_conv_forward.restype = ctypes.c_int32
lib.gf_conv_backward.argtypes = [_dp, _cp, _vp, _vp, _vp, _vp, _fp, _fp, _vp, _fp, _vp,
                                 ctypes.c_size_t, _vp]
lib.gf_conv_backward.restype = ctypes.c_int32
GF_RUN_FORWARD, GF_RUN_BACKWARD, GF_RUN_GRAPH = 1, 2, 4


class gf_item_t(ctypes.Structure):
    _fields_ = [("d", gf_desc_t), ("eps", ctypes.c_float),
                ("I_lo", ctypes.c_void_p), ("p_lo", ctypes.c_void_p), ("I_hi", ctypes.c_void_p),
                ("q_hi", ctypes.c_void_p), ("dq_hi", ctypes.c_void_p),
                ("dI_lo", ctypes.c_void_p), ("dp_lo", ctypes.c_void_p),
                ("dI_hi", ctypes.c_void_p), ("deps", ctypes.c_void_p)]


lib.gf_plan_create.argtypes = [ctypes.POINTER(gf_item_t), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_void_p)]
lib.gf_plan_create.restype = ctypes.c_int32
lib.gf_plan_workspace_size.argtypes = [_vp]
lib.gf_plan_workspace_size.restype = ctypes.c_size_t
lib.gf_batched.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
lib.gf_batched.restype = ctypes.c_int32
lib.gf_plan_destroy.argtypes = [_vp]
lib.gf_plan_destroy.restype = None
lib.gf_autotune.argtypes = [_dp, _gp, _vp, _vp, _vp, _fp, ctypes.c_int32, _vp, _vp, _fp, _fp, _vp,
                            _fp, _fp, _vp, ctypes.c_size_t, ctypes.c_int32, _vp]
lib.gf_autotune.restype = ctypes.c_int32
lib.gf_tune_export.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
lib.gf_tune_export.restype = ctypes.c_size_t
lib.gf_tune_import.argtypes = [ctypes.c_char_p]
lib.gf_tune_import.restype = ctypes.c_int32
lib.gf_status_string.argtypes = [ctypes.c_int32]
lib.gf_status_string.restype = ctypes.c_char_p
lib.gf_last_error_detail.argtypes = []
lib.gf_last_error_detail.restype = ctypes.c_char_p
lib.gf_profile_enable.argtypes = [ctypes.c_int32]
lib.gf_profile_enable.restype = ctypes.c_int32
lib.gf_profile_read.argtypes = [_vp, _vp, _vp, ctypes.c_int32]
lib.gf_profile_read.restype = ctypes.c_int32


def header_functions(path: str = HEADER_PATH) -> list:
    """Names of the functions include/gf.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_]+)\s*\(", text)))


class GFError(RuntimeError):
    def __init__(self, code: int):
        self.code = code
        super().__init__(f"{gf_status_string(code)}: {gf_last_error_detail()}")


# ------------------------------------------------------------------ raw C ABI

def _gref(guide):
    return None if guide is None else ctypes.byref(guide)


def gf_guide_param_count(c_in: int, c: int, hidden: int) -> int:
    return int(lib.gf_guide_param_count(c_in, c, hidden))


def gf_guide_stats_count(c_in: int) -> int:
    return int(lib.gf_guide_stats_count(c_in))


def gf_workspace_size(desc: gf_desc_t, guide, backward: int) -> int:
    return int(lib.gf_workspace_size(ctypes.byref(desc), _gref(guide), int(backward)))


def gf_forward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, q_hi, ws, ws_bytes, stream) -> int:
    return int(lib.gf_forward(ctypes.byref(desc), _gref(guide), I_lo, p_lo, I_hi, eps, eps_count,
                              q_hi, ws, ws_bytes, stream))


def gf_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, dI_lo, dp_lo, dI_hi, deps,
                dparams, ws, ws_bytes, stream) -> int:
    return int(lib.gf_backward(ctypes.byref(desc), _gref(guide), I_lo, p_lo, I_hi, eps,
                               eps_count, dq_hi, dI_lo, dp_lo, dI_hi, deps, dparams, ws,
                               ws_bytes, stream))


def gf_plan_create(items, count):
    """Returns (status, plan handle or None); `items` a ctypes gf_item_t array."""
    h = ctypes.c_void_p()
    st = int(lib.gf_plan_create(items, int(count), ctypes.byref(h)))
    return st, (h.value if st == GF_OK else None)


def gf_plan_workspace_size(plan) -> int:
    return int(lib.gf_plan_workspace_size(plan))


def gf_batched(plan, mode, ws, ws_bytes, stream) -> int:
    return int(lib.gf_batched(plan, int(mode), ws, ws_bytes, stream))


def gf_plan_destroy(plan) -> None:
    lib.gf_plan_destroy(plan)


def gf_autotune(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, q_hi, dq_hi, dI_lo, dp_lo, dI_hi,
                deps, dparams, ws, ws_bytes, iters, stream) -> int:
    return int(lib.gf_autotune(ctypes.byref(desc), _gref(guide), I_lo, p_lo, I_hi, eps,
                               eps_count, q_hi, dq_hi, dI_lo, dp_lo, dI_hi, deps, dparams, ws,
                               ws_bytes, int(iters), stream))


def gf_tune_export() -> str:
    n = int(lib.gf_tune_export(None, 0))
    buf = ctypes.create_string_buffer(n + 1)
    lib.gf_tune_export(buf, n + 1)
    return buf.value.decode()


def gf_tune_import(text: str) -> int:
    return int(lib.gf_tune_import(text.encode()))


def gf_forward_backward(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, q_hi, dI_lo, dp_lo,
                        dI_hi, deps, dparams, ws, ws_bytes, stream) -> int:
    return int(lib.gf_forward_backward(ctypes.byref(desc), _gref(guide), I_lo, p_lo, I_hi, eps,
                                       eps_count, dq_hi, q_hi, dI_lo, dp_lo, dI_hi, deps,
                                       dparams, ws, ws_bytes, stream))


def gf_forward_backward_static(desc, guide, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, q_hi, dI_lo,
                               dp_lo, dI_hi, deps, dparams, stream) -> int:
    return int(lib.gf_forward_backward_static(ctypes.byref(desc), _gref(guide), I_lo, p_lo, I_hi,
                                              eps, eps_count, dq_hi, q_hi, dI_lo, dp_lo, dI_hi,
                                              deps, dparams, stream))


def gf_downsample(n, c, h_hi, w_hi, h_lo, w_lo, io_dtype, I_hi, I_lo, stream) -> int:
    return int(lib.gf_downsample(n, c, h_hi, w_hi, h_lo, w_lo, io_dtype, I_hi, I_lo, stream))


def gf_conv_param_count(c: int, hidden: int) -> int:
    return int(lib.gf_conv_param_count(int(c), int(hidden)))


def gf_conv_workspace_size(desc, conv, backward: int) -> int:
    return int(lib.gf_conv_workspace_size(ctypes.byref(desc), ctypes.byref(conv), int(backward)))


def gf_conv_forward(desc, conv, I_lo, p_lo, I_hi, q_hi, ws, ws_bytes, stream) -> int:
    return int(lib.gf_conv_forward(ctypes.byref(desc), ctypes.byref(conv), I_lo, p_lo, I_hi,
                                   q_hi, ws, ws_bytes, stream))


def gf_conv_backward(desc, conv, I_lo, p_lo, I_hi, dq_hi, dI_lo, dp_lo, dI_hi, dparams, ws,
                     ws_bytes, stream) -> int:
    return int(lib.gf_conv_backward(ctypes.byref(desc), ctypes.byref(conv), I_lo, p_lo, I_hi,
                                    dq_hi, dI_lo, dp_lo, dI_hi, dparams, ws, ws_bytes, stream))


def gf_status_string(code: int) -> str:
    return lib.gf_status_string(int(code)).decode()


def gf_last_error_detail() -> str:
    return lib.gf_last_error_detail().decode()


def gf_profile_enable(on: bool) -> None:
    lib.gf_profile_enable(1 if on else 0)


def gf_profile_read(cap: int = 32) -> dict:
    """{kernel name: (total ms, launches)} since gf_profile_enable(True)."""
    names = ctypes.create_string_buffer(48 * cap)
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int32 * cap)()
    m = lib.gf_profile_read(ctypes.addressof(names), ctypes.addressof(ms), ctypes.addressof(cnt),
                            cap)
    out = {}
    for k in range(min(m, cap)):
        name = names.raw[48 * k:48 * (k + 1)].split(b"\0", 1)[0].decode()
        out[name] = (ms[k], cnt[k])
    return out


# ------------------------------------------------------------------ torch level

def _ptr(t):
    return None if t is None else t.data_ptr()


def make_desc(I_lo: torch.Tensor, I_hi: torch.Tensor, r: int, mean_ab: bool = True,
              c: int = None, align_corners: bool = False, precise: bool = False) -> gf_desc_t:
    """Problem description; `c` (output channels) defaults to I_lo's channels
    (a guide may map c_in input channels to c).  `precise`: FP64 window sums
    at every radius (see gf_desc_t.precise)."""
    n, c_in, h, w = I_lo.shape
    H, W = I_hi.shape[-2:]
    return gf_desc_t(n, c_in if c is None else int(c), h, w, H, W, int(r), int(bool(mean_ab)),
                     DTYPE_CODES[I_lo.dtype], int(bool(align_corners)), int(bool(precise)))


class Guide:
    """Host description of the guidance map G = F(I) (gf_guide_t).

    mode: GF_GUIDE_GREY (channel mean of c_in channels) or GF_GUIDE_TRANSFORM
    (1x1 conv -> adaptive BN -> leaky ReLU -> 1x1 conv; `params` a float32
    device tensor of gf_guide_param_count(c_in, c, hidden) entries, see
    `pack_transform_params`).  `stats` (optional float32 device tensor of
    gf_guide_stats_count(c_in) entries) receives the forward's batch
    statistics; with use_stats the backward reads them back."""

    def __init__(self, mode, c_in, hidden=0, params=None, bn_eps=1e-5, slope=0.2, stats=None,
                 use_stats=False):
        self.mode, self.c_in, self.hidden = int(mode), int(c_in), int(hidden)
        self.params, self.stats, self.use_stats = params, stats, bool(use_stats)
        self.bn_eps, self.slope = float(bn_eps), float(slope)

    def struct(self) -> gf_guide_t:
        return gf_guide_t(self.mode, self.c_in, self.hidden, self.bn_eps, self.slope,
                          _ptr(self.params), _ptr(self.stats), int(self.use_stats))


def pack_transform_params(w1, w2, b2, lam, mu, gamma, beta, device=None) -> torch.Tensor:
    """Flat float32 parameter vector of the transform guide:
    W1 [hidden][c_in] | W2 [c][hidden] | b2 [c] | lam | mu | gamma | beta."""
    parts = [torch.as_tensor(x, dtype=torch.float32).reshape(-1)
             for x in (w1, w2, b2, [float(lam)], [float(mu)], gamma, beta)]
    return torch.cat(parts).to(device).contiguous()


def unpack_transform_params(v: torch.Tensor, c_in: int, c: int, hidden: int) -> dict:
    """Inverse of pack_transform_params (views into v)."""
    sizes = [hidden * c_in, c * hidden, c, 1, 1, hidden, hidden]
    names = ["w1", "w2", "b2", "lam", "mu", "gamma", "beta"]
    out, o = {}, 0
    for name, k in zip(names, sizes):
        out[name] = v[o:o + k]
        o += k
    out["w1"] = out["w1"].reshape(hidden, c_in)
    out["w2"] = out["w2"].reshape(c, hidden)
    return out


def _check(tensors, dtype, device):
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda or t.device != device:
            raise ValueError(f"{name} must be on {device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


def _eps_tensor(eps, n, device):
    if isinstance(eps, torch.Tensor):
        e = eps.to(device=device, dtype=torch.float32).reshape(-1).contiguous()
    else:
        e = torch.tensor([float(x) for x in (eps if hasattr(eps, "__len__") else [eps])],
                         dtype=torch.float32, device=device)
    if e.numel() not in (1, n):
        raise ValueError("eps must have 1 or n entries")
    return e


def _ws(nbytes, device, ws):
    if ws is not None and ws.numel() >= nbytes:
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def _out_channels(I_lo, guide, c):
    if c is not None:
        return int(c)
    if guide is not None and guide.mode == GF_GUIDE_TRANSFORM:
        return 3
    return I_lo.shape[1]


def forward(I_lo, p_lo, I_hi, eps, r=1, mean_ab=True, out=None, ws=None, guide=None,
            align_corners=False, precise=False):
    """q = GF(I_lo, p_lo, I_hi): one gf_forward call on the current stream.
    With a Guide, I_lo and I_hi have guide.c_in channels and q has p_lo's."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, out=out), I_hi.dtype, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab, c=p_lo.shape[1], align_corners=align_corners,
                     precise=precise)
    g = None if guide is None else guide.struct()
    e = _eps_tensor(eps, desc.n, dev)
    q = out if out is not None else torch.empty(
        (desc.n, desc.c, desc.h_hi, desc.w_hi), dtype=I_hi.dtype, device=dev)
    need = gf_workspace_size(desc, g, 0)
    if need == 0 and ws is None:
        st = gf_forward(desc, g, None, None, None, None, 0, None, None, 0, None)
        raise GFError(st if st != GF_OK else GF_ERR_INVALID_ARG)
    ws = _ws(need, dev, ws)
    st = gf_forward(desc, g, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.numel(), _ptr(q),
                    _ptr(ws), ws.numel(), _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return q


def backward(I_lo, p_lo, I_hi, eps, dq, r=1, mean_ab=True, need_dI_lo=True, need_dp_lo=True,
             need_dI_hi=True, need_deps=True, ws=None, outs=None, guide=None,
             need_dparams=None, align_corners=False, precise=False):
    """Gradients (dI_lo, dp_lo, dI_hi, deps, dparams) of sum(q * dq); None
    where not requested.  dparams only with a transform Guide (requested by
    default there)."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, dq=dq), I_hi.dtype, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab, c=p_lo.shape[1], align_corners=align_corners,
                     precise=precise)
    g = None if guide is None else guide.struct()
    transform = guide is not None and guide.mode == GF_GUIDE_TRANSFORM
    if need_dparams is None:
        need_dparams = transform
    e = _eps_tensor(eps, desc.n, dev)
    f32 = dict(dtype=torch.float32, device=dev)
    if outs is not None:
        dI_lo, dp_lo, dI_hi, deps = outs[:4]
        dparams = outs[4] if len(outs) > 4 else None
    else:
        dI_lo = torch.empty(I_lo.shape, **f32) if need_dI_lo else None
        dp_lo = torch.empty(p_lo.shape, **f32) if need_dp_lo else None
        dI_hi = torch.empty_like(I_hi) if need_dI_hi else None
        deps = torch.empty(e.numel(), **f32) if need_deps else None
        dparams = None
        if need_dparams and transform:
            dparams = torch.empty(gf_guide_param_count(guide.c_in, desc.c, guide.hidden), **f32)
    _check(dict(dI_lo=dI_lo, dp_lo=dp_lo, deps=deps, dparams=dparams), torch.float32, dev)
    _check(dict(dI_hi=dI_hi), I_hi.dtype, dev)
    nbytes = gf_workspace_size(desc, g, 1)
    ws = _ws(nbytes, dev, ws)
    st = gf_backward(desc, g, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.numel(), _ptr(dq),
                     _ptr(dI_lo), _ptr(dp_lo), _ptr(dI_hi), _ptr(deps), _ptr(dparams), _ptr(ws),
                     ws.numel(), _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return dI_lo, dp_lo, dI_hi, deps, dparams


def forward_backward(I_lo, p_lo, I_hi, eps, dq, r=1, mean_ab=True, ws=None, outs=None,
                     guide=None, need_dI_lo=True, need_dp_lo=True, need_dI_hi=True,
                     need_deps=True, need_dparams=None, align_corners=False, precise=False):
    """q and the gradients (dI_lo, dp_lo, dI_hi, deps, dparams) in one call
    (gf_forward_backward: coefficients and guide maps computed once)."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, dq=dq), I_hi.dtype, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab, c=p_lo.shape[1], align_corners=align_corners,
                     precise=precise)
    g = None if guide is None else guide.struct()
    transform = guide is not None and guide.mode == GF_GUIDE_TRANSFORM
    if need_dparams is None:
        need_dparams = transform
    e = _eps_tensor(eps, desc.n, dev)
    f32 = dict(dtype=torch.float32, device=dev)
    if outs is not None:
        q, dI_lo, dp_lo, dI_hi, deps = outs[:5]
        dparams = outs[5] if len(outs) > 5 else None
    else:
        q = torch.empty((desc.n, desc.c, desc.h_hi, desc.w_hi), dtype=I_hi.dtype, device=dev)
        dI_lo = torch.empty(I_lo.shape, **f32) if need_dI_lo else None
        dp_lo = torch.empty(p_lo.shape, **f32) if need_dp_lo else None
        dI_hi = torch.empty_like(I_hi) if need_dI_hi else None
        deps = torch.empty(e.numel(), **f32) if need_deps else None
        dparams = None
        if need_dparams and transform:
            dparams = torch.empty(gf_guide_param_count(guide.c_in, desc.c, guide.hidden), **f32)
    _check(dict(dI_lo=dI_lo, dp_lo=dp_lo, deps=deps, dparams=dparams), torch.float32, dev)
    _check(dict(q=q, dI_hi=dI_hi), I_hi.dtype, dev)
    ws = _ws(gf_workspace_size(desc, g, 2), dev, ws)
    st = gf_forward_backward(desc, g, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.numel(),
                             _ptr(dq), _ptr(q), _ptr(dI_lo), _ptr(dp_lo), _ptr(dI_hi), _ptr(deps),
                             _ptr(dparams), _ptr(ws), ws.numel(), _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return q, dI_lo, dp_lo, dI_hi, deps, dparams


def downsample(I_hi: torch.Tensor, h: int, w: int, out: torch.Tensor = None) -> torch.Tensor:
    """I_l = area downsampling of I_hi [n, c, H, W] to (h, w): one
    gf_downsample call on the current stream (the first step of the deep
    guided filtering network, Sec. IV)."""
    dev = I_hi.device
    _check(dict(I_hi=I_hi, out=out), I_hi.dtype, dev)
    n, c, H, W = I_hi.shape
    if out is None:
        out = torch.empty((n, c, int(h), int(w)), dtype=I_hi.dtype, device=dev)
    st = gf_downsample(n, c, H, W, int(h), int(w), DTYPE_CODES[I_hi.dtype], _ptr(I_hi),
                       _ptr(out), _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return out


# ------------------------------------------------------------------ convolutional layer

CONV_HIDDEN = 16


def pack_conv_params(D, W1, W2, W3, device=None) -> torch.Tensor:
    """Flat float32 parameters of the convolutional layer: D [c][3][3] |
    W1 [K][2c] | W2 [K][K] | W3 [c][K]."""
    parts = [torch.as_tensor(x, dtype=torch.float32).reshape(-1) for x in (D, W1, W2, W3)]
    return torch.cat(parts).to(device).contiguous()


def _conv_struct(params, hidden, slope):
    return gf_conv_t(int(hidden), float(slope), _ptr(params))


def conv_forward(I_lo, p_lo, I_hi, params, r=1, hidden=CONV_HIDDEN, slope=0.2, mean_ab=True,
                 out=None, ws=None, align_corners=False):
    """q of the convolutional guided filtering layer (Sec. III-E): one
    gf_conv_forward call on the current stream; r is the dilation."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, out=out), I_hi.dtype, dev)
    _check(dict(params=params), torch.float32, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab, align_corners=align_corners)
    cv = _conv_struct(params, hidden, slope)
    q = out if out is not None else torch.empty_like(I_hi)
    ws = _ws(gf_conv_workspace_size(desc, cv, 0), dev, ws)
    st = gf_conv_forward(desc, cv, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(q), _ptr(ws),
                         ws.numel(), _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return q


def conv_backward(I_lo, p_lo, I_hi, params, dq, r=1, hidden=CONV_HIDDEN, slope=0.2,
                  mean_ab=True, need_dI_lo=True, need_dp_lo=True, need_dI_hi=True,
                  need_dparams=True, ws=None, align_corners=False):
    """(dI_lo, dp_lo, dI_hi, dparams) of the convolutional layer; the low-res
    gradients and dparams are float32."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, dq=dq), I_hi.dtype, dev)
    _check(dict(params=params), torch.float32, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab, align_corners=align_corners)
    cv = _conv_struct(params, hidden, slope)
    f32 = dict(dtype=torch.float32, device=dev)
    dI_lo = torch.empty(I_lo.shape, **f32) if need_dI_lo else None
    dp_lo = torch.empty(p_lo.shape, **f32) if need_dp_lo else None
    dI_hi = torch.empty_like(I_hi) if need_dI_hi else None
    dparams = torch.empty(params.numel(), **f32) if need_dparams else None
    ws = _ws(gf_conv_workspace_size(desc, cv, 1), dev, ws)
    st = gf_conv_backward(desc, cv, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(dq), _ptr(dI_lo),
                          _ptr(dp_lo), _ptr(dI_hi), _ptr(dparams), _ptr(ws), ws.numel(),
                          _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return dI_lo, dp_lo, dI_hi, dparams


class ConvGuidedFilterFn(torch.autograd.Function):
    """Differentiable convolutional guided filtering layer; the backward
    recomputes the low-res statistics from the saved inputs."""

    @staticmethod
    def forward(ctx, I_lo, p_lo, I_hi, params, r, hidden, slope, mean_ab):
        ctx.cfg = (r, hidden, slope, mean_ab)
        ctx.save_for_backward(I_lo, p_lo, I_hi, params)
        return conv_forward(I_lo, p_lo, I_hi, params, r, hidden, slope, mean_ab)

    @staticmethod
    def backward(ctx, dq):
        I_lo, p_lo, I_hi, params = ctx.saved_tensors
        r, hidden, slope, mean_ab = ctx.cfg
        need = ctx.needs_input_grad
        dI_lo, dp_lo, dI_hi, dparams = conv_backward(
            I_lo, p_lo, I_hi, params, dq.contiguous(), r, hidden, slope, mean_ab,
            need_dI_lo=need[0], need_dp_lo=need[1], need_dI_hi=need[2], need_dparams=need[3])
        cast = lambda g, ref: None if g is None else g.to(ref.dtype)
        return cast(dI_lo, I_lo), cast(dp_lo, p_lo), dI_hi, dparams, None, None, None, None


def conv_guided_filter(I_lo, p_lo, I_hi, params, r=1, hidden=CONV_HIDDEN, slope=0.2,
                       mean_ab=True):
    """The convolutional guided filtering layer with autograd (gradients to
    I_lo, p_lo, I_hi and params)."""
    return ConvGuidedFilterFn.apply(I_lo, p_lo, I_hi, params, r, hidden, slope, mean_ab)


class GuidedFilterFn(torch.autograd.Function):
    """Differentiable guided filtering layer; the backward recomputes the
    low-res statistics from the saved inputs (nothing else is stored, apart
    from the transform guide's 24 batch statistics)."""

    @staticmethod
    def forward(ctx, I_lo, p_lo, I_hi, eps, r, mean_ab, guide, params, align_corners, precise):
        e = _eps_tensor(eps, I_lo.shape[0], I_hi.device)
        ctx.r, ctx.mean_ab, ctx.ac, ctx.precise = r, mean_ab, align_corners, precise
        ctx.eps_is_tensor = isinstance(eps, torch.Tensor)
        ctx.guide = guide
        stats = None
        if guide is not None and guide.mode == GF_GUIDE_TRANSFORM:
            stats = torch.empty(gf_guide_stats_count(guide.c_in), dtype=torch.float32,
                                device=I_hi.device)
            guide = Guide(guide.mode, guide.c_in, guide.hidden, params, guide.bn_eps,
                          guide.slope, stats, False)
        ctx.save_for_backward(I_lo, p_lo, I_hi, e, params, stats)
        return forward(I_lo, p_lo, I_hi, e, r, mean_ab, guide=guide, align_corners=align_corners,
                       precise=precise)

    @staticmethod
    def backward(ctx, dq):
        I_lo, p_lo, I_hi, e, params, stats = ctx.saved_tensors
        need = ctx.needs_input_grad
        guide = ctx.guide
        if guide is not None and guide.mode == GF_GUIDE_TRANSFORM:
            guide = Guide(guide.mode, guide.c_in, guide.hidden, params, guide.bn_eps,
                          guide.slope, stats, True)
        dI_lo, dp_lo, dI_hi, deps, dparams = backward(
            I_lo, p_lo, I_hi, e, dq.contiguous(), ctx.r, ctx.mean_ab,
            need_dI_lo=need[0], need_dp_lo=need[1], need_dI_hi=need[2],
            need_deps=need[3] and ctx.eps_is_tensor, guide=guide,
            need_dparams=len(need) > 7 and need[7], align_corners=ctx.ac, precise=ctx.precise)
        cast = lambda g, ref: None if g is None else g.to(ref.dtype)
        return (cast(dI_lo, I_lo), cast(dp_lo, p_lo), dI_hi, deps, None, None, None, dparams,
                None, None)


def guided_filter(I_lo, p_lo, I_hi, r=1, eps=1e-8, mean_ab=True, guide=None,
                  align_corners=False, precise=False):
    """Autograd entry point: q = GF(I_lo, p_lo, I_hi) with radius r and eps
    (a float, or a float32 tensor of 1 or n entries to get its gradient).
    `guide` is None (identity) or a Guide; a transform Guide's `params`
    tensor receives its gradient.  `precise`: FP64 window sums at every
    radius (FP32-level accuracy at tiny eps on nearly flat guides)."""
    params = guide.params if guide is not None else None
    return GuidedFilterFn.apply(I_lo, p_lo, I_hi, eps, r, mean_ab, guide, params, align_corners,
                                precise)


# ------------------------------------------------------------------ batched

class BatchPlan:
    """Many independent problems (identity guide, one dtype) run as one launch
    per phase and launch class (gf_plan_create / gf_batched).

    items: list of dicts with I_lo, p_lo, I_hi (device tensors), r, eps and
    optionally mean_ab (default True), precise (default False) and the outputs q, dq, dI_lo, dp_lo,
    dI_hi, deps (device tensors; deps one float32).  The plan keeps the
    tensors alive and every run reads and writes them in place."""

    def __init__(self, items):
        self.items = [dict(it) for it in items]
        arr = (gf_item_t * len(items))()
        for k, it in enumerate(self.items):
            I_lo, I_hi, p_lo = it["I_lo"], it["I_hi"], it["p_lo"]
            dev = I_hi.device
            _check({f"item {k} " + n: it.get(n) for n in ("I_lo", "p_lo", "I_hi", "q", "dq",
                                                           "dI_hi")}, I_hi.dtype, dev)
            _check({f"item {k} " + n: it.get(n) for n in ("dI_lo", "dp_lo", "deps")},
                   torch.float32, dev)
            arr[k].d = make_desc(I_lo, I_hi, it["r"], it.get("mean_ab", True), c=p_lo.shape[1],
                                 align_corners=it.get("align_corners", False),
                                 precise=it.get("precise", False))
            arr[k].eps = float(it["eps"])
            for field, key in (("I_lo", "I_lo"), ("p_lo", "p_lo"), ("I_hi", "I_hi"),
                               ("q_hi", "q"), ("dq_hi", "dq"), ("dI_lo", "dI_lo"),
                               ("dp_lo", "dp_lo"), ("dI_hi", "dI_hi"), ("deps", "deps")):
                setattr(arr[k], field, _ptr(it.get(key)))
        self._arr = arr
        st, self.handle = gf_plan_create(arr, len(items))
        if st != GF_OK:
            raise GFError(st)
        self.device = self.items[0]["I_hi"].device
        self.ws = torch.empty(max(gf_plan_workspace_size(self.handle), 256), dtype=torch.uint8,
                              device=self.device)

    def run(self, mode=GF_RUN_FORWARD | GF_RUN_BACKWARD, graph=False):
        m = int(mode) | (GF_RUN_GRAPH if graph else 0)
        st = gf_batched(self.handle, m, self.ws.data_ptr(), self.ws.numel(),
                        _stream(self.device))
        if st != GF_OK:
            raise GFError(st)

    def close(self):
        if getattr(self, "handle", None):
            gf_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(I_lo, p_lo, I_hi, eps, dq, r=1, mean_ab=True, iters=5, guide=None,
             align_corners=False, precise=False):
    """Times the candidate launch shapes on these buffers and stores the
    fastest per kernel for this (dtype, factor, radius, guide, mean_ab).  The
    key leaves out `precise`: shapes tuned with one walker kind are used by
    the other as well (every candidate is valid for both), so tune with the
    setting that will run."""
    dev = I_hi.device
    desc = make_desc(I_lo, I_hi, r, mean_ab, c=p_lo.shape[1], align_corners=align_corners,
                     precise=precise)
    g = None if guide is None else guide.struct()
    e = _eps_tensor(eps, desc.n, dev)
    f32 = dict(dtype=torch.float32, device=dev)
    q = torch.empty((desc.n, desc.c, desc.h_hi, desc.w_hi), dtype=I_hi.dtype, device=dev)
    dI_lo = torch.empty(I_lo.shape, **f32)
    dp_lo = torch.empty(p_lo.shape, **f32)
    dI_hi = torch.empty_like(I_hi)
    deps = torch.empty(e.numel(), **f32)
    dparams = None
    if guide is not None and guide.mode == GF_GUIDE_TRANSFORM:
        dparams = torch.empty(gf_guide_param_count(guide.c_in, desc.c, guide.hidden), **f32)
    # room for the largest candidate shapes
    nbytes = 2 * max(gf_workspace_size(desc, g, 0), gf_workspace_size(desc, g, 1)) + (1 << 20)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = gf_autotune(desc, g, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.numel(), _ptr(q),
                     _ptr(dq), _ptr(dI_lo), _ptr(dp_lo), _ptr(dI_hi), _ptr(deps), _ptr(dparams),
                     _ptr(ws), ws.numel(), iters, _stream(dev))
    if st != GF_OK:
        raise GFError(st)


def autotune_batch(items, iters=3):
    """Autotune the launch shapes for a batch of items (BatchPlan's item
    dicts) before creating its plan: once per (factor, radius, mean_ab,
    alignment) key, on that key's largest image repeated as many times as
    the key has items, since the batched launch sees about that much work
    (which decides between short and long walks)."""
    keys = {}
    for it in items:
        s = it["I_hi"].shape[-1] // it["I_lo"].shape[-1]
        key = (s, it["r"], bool(it.get("mean_ab", True)), bool(it.get("align_corners", False)))
        big, cnt = keys.get(key, (None, 0))
        size = it["I_hi"].shape[-2] * it["I_hi"].shape[-1]
        if big is None or size > big[0]:
            big = (size, it)
        keys[key] = (big, cnt + 1)
    for key, ((_, it), cnt) in sorted(keys.items()):
        rep = lambda x: x.expand(cnt * x.shape[0], *x.shape[1:]).contiguous() \
            if x.shape[0] == 1 else torch.cat([x] * cnt)
        autotune(rep(it["I_lo"]), rep(it["p_lo"]), rep(it["I_hi"]), it["eps"], rep(it["dq"]),
                 r=it["r"], mean_ab=it.get("mean_ab", True), iters=iters,
                 align_corners=it.get("align_corners", False))
        torch.cuda.empty_cache()
    return len(keys)
