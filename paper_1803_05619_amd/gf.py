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
                ("n", "c", "h_lo", "w_lo", "h_hi", "w_hi", "r", "mean_ab", "io_dtype")]


_vp = ctypes.c_void_p
_fp = ctypes.c_void_p  # float* passed as raw addresses
lib.gf_workspace_size.argtypes = [ctypes.POINTER(gf_desc_t), ctypes.c_int32]
lib.gf_workspace_size.restype = ctypes.c_size_t
lib.gf_forward.argtypes = [ctypes.POINTER(gf_desc_t), _vp, _vp, _vp, _fp, ctypes.c_int32, _vp,
                           _vp, ctypes.c_size_t, _vp]
lib.gf_forward.restype = ctypes.c_int32
lib.gf_backward.argtypes = [ctypes.POINTER(gf_desc_t), _vp, _vp, _vp, _fp, ctypes.c_int32, _vp,
                            _fp, _fp, _vp, _fp, _vp, ctypes.c_size_t, _vp]
lib.gf_backward.restype = ctypes.c_int32
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

def gf_workspace_size(desc: gf_desc_t, backward: int) -> int:
    return int(lib.gf_workspace_size(ctypes.byref(desc), int(backward)))


def gf_forward(desc, I_lo, p_lo, I_hi, eps, eps_count, q_hi, ws, ws_bytes, stream) -> int:
    return int(lib.gf_forward(ctypes.byref(desc), I_lo, p_lo, I_hi, eps, eps_count, q_hi, ws,
                              ws_bytes, stream))


def gf_backward(desc, I_lo, p_lo, I_hi, eps, eps_count, dq_hi, dI_lo, dp_lo, dI_hi, deps, ws,
                ws_bytes, stream) -> int:
    return int(lib.gf_backward(ctypes.byref(desc), I_lo, p_lo, I_hi, eps, eps_count, dq_hi,
                               dI_lo, dp_lo, dI_hi, deps, ws, ws_bytes, stream))


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


def make_desc(I_lo: torch.Tensor, I_hi: torch.Tensor, r: int, mean_ab: bool = True) -> gf_desc_t:
    n, c, h, w = I_lo.shape
    H, W = I_hi.shape[-2:]
    return gf_desc_t(n, c, h, w, H, W, int(r), int(bool(mean_ab)), DTYPE_CODES[I_lo.dtype])


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


def forward(I_lo, p_lo, I_hi, eps, r=1, mean_ab=True, out=None, ws=None):
    """q = GF(I_lo, p_lo, I_hi): one gf_forward call on the current stream."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, out=out), I_hi.dtype, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab)
    e = _eps_tensor(eps, desc.n, dev)
    q = out if out is not None else torch.empty_like(I_hi)
    need = gf_workspace_size(desc, 0)
    ws = _ws(need, dev, ws)
    st = gf_forward(desc, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.numel(), _ptr(q),
                    _ptr(ws), ws.numel(), _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return q


def backward(I_lo, p_lo, I_hi, eps, dq, r=1, mean_ab=True, need_dI_lo=True, need_dp_lo=True,
             need_dI_hi=True, need_deps=True, ws=None, outs=None):
    """Gradients (dI_lo, dp_lo, dI_hi, deps) of sum(q * dq); None where not requested."""
    dev = I_hi.device
    _check(dict(I_lo=I_lo, p_lo=p_lo, I_hi=I_hi, dq=dq), I_hi.dtype, dev)
    desc = make_desc(I_lo, I_hi, r, mean_ab)
    e = _eps_tensor(eps, desc.n, dev)
    if outs is not None:
        dI_lo, dp_lo, dI_hi, deps = outs
    else:
        f32 = dict(dtype=torch.float32, device=dev)
        dI_lo = torch.empty(I_lo.shape, **f32) if need_dI_lo else None
        dp_lo = torch.empty(p_lo.shape, **f32) if need_dp_lo else None
        dI_hi = torch.empty_like(I_hi) if need_dI_hi else None
        deps = torch.empty(e.numel(), **f32) if need_deps else None
    _check(dict(dI_lo=dI_lo, dp_lo=dp_lo, deps=deps), torch.float32, dev)
    _check(dict(dI_hi=dI_hi), I_hi.dtype, dev)
    nbytes = gf_workspace_size(desc, 1)
    ws = _ws(nbytes, dev, ws)
    st = gf_backward(desc, _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.numel(), _ptr(dq),
                     _ptr(dI_lo), _ptr(dp_lo), _ptr(dI_hi), _ptr(deps), _ptr(ws), ws.numel(),
                     _stream(dev))
    if st != GF_OK:
        raise GFError(st)
    return dI_lo, dp_lo, dI_hi, deps


class GuidedFilterFn(torch.autograd.Function):
    """Differentiable guided filtering layer; the backward recomputes the
    low-res statistics from the saved inputs (nothing else is stored)."""

    @staticmethod
    def forward(ctx, I_lo, p_lo, I_hi, eps, r, mean_ab):
        e = _eps_tensor(eps, I_lo.shape[0], I_hi.device)
        ctx.save_for_backward(I_lo, p_lo, I_hi, e)
        ctx.r, ctx.mean_ab = r, mean_ab
        ctx.eps_is_tensor = isinstance(eps, torch.Tensor)
        return forward(I_lo, p_lo, I_hi, e, r, mean_ab)

    @staticmethod
    def backward(ctx, dq):
        I_lo, p_lo, I_hi, e = ctx.saved_tensors
        need = ctx.needs_input_grad
        dI_lo, dp_lo, dI_hi, deps = backward(
            I_lo, p_lo, I_hi, e, dq.contiguous(), ctx.r, ctx.mean_ab,
            need_dI_lo=need[0], need_dp_lo=need[1], need_dI_hi=need[2],
            need_deps=need[3] and ctx.eps_is_tensor)
        cast = lambda g, ref: None if g is None else g.to(ref.dtype)
        return cast(dI_lo, I_lo), cast(dp_lo, p_lo), dI_hi, deps, None, None


def guided_filter(I_lo, p_lo, I_hi, r=1, eps=1e-8, mean_ab=True):
    """Autograd entry point: q = GF(I_lo, p_lo, I_hi) with radius r and eps
    (a float, or a float32 tensor of 1 or n entries to get its gradient)."""
    return GuidedFilterFn.apply(I_lo, p_lo, I_hi, eps, r, mean_ab)
