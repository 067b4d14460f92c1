"""FP64 CPU oracle of the fast guided filtering layer (arXiv 1803.05619).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product path (``paper_1803_05619_amd``) never imports it, and this package
never imports the product path: the two share no code.

The arithmetic lives in ``gf_oracle.c`` (plain C, double precision,
brute-force window loops; see its header for the definition it follows,
Sec. III-B/C/D, Eq. (1)-(2) and Algorithm 1 of the paper).  This module
only builds it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_SRC_CONV = os.path.join(_HERE, "gf_conv_oracle.c")
_LIB = os.path.join(_HERE, "libgf_oracle.so")

GUIDE_MODES = {"identity": 0, "grey": 1, "transform": 2}

_lib = None


def build(force: bool = True) -> str:
    """Compile gf_oracle.c and gf_conv_oracle.c into libgf_oracle.so (gcc,
    -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-Wall", "-o", tmp, _SRC, _SRC_CONV, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Guide(ctypes.Structure):
    _fields_ = [
        ("hidden", ctypes.c_int),
        ("w1", ctypes.POINTER(ctypes.c_double)),
        ("w2", ctypes.POINTER(ctypes.c_double)),
        ("b2", ctypes.POINTER(ctypes.c_double)),
        ("lam", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("gamma", ctypes.POINTER(ctypes.c_double)),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("bn_eps", ctypes.c_double),
        ("slope", ctypes.c_double),
        ("flip_delta", ctypes.c_double),
    ]


class _Conv(ctypes.Structure):
    _fields_ = [
        ("hidden", ctypes.c_int),
        ("D", ctypes.POINTER(ctypes.c_double)),
        ("W1", ctypes.POINTER(ctypes.c_double)),
        ("W2", ctypes.POINTER(ctypes.c_double)),
        ("W3", ctypes.POINTER(ctypes.c_double)),
        ("slope", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ci = ctypes.c_int
        lib.gfo_forward.argtypes = [ci] * 11 + [ctypes.POINTER(_Guide), dp, dp, dp, dp, ci, dp]
        lib.gfo_forward.restype = ci
        lib.gfo_backward.argtypes = ([ci] * 11 + [ctypes.POINTER(_Guide), dp, dp, dp, dp, ci]
                                     + [dp] * 8)
        lib.gfo_backward.restype = ci
        lib.gfo_guide_apply.argtypes = [ci, ctypes.POINTER(_Guide), ci, ci, ci, ctypes.c_long, dp, dp]
        lib.gfo_guide_apply.restype = ci
        lib.gfo_guide_preact.argtypes = [ctypes.POINTER(_Guide), ci, ci, ctypes.c_long, dp, dp]
        lib.gfo_guide_preact.restype = ci
        lib.gfo_guide_grad_size.argtypes = [ci, ci, ci]
        lib.gfo_guide_grad_size.restype = ctypes.c_long
        lib.gfo_area_down.argtypes = [ci] * 6 + [dp, dp]
        lib.gfo_area_down.restype = ci
        lib.gfo_conv_param_count.argtypes = [ci, ci]
        lib.gfo_conv_param_count.restype = ctypes.c_long
        lib.gfo_conv_forward.argtypes = [ci] * 9 + [ctypes.POINTER(_Conv), dp, dp, dp, dp]
        lib.gfo_conv_forward.restype = ci
        lib.gfo_conv_backward.argtypes = ([ci] * 9 + [ctypes.POINTER(_Conv)] + [dp] * 9)
        lib.gfo_conv_backward.restype = ci
        lib.gfo_set_threads.argtypes = [ci]
        lib.gfo_set_threads.restype = None
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's following calls."""
    _load().gfo_set_threads(int(n))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _guide_struct(guide, keep):
    """Build the ctypes struct for a transform-guide parameter dict."""
    if guide is None:
        return None
    arrs = {k: _f64(guide[k]).ravel() for k in ("w1", "w2", "b2", "gamma", "beta")}
    keep.extend(arrs.values())
    hidden = int(np.asarray(guide["w1"]).shape[0])
    g = _Guide(hidden, _ptr(arrs["w1"]), _ptr(arrs["w2"]), _ptr(arrs["b2"]),
               float(guide["lam"]), float(guide["mu"]), _ptr(arrs["gamma"]),
               _ptr(arrs["beta"]), float(guide.get("bn_eps", 1e-5)),
               float(guide.get("slope", 0.2)), float(guide.get("flip_delta", 0.0)))
    return g


def _mode(guide_mode, guide):
    if guide_mode is None:
        guide_mode = "transform" if guide is not None else "identity"
    return GUIDE_MODES[guide_mode]


def _common(I_lo, p_lo, I_hi, eps):
    I_lo, p_lo, I_hi = _f64(I_lo), _f64(p_lo), _f64(I_hi)
    n, cin, h, w = I_lo.shape
    n2, c, h2, w2 = p_lo.shape
    n3, cin3, H, W = I_hi.shape
    if (n2, h2, w2) != (n, h, w) or (n3, cin3) != (n, cin):
        raise ValueError("inconsistent shapes")
    e = _f64(np.atleast_1d(eps)).ravel()
    if e.size not in (1, n):
        raise ValueError("eps must have 1 or n entries")
    return I_lo, p_lo, I_hi, e, (n, c, h, w, H, W, cin)


def forward(I_lo, p_lo, I_hi, r, eps, *, align_corners=False, mean_ab=True,
            guide=None, guide_mode=None):
    """q = GF(I_lo, p_lo, I_hi) in float64 (shape [n, c, H, W])."""
    lib = _load()
    I_lo, p_lo, I_hi, e, (n, c, h, w, H, W, cin) = _common(I_lo, p_lo, I_hi, eps)
    keep = []
    g = _guide_struct(guide, keep)
    q = np.empty((n, c, H, W), np.float64)
    rc = lib.gfo_forward(n, c, h, w, H, W, int(r), int(bool(align_corners)),
                         int(bool(mean_ab)), _mode(guide_mode, guide), cin,
                         ctypes.byref(g) if g is not None else None,
                         _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.size, _ptr(q))
    if rc != 0:
        raise RuntimeError(f"gfo_forward failed ({rc})")
    return q


def backward(I_lo, p_lo, I_hi, r, eps, dq, *, align_corners=False, mean_ab=True,
             guide=None, guide_mode=None):
    """Gradients of <q, dq> w.r.t. every input, in float64.

    Returns a dict with dI_lo, dp_lo, dI_hi, deps (one entry per eps entry),
    deps_abs (sum of the magnitudes of the terms of deps, an error scale)
    and, for the transform guide, dguide (flat, see guide_grad_split) and
    dguide_abs (per entry, the sum of the magnitudes of the per-pixel terms
    that entry adds up: the error scale of a sum, as deps_abs for deps).
    """
    lib = _load()
    I_lo, p_lo, I_hi, e, (n, c, h, w, H, W, cin) = _common(I_lo, p_lo, I_hi, eps)
    dq = _f64(dq)
    if dq.shape != (n, c, H, W):
        raise ValueError("dq shape")
    keep = []
    g = _guide_struct(guide, keep)
    mode = _mode(guide_mode, guide)
    dI_lo = np.empty_like(I_lo)
    dp_lo = np.empty_like(p_lo)
    dI_hi = np.empty_like(I_hi)
    deps = np.empty(e.size, np.float64)
    deps_abs = np.empty(e.size, np.float64)
    dguide = dguide_abs = None
    if mode == GUIDE_MODES["transform"]:
        dguide = np.zeros(lib.gfo_guide_grad_size(cin, c, g.hidden), np.float64)
        dguide_abs = np.zeros_like(dguide)
    rc = lib.gfo_backward(n, c, h, w, H, W, int(r), int(bool(align_corners)),
                          int(bool(mean_ab)), mode, cin,
                          ctypes.byref(g) if g is not None else None,
                          _ptr(I_lo), _ptr(p_lo), _ptr(I_hi), _ptr(e), e.size, _ptr(dq),
                          _ptr(dI_lo), _ptr(dp_lo), _ptr(dI_hi), _ptr(deps), _ptr(deps_abs),
                          _ptr(dguide), _ptr(dguide_abs))
    if rc != 0:
        raise RuntimeError(f"gfo_backward failed ({rc})")
    out = {"dI_lo": dI_lo, "dp_lo": dp_lo, "dI_hi": dI_hi, "deps": deps, "deps_abs": deps_abs}
    if dguide is not None:
        out["dguide"] = dguide
        out["dguide_abs"] = dguide_abs
    return out


def guide_apply(X, guide=None, guide_mode=None, cout=None):
    """G = F(X) for one call (X: [n, cin, H, W]); batch statistics of X."""
    lib = _load()
    X = _f64(X)
    n, cin, H, W = X.shape
    mode = _mode(guide_mode, guide)
    if cout is None:
        cout = np.asarray(guide["w2"]).shape[0] if guide is not None else cin
    keep = []
    g = _guide_struct(guide, keep)
    G = np.empty((n, cout, H, W), np.float64)
    rc = lib.gfo_guide_apply(mode, ctypes.byref(g) if g is not None else None,
                             n, cin, cout, H * W, _ptr(X), _ptr(G))
    if rc != 0:
        raise RuntimeError(f"gfo_guide_apply failed ({rc})")
    return G


def guide_preact(X, guide):
    """Pre-activations y = lam h + mu BN(h) of the transform guide for one
    call (X: [n, cin, H, W]; batch statistics of X): [n, hidden, H, W]."""
    lib = _load()
    X = _f64(X)
    n, cin, H, W = X.shape
    keep = []
    g = _guide_struct(guide, keep)
    Y = np.empty((n, g.hidden, H, W), np.float64)
    rc = lib.gfo_guide_preact(ctypes.byref(g), n, cin, H * W, _ptr(X), _ptr(Y))
    if rc != 0:
        raise RuntimeError(f"gfo_guide_preact failed ({rc})")
    return Y


def area_down(X, h, w):
    """Area downsampling [n, c, H, W] -> [n, c, h, w] in float64 (the
    downsampling step of the DGF framework, Sec. IV)."""
    lib = _load()
    X = _f64(X)
    n, c, H, W = X.shape
    Y = np.empty((n, c, int(h), int(w)), np.float64)
    rc = lib.gfo_area_down(n, c, H, W, int(h), int(w), _ptr(X), _ptr(Y))
    if rc != 0:
        raise RuntimeError(f"gfo_area_down failed ({rc})")
    return Y


def guide_grad_split(flat, cin, cout, hidden):
    """Split the flat guide gradient into named parts."""
    o = 0
    out = {}
    for name, size, shape in (("w1", hidden * cin, (hidden, cin)),
                              ("w2", cout * hidden, (cout, hidden)),
                              ("b2", cout, (cout,)), ("lam", 1, ()), ("mu", 1, ()),
                              ("gamma", hidden, (hidden,)), ("beta", hidden, (hidden,))):
        out[name] = np.asarray(flat[o:o + size]).reshape(shape)
        o += size
    return out


# ---------------------------------------------------------------- convolutional layer

CONV_GROUPS = ("D", "W1", "W2", "W3")


def conv_param_count(c, hidden):
    return int(_load().gfo_conv_param_count(int(c), int(hidden)))


def conv_split(flat, c, hidden):
    """Split a flat parameter (or gradient) vector D | W1 | W2 | W3."""
    K = int(hidden)
    out, o = {}, 0
    for name, shape in (("D", (c, 3, 3)), ("W1", (K, 2 * c)), ("W2", (K, K)), ("W3", (c, K))):
        size = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + size]).reshape(shape)
        o += size
    return out


def _conv_struct(params, keep):
    arrs = {k: _f64(params[k]).ravel() for k in CONV_GROUPS}
    keep.extend(arrs.values())
    return _Conv(int(np.asarray(params["W1"]).shape[0]), _ptr(arrs["D"]), _ptr(arrs["W1"]),
                 _ptr(arrs["W2"]), _ptr(arrs["W3"]), float(params.get("slope", 0.2)))


def conv_forward(I_lo, p_lo, I_hi, r, params, *, align_corners=False, mean_ab=True):
    """q of the convolutional guided filtering layer (Sec. III-E) in float64;
    params: D [c, 3, 3], W1 [K, 2c], W2 [K, K], W3 [c, K], slope."""
    lib = _load()
    I_lo, p_lo, I_hi = _f64(I_lo), _f64(p_lo), _f64(I_hi)
    n, c, h, w = p_lo.shape
    H, W = I_hi.shape[-2:]
    if I_lo.shape != p_lo.shape or I_hi.shape[:2] != (n, c):
        raise ValueError("inconsistent shapes")
    keep = []
    P = _conv_struct(params, keep)
    q = np.empty((n, c, H, W), np.float64)
    rc = lib.gfo_conv_forward(n, c, h, w, H, W, int(r), int(bool(align_corners)),
                              int(bool(mean_ab)), ctypes.byref(P), _ptr(I_lo), _ptr(p_lo),
                              _ptr(I_hi), _ptr(q))
    if rc != 0:
        raise RuntimeError(f"gfo_conv_forward failed ({rc})")
    return q


def conv_backward(I_lo, p_lo, I_hi, r, params, dq, *, align_corners=False, mean_ab=True):
    """Gradients of <q, dq>: dI_lo, dp_lo, dI_hi, dparams (flat D | W1 | W2 |
    W3) and dparams_abs (per entry, the sum of the magnitudes of the terms
    it adds up)."""
    lib = _load()
    I_lo, p_lo, I_hi, dq = _f64(I_lo), _f64(p_lo), _f64(I_hi), _f64(dq)
    n, c, h, w = p_lo.shape
    H, W = I_hi.shape[-2:]
    keep = []
    P = _conv_struct(params, keep)
    npar = conv_param_count(c, P.hidden)
    out = {"dI_lo": np.empty_like(I_lo), "dp_lo": np.empty_like(p_lo),
           "dI_hi": np.empty_like(I_hi), "dparams": np.empty(npar), "dparams_abs": np.empty(npar)}
    rc = lib.gfo_conv_backward(n, c, h, w, H, W, int(r), int(bool(align_corners)),
                               int(bool(mean_ab)), ctypes.byref(P), _ptr(I_lo), _ptr(p_lo),
                               _ptr(I_hi), _ptr(dq), _ptr(out["dI_lo"]), _ptr(out["dp_lo"]),
                               _ptr(out["dI_hi"]), _ptr(out["dparams"]),
                               _ptr(out["dparams_abs"]))
    if rc != 0:
        raise RuntimeError(f"gfo_conv_backward failed ({rc})")
    return out
