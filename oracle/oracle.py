"""ctypes front end of the FP64 C oracle (test infrastructure only).

All arguments are numpy arrays (float32 inputs, float64 outputs) or torch CPU
tensors, converted here; results come back as float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = C.c_int64


def load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "libffdp_oracle.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.orc_warp.argtypes = [vp, vp, _i64, _i64, _i64, C.c_int, vp, vp]
    lib.orc_lncc_loss.argtypes = [vp, vp, _i64, _i64, _i64, vp, C.c_int, C.c_double]
    lib.orc_lncc_loss.restype = C.c_double
    lib.orc_lncc.argtypes = [vp, vp, vp, _i64, _i64, _i64, vp, C.c_int, C.c_double, C.c_int, C.c_int, vp, vp]
    lib.orc_lncc_grad_u_at.argtypes = [vp, vp, vp, _i64, _i64, _i64, vp, C.c_int, C.c_double, C.c_int, C.c_int,
                                       vp, _i64, vp]
    lib.orc_mi.argtypes = [vp, vp, vp, _i64, _i64, _i64, vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
    lib.orc_parzen.argtypes = [C.c_double, C.c_int, C.c_int, vp, vp]
    lib.orc_mi_pmf.argtypes = [vp, vp, vp, _i64, _i64, _i64, vp, C.c_int, C.c_int, C.c_int, vp, C.c_double, vp]
    lib.orc_mi_grad_u_at.argtypes = [vp, vp, vp, _i64, _i64, _i64, vp, C.c_int, C.c_int, C.c_int, vp, _i64, vp, vp]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_max_threads.argtypes = []
    lib.orc_adam.argtypes = [vp, vp, vp, vp, _i64, C.c_double, C.c_double, C.c_double, C.c_double, _i64]
    lib.orc_resample.argtypes = [vp, _i64, _i64, _i64, vp, _i64, _i64, _i64, C.c_int, C.c_double]
    lib.orc_gaussian_smooth.argtypes = [vp, _i64, _i64, _i64, C.c_int, C.c_double, vp]
    lib.orc_warp_affine.argtypes = [vp, vp, _i64, _i64, _i64, vp, vp, vp, C.c_int, vp, vp]
    lib.orc_warp_affine_bwd.argtypes = [vp, vp, _i64, _i64, _i64, vp, vp, vp, C.c_int, vp, vp, vp]
    lib.orc_mi_affine.argtypes = [vp, vp, vp, _i64, _i64, _i64, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, vp,
                                  vp, vp]
    lib.orc_conv3d_fwd.argtypes = [vp, vp, vp, vp] + [_i64] * 9 + [C.c_int, C.c_double, vp]
    lib.orc_conv3d_bwd_data.argtypes = [vp, vp] + [_i64] * 8 + [vp]
    lib.orc_conv3d_bwd_weight.argtypes = [vp, vp, vp] + [_i64] * 9 + [vp, vp]
    for f in ("orc_warp", "orc_lncc", "orc_lncc_grad_u_at", "orc_mi", "orc_mi_pmf", "orc_mi_grad_u_at", "orc_parzen", "orc_adam", "orc_resample",
              "orc_gaussian_smooth", "orc_warp_affine", "orc_warp_affine_bwd", "orc_mi_affine", "orc_conv3d_fwd", "orc_conv3d_bwd_data", "orc_conv3d_bwd_weight"):
        getattr(lib, f).restype = C.c_int
    _LIB = lib
    return lib


def _f32(a):
    if a is None:
        return None
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _roi(roi):
    if roi is None:
        return None
    r = np.asarray(roi, dtype=np.int64).reshape(-1)
    assert r.size == 6
    return np.ascontiguousarray(r)


def warp(M, u=None, pad: int = 0, with_grad: bool = False):
    """Mw = M(x + u) in float64 (and dMw/dp [3][D][H][W] if with_grad)."""
    lib = load()
    M = _f32(M)
    u = _f32(u)
    D, H, W = M.shape
    out = np.empty((D, H, W), np.float64)
    dout = np.empty((3, D, H, W), np.float64) if with_grad else None
    lib.orc_warp(_ptr(M), _ptr(u), D, H, W, pad, _ptr(out), _ptr(dout))
    return (out, dout) if with_grad else out


def lncc_loss_mw(F, Mw, roi=None, window: int = 5, eps: float = 1e-5) -> float:
    """LNCC loss of F against an already warped (float64) moving image."""
    lib = load()
    F = _f32(F)
    Mw = np.ascontiguousarray(Mw, dtype=np.float64)
    D, H, W = F.shape
    r = _roi(roi)
    return float(lib.orc_lncc_loss(_ptr(F), _ptr(Mw), D, H, W, _ptr(r), window, eps))


def lncc(F, M, u=None, roi=None, window: int = 5, eps: float = 1e-5, ants: bool = False, pad: int = 0,
         with_grad: bool = True):
    """(loss, dloss/du [3][D][H][W] or None)."""
    lib = load()
    F, M, u = _f32(F), _f32(M), _f32(u)
    D, H, W = F.shape
    r = _roi(roi)
    loss = np.zeros(1, np.float64)
    g = np.empty((3, D, H, W), np.float64) if with_grad else None
    lib.orc_lncc(_ptr(F), _ptr(M), _ptr(u), D, H, W, _ptr(r), window, eps, int(ants), pad, _ptr(loss), _ptr(g))
    return float(loss[0]), g


def lncc_grad_u_at(F, M, u, idx, roi=None, window: int = 5, eps: float = 1e-5, ants: bool = False, pad: int = 0):
    """dloss/du at the voxels idx [n,3] (z,y,x) -> [n,3] (d/du_x, d/du_y, d/du_z)."""
    lib = load()
    F, M, u = _f32(F), _f32(M), _f32(u)
    D, H, W = F.shape
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1, 3))
    out = np.empty((idx.shape[0], 3), np.float64)
    r = _roi(roi)
    lib.orc_lncc_grad_u_at(_ptr(F), _ptr(M), _ptr(u), D, H, W, _ptr(r), window, eps, int(ants), pad,
                           _ptr(idx), idx.shape[0], _ptr(out))
    return out


def mi(F, M, u=None, roi=None, bins: int = 32, hard: int = 0, pad: int = 0, with_grad: bool = True):
    """(loss = -MI, joint PMF p[B][B], dloss/du or None).  hard: 0 exact
    Parzen, 1 box kernel, 2 the approximate estimator (hard-bin counts
    convolved with the kernel)."""
    lib = load()
    F, M, u = _f32(F), _f32(M), _f32(u)
    D, H, W = F.shape
    r = _roi(roi)
    loss = np.zeros(1, np.float64)
    p = np.empty((bins, bins), np.float64)
    g = np.empty((3, D, H, W), np.float64) if with_grad else None
    lib.orc_mi(_ptr(F), _ptr(M), _ptr(u), D, H, W, _ptr(r), bins, int(hard), pad, _ptr(loss), _ptr(p), _ptr(g))
    return float(loss[0]), p, g


def mi_pmf(F, M, u=None, roi=None, bins: int = 32, hard: int = 0, pad: int = 0, edge_tol: float = 0.0,
           with_edges: bool = False):
    """Joint PMF p[B][B] of (F, M(x+u)) over the ROI, sampled on the fly (for
    volumes too large for mi()); the same estimator as mi().  with_edges:
    also return the number of ROI voxels whose clamped warped value lies
    within edge_tol of an interior bin edge."""
    lib = load()
    F, M, u = _f32(F), _f32(M), _f32(u)
    D, H, W = F.shape
    p = np.empty((bins, bins), np.float64)
    ne = np.zeros(1, np.int64)
    lib.orc_mi_pmf(_ptr(F), _ptr(M), _ptr(u), D, H, W, _ptr(_roi(roi)), bins, int(hard), pad, _ptr(p),
                   float(edge_tol), _ptr(ne))
    return (p, int(ne[0])) if with_edges else p


def mi_grad_u_at(F, M, u, points, p, roi=None, bins: int = 32, hard: int = 0, pad: int = 0):
    """dloss/du [npts][3] at voxels points [npts][3] (z, y, x) for the PMF p
    of the same inputs (from mi_pmf or mi)."""
    lib = load()
    F, M, u = _f32(F), _f32(M), _f32(u)
    D, H, W = F.shape
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int64).reshape(-1, 3))
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(bins, bins))
    out = np.empty((pts.shape[0], 3), np.float64)
    lib.orc_mi_grad_u_at(_ptr(F), _ptr(M), _ptr(u), D, H, W, _ptr(_roi(roi)), bins, int(hard), pad, _ptr(p),
                         pts.shape[0], _ptr(pts), _ptr(out))
    return out


def parzen(v: float, bins: int, hard: bool = False):
    lib = load()
    k = np.empty(bins, np.float64)
    o = np.empty(bins, np.float64)
    lib.orc_parzen(float(v), bins, int(hard), _ptr(k), _ptr(o))
    return k, o


def adam(x, g, m, v, lr, b1=0.9, b2=0.999, eps=1e-8, step=1):
    """In-place float64 Adam step on numpy float64 arrays."""
    lib = load()
    for a in (x, g, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib.orc_adam(_ptr(x), _ptr(g), _ptr(m), _ptr(v), x.size, lr, b1, b2, eps, step)
    return x, m, v


def resample(src, dst_shape: Sequence[int], value_scale: float = 1.0):
    """src [C][D][H][W] or [D][H][W] float32 -> float64 of dst_shape (same channel count)."""
    lib = load()
    src = _f32(src)
    squeeze = src.ndim == 3
    if squeeze:
        src = src[None]
    Cn, sD, sH, sW = src.shape
    dD, dH, dW = dst_shape
    out = np.empty((Cn, dD, dH, dW), np.float64)
    lib.orc_resample(_ptr(src), sD, sH, sW, _ptr(out), dD, dH, dW, Cn, value_scale)
    return out[0] if squeeze else out



def gaussian_smooth(src, sigma: float):
    """src [C][D][H][W] or [D][H][W] float32 -> float64 Gaussian-smoothed field
    (direct (2R+1)^3 sum, R = ceil(3 sigma), edge replication)."""
    lib = load()
    src = _f32(src)
    squeeze = src.ndim == 3
    if squeeze:
        src = src[None]
    Cn, D, H, W = src.shape
    out = np.empty((Cn, D, H, W), np.float64)
    if lib.orc_gaussian_smooth(_ptr(src), D, H, W, Cn, float(sigma), _ptr(out)) != 0:
        raise ValueError("sigma must be > 0")
    return out[0] if squeeze else out


def _affine3(A, t, S):
    A = np.ascontiguousarray(np.eye(3) if A is None else A, dtype=np.float64).reshape(9)
    t = np.ascontiguousarray(np.zeros(3) if t is None else t, dtype=np.float64).reshape(3)
    S = np.ascontiguousarray(np.eye(3) if S is None else S, dtype=np.float64).reshape(9)
    return A, t, S


def warp_affine(M, u=None, A=None, t=None, S=None, pad: int = 0, with_grad: bool = False):
    """M(A X + t + S u(X)), X = (x, y, z) voxel coordinates -> float64 [D][H][W]
    (and dM/dp [3][D][H][W] at the sample points if with_grad)."""
    lib = load()
    M, u = _f32(M), _f32(u)
    D, H, W = M.shape
    A, t, S = _affine3(A, t, S)
    out = np.empty((D, H, W), np.float64)
    d = np.empty((3, D, H, W), np.float64) if with_grad else None
    lib.orc_warp_affine(_ptr(M), _ptr(u), D, H, W, _ptr(A), _ptr(t), _ptr(S), pad, _ptr(out), _ptr(d))
    return (out, d) if with_grad else out


def warp_affine_bwd(M, gout, u=None, A=None, t=None, S=None, pad: int = 0):
    """(dL/du [3][D][H][W], dL/dA [3][3], dL/dt [3]) for the upstream gradient gout [D][H][W]."""
    lib = load()
    M, u = _f32(M), _f32(u)
    D, H, W = M.shape
    A, t, S = _affine3(A, t, S)
    gout = np.ascontiguousarray(gout, dtype=np.float64)
    gu = np.empty((3, D, H, W), np.float64)
    gAt = np.empty(12, np.float64)
    lib.orc_warp_affine_bwd(_ptr(M), _ptr(u), D, H, W, _ptr(A), _ptr(t), _ptr(S), pad, _ptr(gout), _ptr(gu),
                            _ptr(gAt))
    return gu, gAt[:9].reshape(3, 3), gAt[9:]


def mi_affine(F, M, u=None, A=None, t=None, S=None, roi=None, bins: int = 32, hard: int = 0, pad: int = 0):
    """MI of (F, M(A X + t + S u)): (loss, p, dL/du, dL/dA [3][3], dL/dt [3])."""
    lib = load()
    F, M, u = _f32(F), _f32(M), _f32(u)
    D, H, W = F.shape
    A, t, S = _affine3(A, t, S)
    r = _roi(roi)
    loss = np.zeros(1, np.float64)
    p = np.empty((bins, bins), np.float64)
    gu = np.empty((3, D, H, W), np.float64)
    gAt = np.empty(12, np.float64)
    lib.orc_mi_affine(_ptr(F), _ptr(M), _ptr(u), D, H, W, _ptr(r), _ptr(A), _ptr(t), _ptr(S), bins, int(hard), pad,
                      _ptr(loss), _ptr(p), _ptr(gu), _ptr(gAt))
    return float(loss[0]), p, gu, gAt[:9].reshape(3, 3), gAt[9:]

def _f64(a):
    if a is None:
        return None
    if hasattr(a, "detach"):
        a = a.detach().cpu().double().numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def conv3d_fwd(xa, xb, w, bias, N, Di, Hi, Wi, Ca, Cb, Cout, stride=1, ups=False, act=False, slope=0.2):
    """Direct 3x3x3 convolution (channels-last) -> float64 [N][Do][Ho][Wo][Cout]."""
    lib = load()
    xa, xb, w, bias = _f64(xa), _f64(xb), _f64(w), _f64(bias)
    Do, Ho, Wo = (Di - 1) // stride + 1, (Hi - 1) // stride + 1, (Wi - 1) // stride + 1
    y = np.empty((N, Do, Ho, Wo, Cout), np.float64)
    lib.orc_conv3d_fwd(_ptr(xa), _ptr(xb), _ptr(w), _ptr(bias), N, Di, Hi, Wi, Ca, Cb, Cout, stride, int(ups),
                       int(act), slope, _ptr(y))
    return y


def conv3d_bwd_data(P, w, N, Di, Hi, Wi, Ca, Cb, Cout, stride=1):
    """Adjoint w.r.t. the (concatenated, fine-resolution) input -> [N][Di][Hi][Wi][Ca+Cb]."""
    lib = load()
    P, w = _f64(P), _f64(w)
    dx = np.empty((N, Di, Hi, Wi, Ca + Cb), np.float64)
    lib.orc_conv3d_bwd_data(_ptr(P), _ptr(w), N, Di, Hi, Wi, Ca, Cb, Cout, stride, _ptr(dx))
    return dx


def conv3d_bwd_weight(xa, xb, P, N, Di, Hi, Wi, Ca, Cb, Cout, stride=1, ups=False):
    """(dW [Cout][27][Cin], db [Cout]) in float64."""
    lib = load()
    xa, xb, P = _f64(xa), _f64(xb), _f64(P)
    dw = np.empty((Cout, 27, Ca + Cb), np.float64)
    db = np.empty(Cout, np.float64)
    lib.orc_conv3d_bwd_weight(_ptr(xa), _ptr(xb), _ptr(P), N, Di, Hi, Wi, Ca, Cb, Cout, stride, int(ups),
                              _ptr(dw), _ptr(db))
    return dw, db


def set_threads(n: int) -> None:
    """Width of the oracle's OpenMP loops (for timing)."""
    if load().orc_set_threads(int(n)) != 0:
        raise ValueError("threads must be >= 1")


def max_threads() -> int:
    return int(load().orc_max_threads())
