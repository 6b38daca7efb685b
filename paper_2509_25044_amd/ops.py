"""Torch-tensor front end of the C ABI, one function per entry point, same names.

Tensors must be float32, contiguous and on a HIP device; every call runs on
the current torch stream of that device.  Only argument marshalling happens
here: the computation is entirely in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import Affine, ConvGeom, Grid, LnccParams, MiParams, check

PAD = {"border": 0, "zeros": 1, 0: 0, 1: 1}

_ws_cache: dict = {}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _vol(t: torch.Tensor, name: str, ndim: int = 3):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device (got {t.device}); the library has no CPU path")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions (got shape {tuple(t.shape)})")
    return t


def _out(t: torch.Tensor, name: str, shape, device, dtype=torch.float32):
    """A caller-supplied output or operand: exact shape, dtype, contiguous, on `device`."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device} (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(int(s) for s in shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    return t


def _dev_scalar(t: Optional[torch.Tensor], name: str, device, dtype=torch.float32, n: int = 1):
    """A device scalar (or small array) the kernels read or write: dtype, device, at least n elements."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if t.numel() < n:
        raise ValueError(f"{name} must hold at least {n} elements (got {t.numel()})")
    return t


def _ws_bytes(ws: torch.Tensor, device) -> int:
    if not isinstance(ws, torch.Tensor) or ws.device != device or not ws.is_contiguous():
        raise ValueError(f"workspace must be a contiguous tensor on {device}")
    return ws.numel() * ws.element_size()


def make_grid(shape: Sequence[int], roi=None) -> Grid:
    """shape (D, H, W); roi ((z0,z1),(y0,y1),(x0,x1)) or None for the full array."""
    D, H, W = (int(s) for s in shape)
    g = Grid()
    g.D, g.H, g.W = D, H, W
    if roi is None:
        roi = ((0, D), (0, H), (0, W))
    for k in range(3):
        g.roi_lo[k] = int(roi[k][0])
        g.roi_hi[k] = int(roi[k][1])
    return g


def roi_voxels(shape, roi=None) -> int:
    if roi is None:
        return int(shape[0]) * int(shape[1]) * int(shape[2])
    return (roi[0][1] - roi[0][0]) * (roi[1][1] - roi[1][0]) * (roi[2][1] - roi[2][0])


def _workspace(nbytes: int, device, ws: Optional[torch.Tensor]) -> torch.Tensor:
    if ws is not None:
        _ws_bytes(ws, device)
        return ws
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = t
    return t


def _check_pair(F, M, u):
    _vol(F, "F")
    _vol(M, "M")
    if F.shape != M.shape:
        raise ValueError(f"F and M shapes differ: {tuple(F.shape)} vs {tuple(M.shape)}")
    if F.device != M.device:
        raise ValueError("F and M are on different devices")
    if u is not None:
        _vol(u, "u", 4)
        if tuple(u.shape) != (3,) + tuple(F.shape) or u.device != F.device:
            raise ValueError(f"u must be [3, D, H, W] on F's device (got {tuple(u.shape)})")


def lncc_params(window=5, eps=1e-5, ants=False, pad="border", check=False) -> LnccParams:
    """check: checked mode (the call scans its inputs, waits for the stream and raises FfdpError with code
    FFDP_ERR_NONFINITE on a NaN or infinite input or loss)."""
    p = LnccParams()
    p.window, p.eps, p.ants_approx, p.pad_mode = int(window), float(eps), int(bool(ants)), PAD[pad]
    p.check_finite = int(bool(check))
    return p


MI_ESTIMATORS = {"parzen": 0, "box": 1, "approx": 2}


def mi_params(bins=32, hard=False, pad="border", check=False) -> MiParams:
    """hard: False/"parzen" exact Parzen window, True/"box" box kernel (test
    mode), "approx" the approximate estimator (hard-bin counts convolved
    with the kernel; exact-kernel backward)."""
    p = MiParams()
    mode = MI_ESTIMATORS[hard] if isinstance(hard, str) else int(bool(hard))
    p.bins, p.hard_bins, p.pad_mode, p.check_finite = int(bins), mode, PAD[pad], int(bool(check))
    return p


def lncc_workspace_bytes(shape, roi=None, window=5) -> int:
    g = make_grid(shape, roi)
    return int(_lib.lib().ffdp_lncc_workspace_bytes(C.byref(g), C.byref(lncc_params(window))))


def mi_workspace_bytes(bins=32) -> int:
    g = make_grid((1, 1, 1))
    return int(_lib.lib().ffdp_mi_workspace_bytes(C.byref(g), C.byref(mi_params(bins))))


def mi_state_floats(bins=32) -> int:
    return int(_lib.lib().ffdp_mi_state_floats(int(bins)))


# ----------------------------------------------------------------------------
def warp(M: torch.Tensor, u: Optional[torch.Tensor] = None, pad="border", out=None) -> torch.Tensor:
    """M(x + u(x)) by trilinear sampling (ffdp_warp)."""
    _vol(M, "M")
    if u is not None:
        _out(u, "u", (3,) + tuple(M.shape), M.device)
    out = torch.empty_like(M) if out is None else _out(out, "out", M.shape, M.device)
    g = make_grid(M.shape)
    check("ffdp_warp", _lib.lib().ffdp_warp(_ptr(M), _ptr(u), C.byref(g), PAD[pad], _ptr(out), _stream(M)))
    return out


def resample(src: torch.Tensor, size: Sequence[int], value_scale: float = 1.0, out=None) -> torch.Tensor:
    """Corner-aligned trilinear resize of [C, D, H, W] or [D, H, W] (ffdp_resample)."""
    squeeze = src.dim() == 3
    s4 = src[None] if squeeze else src
    _vol(s4, "src", 4)
    Cn = s4.shape[0]
    dD, dH, dW = (int(v) for v in size)
    if out is None:
        o4 = torch.empty((Cn, dD, dH, dW), dtype=torch.float32, device=src.device)
    else:
        _out(out, "out", ((Cn,) if not squeeze else ()) + (dD, dH, dW), src.device)
        o4 = out.view(Cn, dD, dH, dW)
    check("ffdp_resample", _lib.lib().ffdp_resample(_ptr(s4), s4.shape[1], s4.shape[2], s4.shape[3], _ptr(o4),
                                                     dD, dH, dW, Cn, float(value_scale), _stream(src)))
    return o4[0] if squeeze else o4


def warp_lncc_fwd(F, M, u=None, window=5, eps=1e-5, pad="border", roi=None, loss=None, ws=None,
                  check_finite=False) -> torch.Tensor:
    """LNCC loss 1 - mean n_i of (F, M(x+u)) over the ROI -> float32 tensor [1] (ffdp_warp_lncc_fwd)."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = lncc_params(window, eps, False, pad, check_finite)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_lncc_workspace_bytes(C.byref(g), C.byref(p))), F.device, ws)
    loss = torch.empty(1, dtype=torch.float32, device=F.device) if loss is None else _dev_scalar(loss, "loss", F.device)
    check("ffdp_warp_lncc_fwd", L.ffdp_warp_lncc_fwd(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(p), _ptr(loss),
                                                      _ptr(ws), _ws_bytes(ws, ws.device), _stream(F)))
    return loss


def warp_lncc_bwd(F, M, u=None, window=5, eps=1e-5, ants=False, pad="border", roi=None, grad_scale=None,
                  grad_u=None, loss=None, want_loss=True, ws=None,
                  check_finite=False) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    """Fused LNCC forward + adjoint: (grad_u [3,D,H,W], loss [1] or None) (ffdp_warp_lncc_bwd)."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = lncc_params(window, eps, ants, pad, check_finite)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_lncc_workspace_bytes(C.byref(g), C.byref(p))), F.device, ws)
    if grad_u is None:
        grad_u = torch.empty((3,) + tuple(F.shape), dtype=torch.float32, device=F.device)
    else:
        _out(grad_u, "grad_u", (3,) + tuple(F.shape), F.device)
    if loss is None and want_loss:
        loss = torch.empty(1, dtype=torch.float32, device=F.device)
    _dev_scalar(loss, "loss", F.device)
    _dev_scalar(grad_scale, "grad_scale", F.device)
    check("ffdp_warp_lncc_bwd", L.ffdp_warp_lncc_bwd(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(p),
                                                      _ptr(grad_scale), _ptr(grad_u), _ptr(loss), _ptr(ws),
                                                      _ws_bytes(ws, ws.device), _stream(F)))
    return grad_u, loss


def warp_lncc_bwd_noalloc(F, M, u, grad_u, loss=None, window=5, eps=1e-5, ants=False, pad="border", roi=None,
                          grad_scale=None):
    """ffdp_warp_lncc_bwd with the library-owned scratch (ffdp_warp_lncc_bwd_noalloc): the caller passes every
    output (grad_u [3,D,H,W], loss [1] or None); nothing is allocated."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = lncc_params(window, eps, ants, pad)
    L = _lib.lib()
    _out(grad_u, "grad_u", (3,) + tuple(F.shape), F.device)
    _dev_scalar(loss, "loss", F.device)
    _dev_scalar(grad_scale, "grad_scale", F.device)
    check("ffdp_warp_lncc_bwd_noalloc",
          L.ffdp_warp_lncc_bwd_noalloc(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(p), _ptr(grad_scale),
                                       _ptr(grad_u), _ptr(loss), _stream(F)))
    return grad_u, loss


def warp_mi_fwd(F, M, u=None, bins=32, hard=False, pad="border", roi=None, state=None, loss=None, ws=None,
                check_finite=False):
    """Parzen MI: (loss = -MI [1], mi_state) (ffdp_warp_mi_fwd)."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = mi_params(bins, hard, pad, check_finite)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_mi_workspace_bytes(C.byref(g), C.byref(p))), F.device, ws)
    if state is None:
        state = torch.empty(int(L.ffdp_mi_state_floats(int(bins))), dtype=torch.float32, device=F.device)
    _dev_scalar(state, "state", F.device, n=int(L.ffdp_mi_state_floats(int(bins))))
    loss = torch.empty(1, dtype=torch.float32, device=F.device) if loss is None else _dev_scalar(loss, "loss", F.device)
    check("ffdp_warp_mi_fwd", L.ffdp_warp_mi_fwd(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(p), _ptr(loss),
                                                  _ptr(state), _ptr(ws), _ws_bytes(ws, ws.device), _stream(F)))
    return loss, state


def warp_mi_bwd(F, M, u, state, bins=32, hard=False, pad="border", roi=None, grad_scale=None, grad_u=None, ws=None,
                check_finite=False):
    """MI adjoint -> grad_u [3,D,H,W] (ffdp_warp_mi_bwd)."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = mi_params(bins, hard, pad, check_finite)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_mi_workspace_bytes(C.byref(g), C.byref(p))), F.device, ws)
    if grad_u is None:
        grad_u = torch.empty((3,) + tuple(F.shape), dtype=torch.float32, device=F.device)
    else:
        _out(grad_u, "grad_u", (3,) + tuple(F.shape), F.device)
    _dev_scalar(state, "state", F.device, n=int(L.ffdp_mi_state_floats(int(bins))))
    _dev_scalar(grad_scale, "grad_scale", F.device)
    check("ffdp_warp_mi_bwd", L.ffdp_warp_mi_bwd(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(p), _ptr(state),
                                                  _ptr(grad_scale), _ptr(grad_u), _ptr(ws), _ws_bytes(ws, ws.device), _stream(F)))
    return grad_u



# ------------------------------------------------- composite (affine) sampler --
def affine_params(A=None, t=None, S=None) -> Affine:
    """ffdp_affine from host values: A, S 3x3 (row-major, acting on (x, y, z)),
    t 3-vector, in voxel units; None means identity / zero."""
    def flat(v, n, default):
        if v is None:
            return default
        if isinstance(v, torch.Tensor):
            v = v.detach().cpu().double()
        v = [float(x) for x in np.asarray(v, dtype=np.float64).reshape(-1)]
        if len(v) != n:
            raise ValueError(f"expected {n} values, got {len(v)}")
        return v
    eye = [1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0]
    a = Affine()
    a.A[:] = flat(A, 9, eye)
    a.t[:] = flat(t, 3, [0.0, 0.0, 0.0])
    a.S[:] = flat(S, 9, eye)
    return a


def warp_affine(M, u=None, A=None, t=None, S=None, pad="border", out=None) -> torch.Tensor:
    """Composite sampler forward M(A X + t + S u(X)) (ffdp_warp_affine)."""
    _vol(M, "M")
    if u is not None:
        _out(u, "u", (3,) + tuple(M.shape), M.device)
    out = torch.empty_like(M) if out is None else _out(out, "out", M.shape, M.device)
    g = make_grid(M.shape)
    f = affine_params(A, t, S)
    check("ffdp_warp_affine", _lib.lib().ffdp_warp_affine(_ptr(M), _ptr(u), C.byref(g), C.byref(f), PAD[pad],
                                                           _ptr(out), _stream(M)))
    return out


def warp_affine_bwd(M, gout, u=None, A=None, t=None, S=None, pad="border", want_grad_u=True, grad_u=None, ws=None):
    """Composite sampler adjoint: (dL/du [3,D,H,W] or None, dL/dA [3,3], dL/dt [3]) as float64 device
    tensors for dL/dA, dL/dt (ffdp_warp_affine_bwd)."""
    _vol(M, "M")
    _out(gout, "gout", M.shape, M.device)
    if u is not None:
        _out(u, "u", (3,) + tuple(M.shape), M.device)
    g = make_grid(M.shape)
    f = affine_params(A, t, S)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_affine_workspace_bytes(C.byref(g))), M.device, ws)
    if want_grad_u and grad_u is None:
        grad_u = torch.empty((3,) + tuple(M.shape), dtype=torch.float32, device=M.device)
    elif want_grad_u:
        _out(grad_u, "grad_u", (3,) + tuple(M.shape), M.device)
    gAt = torch.empty(12, dtype=torch.float64, device=M.device)
    check("ffdp_warp_affine_bwd", L.ffdp_warp_affine_bwd(_ptr(M), _ptr(u), C.byref(g), C.byref(f), PAD[pad],
                                                          _ptr(gout), _ptr(grad_u if want_grad_u else None),
                                                          _ptr(gAt), _ptr(ws), _ws_bytes(ws, ws.device), _stream(M)))
    return (grad_u if want_grad_u else None), gAt[:9].view(3, 3), gAt[9:]


def warp_mi_affine_fwd(F, M, u=None, A=None, t=None, S=None, bins=32, hard=False, pad="border", roi=None,
                       state=None, loss=None, ws=None):
    """MI through the composite sampler: (loss = -MI [1], mi_state) (ffdp_warp_mi_affine_fwd)."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = mi_params(bins, hard, pad)
    f = affine_params(A, t, S)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_mi_workspace_bytes(C.byref(g), C.byref(p))), F.device, ws)
    if state is None:
        state = torch.empty(int(L.ffdp_mi_state_floats(int(bins))), dtype=torch.float32, device=F.device)
    _dev_scalar(state, "state", F.device, n=int(L.ffdp_mi_state_floats(int(bins))))
    loss = torch.empty(1, dtype=torch.float32, device=F.device) if loss is None else _dev_scalar(loss, "loss", F.device)
    check("ffdp_warp_mi_affine_fwd", L.ffdp_warp_mi_affine_fwd(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(f),
                                                                C.byref(p), _ptr(loss), _ptr(state), _ptr(ws),
                                                                _ws_bytes(ws, ws.device), _stream(F)))
    return loss, state


def warp_mi_affine_bwd(F, M, u, state, A=None, t=None, S=None, bins=32, hard=False, pad="border", roi=None,
                       grad_scale=None, want_grad_u=False, grad_u=None, ws=None):
    """MI adjoint through the composite sampler: (dL/du or None, dL/dA [3,3], dL/dt [3]) (float64 for
    the affine part) (ffdp_warp_mi_affine_bwd)."""
    _check_pair(F, M, u)
    g = make_grid(F.shape, roi)
    p = mi_params(bins, hard, pad)
    f = affine_params(A, t, S)
    L = _lib.lib()
    ws = _workspace(int(L.ffdp_affine_workspace_bytes(C.byref(g))), F.device, ws)
    if want_grad_u and grad_u is None:
        grad_u = torch.empty((3,) + tuple(F.shape), dtype=torch.float32, device=F.device)
    elif want_grad_u:
        _out(grad_u, "grad_u", (3,) + tuple(F.shape), F.device)
    _dev_scalar(state, "state", F.device, n=int(L.ffdp_mi_state_floats(int(bins))))
    _dev_scalar(grad_scale, "grad_scale", F.device)
    gAt = torch.empty(12, dtype=torch.float64, device=F.device)
    check("ffdp_warp_mi_affine_bwd", L.ffdp_warp_mi_affine_bwd(_ptr(F), _ptr(M), _ptr(u), C.byref(g), C.byref(f),
                                                                C.byref(p), _ptr(state), _ptr(grad_scale),
                                                                _ptr(grad_u if want_grad_u else None), _ptr(gAt),
                                                                _ptr(ws), _ws_bytes(ws, ws.device), _stream(F)))
    return (grad_u if want_grad_u else None), gAt[:9].view(3, 3), gAt[9:]

def adam_step(x, g, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
    """In-place Adam on x, m, v (ffdp_adam_step)."""
    for t, n in ((x, "x"), (g, "g"), (m, "m"), (v, "v")):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{n} must be a contiguous float32 device tensor")
        if t.numel() != x.numel() or t.device != x.device:
            raise ValueError("x, g, m, v must have the same number of elements and device")
    check("ffdp_adam_step", _lib.lib().ffdp_adam_step(_ptr(x), _ptr(g), _ptr(m), _ptr(v), x.numel(), float(lr),
                                                       float(beta1), float(beta2), float(eps), int(step),
                                                       _stream(x)))
    return x



def gaussian_smooth(src: torch.Tensor, sigma: float, out=None) -> torch.Tensor:
    """Separable Gaussian smoothing of [C, D, H, W] or [D, H, W], taps to
    radius ceil(3 sigma), edge replication (ffdp_gaussian_smooth)."""
    squeeze = src.dim() == 3
    s4 = src[None] if squeeze else src
    _vol(s4, "src", 4)
    o4 = torch.empty_like(s4) if out is None else _out(out, "out", src.shape, src.device).view(s4.shape)
    check("ffdp_gaussian_smooth", _lib.lib().ffdp_gaussian_smooth(_ptr(s4), _ptr(o4), s4.shape[1], s4.shape[2],
                                                                   s4.shape[3], s4.shape[0], float(sigma),
                                                                   _stream(src)))
    return o4[0] if squeeze else o4


def smooth_adam_step(x, g, m, v, sigma: float, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
    """In-place Adam on x, m, v with the gradient g smoothed first, bitwise
    gaussian_smooth then adam_step, the smoothed gradient never stored
    (ffdp_smooth_adam_step).  All [C, D, H, W] or [D, H, W]."""
    for t, n in ((x, "x"), (g, "g"), (m, "m"), (v, "v")):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{n} must be a contiguous float32 device tensor")
        if t.shape != x.shape or t.device != x.device:
            raise ValueError("x, g, m, v must have the same shape and device")
    shp = x.shape if x.dim() == 4 else (1,) + tuple(x.shape)
    if len(shp) != 4:
        raise ValueError("x must be [C, D, H, W] or [D, H, W]")
    check("ffdp_smooth_adam_step", _lib.lib().ffdp_smooth_adam_step(
        _ptr(x), _ptr(g), _ptr(m), _ptr(v), shp[1], shp[2], shp[3], shp[0], float(sigma), float(lr), float(beta1),
        float(beta2), float(eps), int(step), _stream(x)))
    return x

# ------------------------------------------------------------ U-Net kernels --
def _dev_t(t, name, dtype):
    if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")
    return t


def conv_geom(N, Di, Hi, Wi, Ca, Cb, Cout, stride=1, ups=False) -> ConvGeom:
    g = ConvGeom()
    g.N, g.Di, g.Hi, g.Wi, g.Ca, g.Cb, g.Cout, g.stride, g.ups = (int(N), int(Di), int(Hi), int(Wi), int(Ca),
                                                                  int(Cb), int(Cout), int(stride), int(bool(ups)))
    return g


def conv_out_shape(g: ConvGeom):
    s = g.stride
    return ((g.Di - 1) // s + 1, (g.Hi - 1) // s + 1, (g.Wi - 1) // s + 1)


def _conv_inputs(xa, xb, g: ConvGeom):
    """Channels-last bf16 inputs of a convolution: part a at half resolution
    when g.ups, part b (the skip) at full resolution when g.Cb > 0."""
    if not isinstance(xa, torch.Tensor) or xa.device.type != "cuda":
        raise ValueError("xa must be a device tensor")
    sa = (g.Di // 2, g.Hi // 2, g.Wi // 2) if g.ups else (g.Di, g.Hi, g.Wi)
    _out(xa, "xa", (g.N,) + sa + (g.Ca,), xa.device, torch.bfloat16)
    if g.Cb > 0:
        if xb is None:
            raise ValueError("xb is required when Cb > 0")
        _out(xb, "xb", (g.N, g.Di, g.Hi, g.Wi, g.Cb), xa.device, torch.bfloat16)
    return xa.device


def conv3d_fwd(xa, xb, w_bf16, bias, g: ConvGeom, act=True, slope=0.2, y_bf16=None, y_f32=None, want_bf16=True,
               want_f32=False):
    """3x3x3 BF16-MFMA convolution (ffdp_conv3d_fwd); bf16 tensors are torch.bfloat16."""
    dev = _conv_inputs(xa, xb, g)
    _out(w_bf16, "w_bf16", (g.Cout, 27, g.Ca + g.Cb), dev, torch.bfloat16)
    if bias is not None:
        _out(bias, "bias", (g.Cout,), dev)
    Do, Ho, Wo = conv_out_shape(g)
    shape = (g.N, Do, Ho, Wo, g.Cout)
    if want_bf16 and y_bf16 is None:
        y_bf16 = torch.empty(shape, dtype=torch.bfloat16, device=xa.device)
    elif y_bf16 is not None:
        _out(y_bf16, "y_bf16", shape, dev, torch.bfloat16)
    if want_f32 and y_f32 is None:
        y_f32 = torch.empty(shape, dtype=torch.float32, device=xa.device)
    elif y_f32 is not None:
        _out(y_f32, "y_f32", shape, dev)
    check("ffdp_conv3d_fwd", _lib.lib().ffdp_conv3d_fwd(_ptr(xa), _ptr(xb), _ptr(w_bf16), _ptr(bias), C.byref(g),
                                                        int(bool(act)), float(slope), _ptr(y_bf16), _ptr(y_f32),
                                                        _stream(xa)))
    return y_bf16 if y_f32 is None else (y_f32 if y_bf16 is None else (y_bf16, y_f32))


def conv3d_bwd_data(dy, y, wt_bf16, g: ConvGeom, slope=0.2, dx=None, accumulate=False):
    """Input gradient over the concatenated fine-resolution input (ffdp_conv3d_bwd_data)."""
    oshape = (g.N,) + conv_out_shape(g) + (g.Cout,)
    _out(dy, "dy", oshape, dy.device)
    if y is not None:
        _out(y, "y", oshape, dy.device, torch.bfloat16)
    _out(wt_bf16, "wt_bf16", (g.Ca + g.Cb, 27, g.Cout), dy.device, torch.bfloat16)
    if dx is None:
        dx = torch.empty((g.N, g.Di, g.Hi, g.Wi, g.Ca + g.Cb), dtype=torch.float32, device=dy.device)
    else:
        _out(dx, "dx", (g.N, g.Di, g.Hi, g.Wi, g.Ca + g.Cb), dy.device)
    check("ffdp_conv3d_bwd_data", _lib.lib().ffdp_conv3d_bwd_data(_ptr(dy), _ptr(y), float(slope), _ptr(wt_bf16),
                                                                  C.byref(g), _ptr(dx), int(bool(accumulate)),
                                                                  _stream(dy)))
    return dx


def conv3d_act_grad(dy, y, slope=0.2, p=None):
    """P = bf16(dy * act'(y)) in dy's layout (ffdp_conv3d_act_grad); y None: no activation."""
    _out(dy, "dy", tuple(dy.shape), dy.device)
    if y is not None:
        _out(y, "y", tuple(dy.shape), dy.device, torch.bfloat16)
    if p is None:
        p = torch.empty(tuple(dy.shape), dtype=torch.bfloat16, device=dy.device)
    else:
        _out(p, "p", tuple(dy.shape), dy.device, torch.bfloat16)
    check("ffdp_conv3d_act_grad", _lib.lib().ffdp_conv3d_act_grad(_ptr(dy), _ptr(y), float(slope), int(dy.numel()),
                                                                  _ptr(p), _stream(dy)))
    return p


def conv3d_bwd_data_bf16(p, wt_bf16, g: ConvGeom, dx=None, accumulate=False):
    """ffdp_conv3d_bwd_data from P (bf16 [N][Do][Ho][Wo][Cout], ffdp_conv3d_bwd_data_bf16)."""
    oshape = (g.N,) + conv_out_shape(g) + (g.Cout,)
    _out(p, "p", oshape, p.device, torch.bfloat16)
    _out(wt_bf16, "wt_bf16", (g.Ca + g.Cb, 27, g.Cout), p.device, torch.bfloat16)
    if dx is None:
        dx = torch.empty((g.N, g.Di, g.Hi, g.Wi, g.Ca + g.Cb), dtype=torch.float32, device=p.device)
    else:
        _out(dx, "dx", (g.N, g.Di, g.Hi, g.Wi, g.Ca + g.Cb), p.device)
    check("ffdp_conv3d_bwd_data_bf16", _lib.lib().ffdp_conv3d_bwd_data_bf16(_ptr(p), _ptr(wt_bf16), C.byref(g),
                                                                            _ptr(dx), int(bool(accumulate)),
                                                                            _stream(p)))
    return dx


def conv3d_bwd_weight(xa, xb, dy, y, g: ConvGeom, slope=0.2, dw=None, db=None, ws=None):
    """(dW [Cout][27][Cin], db [Cout]) fp32 (ffdp_conv3d_bwd_weight)."""
    L = _lib.lib()
    dev = _conv_inputs(xa, xb, g)
    oshape = (g.N,) + conv_out_shape(g) + (g.Cout,)
    _out(dy, "dy", oshape, dev)
    if y is not None:
        _out(y, "y", oshape, dev, torch.bfloat16)
    nb = int(L.ffdp_conv3d_bwd_weight_workspace_bytes(C.byref(g)))
    if ws is None or _ws_bytes(ws, dev) < nb:
        ws = torch.empty(max(nb, 16), dtype=torch.uint8, device=dy.device)
    if dw is None:
        dw = torch.empty((g.Cout, 27, g.Ca + g.Cb), dtype=torch.float32, device=dy.device)
    else:
        _out(dw, "dw", (g.Cout, 27, g.Ca + g.Cb), dev)
    if db is None:
        db = torch.empty(g.Cout, dtype=torch.float32, device=dy.device)
    else:
        _out(db, "db", (g.Cout,), dev)
    check("ffdp_conv3d_bwd_weight", L.ffdp_conv3d_bwd_weight(_ptr(xa), _ptr(xb), _ptr(dy), _ptr(y), float(slope),
                                                             C.byref(g), _ptr(dw), _ptr(db), _ptr(ws), _ws_bytes(ws, dev),
                                                             _stream(dy)))
    return dw, db


def conv3d_bwd_weight_bf16(xa, xb, p, g: ConvGeom, dw=None, db=None, ws=None):
    """ffdp_conv3d_bwd_weight from P (bf16 [N][Do][Ho][Wo][Cout], ffdp_conv3d_bwd_weight_bf16)."""
    L = _lib.lib()
    dev = _conv_inputs(xa, xb, g)
    _out(p, "p", (g.N,) + conv_out_shape(g) + (g.Cout,), dev, torch.bfloat16)
    nb = int(L.ffdp_conv3d_bwd_weight_workspace_bytes(C.byref(g)))
    if ws is None or _ws_bytes(ws, dev) < nb:
        ws = torch.empty(max(nb, 16), dtype=torch.uint8, device=dev)
    if dw is None:
        dw = torch.empty((g.Cout, 27, g.Ca + g.Cb), dtype=torch.float32, device=dev)
    else:
        _out(dw, "dw", (g.Cout, 27, g.Ca + g.Cb), dev)
    if db is None:
        db = torch.empty(g.Cout, dtype=torch.float32, device=dev)
    else:
        _out(db, "db", (g.Cout,), dev)
    check("ffdp_conv3d_bwd_weight_bf16", L.ffdp_conv3d_bwd_weight_bf16(_ptr(xa), _ptr(xb), _ptr(p), C.byref(g), _ptr(dw),
                                                                       _ptr(db), _ptr(ws), _ws_bytes(ws, dev),
                                                                       _stream(p)))
    return dw, db


def conv3d_bwd_weight_workspace_bytes(g: ConvGeom) -> int:
    return int(_lib.lib().ffdp_conv3d_bwd_weight_workspace_bytes(C.byref(g)))


def conv3d_weight_prep(w, w_bf16=None, wt_bf16=None):
    """fp32 [Cout][27][Cin] -> (bf16 copy, bf16 [Cin][27][Cout]) (ffdp_conv3d_weight_prep)."""
    if w.dim() != 3 or w.shape[1] != 27:
        raise ValueError(f"w must be [Cout, 27, Cin] (got {tuple(w.shape)})")
    Cout, _, Cin = w.shape
    _out(w, "w", w.shape, w.device)
    if w_bf16 is None:
        w_bf16 = torch.empty(w.shape, dtype=torch.bfloat16, device=w.device)
    else:
        _out(w_bf16, "w_bf16", w.shape, w.device, torch.bfloat16)
    if wt_bf16 is None:
        wt_bf16 = torch.empty((Cin, 27, Cout), dtype=torch.bfloat16, device=w.device)
    else:
        _out(wt_bf16, "wt_bf16", (Cin, 27, Cout), w.device, torch.bfloat16)
    check("ffdp_conv3d_weight_prep", _lib.lib().ffdp_conv3d_weight_prep(_ptr(w), Cout, Cin, _ptr(w_bf16),
                                                                        _ptr(wt_bf16), _stream(w)))
    return w_bf16, wt_bf16


def unet_pack_pair(F, M, out=None):
    """(F, M) fp32 [..] -> bf16 [.., 4] (ffdp_unet_pack_pair)."""
    _out(F, "F", F.shape, F.device)
    _out(M, "M", F.shape, F.device)
    n = F.numel()
    if out is None:
        out = torch.empty(tuple(F.shape) + (4,), dtype=torch.bfloat16, device=F.device)
    else:
        _out(out, "out", tuple(F.shape) + (4,), F.device, torch.bfloat16)
    check("ffdp_unet_pack_pair", _lib.lib().ffdp_unet_pack_pair(_ptr(F), _ptr(M), n, _ptr(out), _stream(F)))
    return out


def concat_grad_split(dxcat, g: ConvGeom, dxa=None, dxb=None, acc_a=False, acc_b=False):
    """Split the gradient of an upsampled+concatenated input (ffdp_concat_grad_split)."""
    dev = dxcat.device
    _out(dxcat, "dxcat", (g.N, g.Di, g.Hi, g.Wi, g.Ca + g.Cb), dev)
    if dxa is None:
        dxa = torch.empty((g.N, g.Di // 2, g.Hi // 2, g.Wi // 2, g.Ca), dtype=torch.float32, device=dev)
    else:
        _out(dxa, "dxa", (g.N, g.Di // 2, g.Hi // 2, g.Wi // 2, g.Ca), dev)
    if dxb is None and g.Cb > 0:
        dxb = torch.empty((g.N, g.Di, g.Hi, g.Wi, g.Cb), dtype=torch.float32, device=dev)
    elif dxb is not None:
        _out(dxb, "dxb", (g.N, g.Di, g.Hi, g.Wi, g.Cb), dev)
    check("ffdp_concat_grad_split", _lib.lib().ffdp_concat_grad_split(_ptr(dxcat), C.byref(g), _ptr(dxa), _ptr(dxb),
                                                                      int(bool(acc_a)), int(bool(acc_b)),
                                                                      _stream(dxcat)))
    return dxa, dxb


def mse_disp(pred, target, dpred=None, want_grad=True, loss=None, ws=None):
    """MSE of pred [N, ..., Cp] channels 0..2 against target [N, 3, ...] (ffdp_mse_disp)."""
    L = _lib.lib()
    if not isinstance(pred, torch.Tensor) or pred.dim() < 3:
        raise ValueError("pred must be [N, ..., Cp]")
    _out(pred, "pred", pred.shape, pred.device)
    N = pred.shape[0]
    Cp = pred.shape[-1]
    if Cp < 3:
        raise ValueError("pred needs at least 3 channels")
    nvox = pred.numel() // (N * Cp)
    _out(target, "target", (N, 3) + tuple(pred.shape[1:-1]), pred.device)
    if ws is None:
        ws = _workspace(int(L.ffdp_mse_workspace_bytes()), pred.device, None)
    else:
        _ws_bytes(ws, pred.device)
    if want_grad and dpred is None:
        dpred = torch.empty_like(pred)
    elif dpred is not None:
        _out(dpred, "dpred", pred.shape, pred.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=pred.device)
    _dev_scalar(loss, "loss", pred.device)
    check("ffdp_mse_disp", L.ffdp_mse_disp(_ptr(pred), Cp, _ptr(target), nvox, N, _ptr(dpred), _ptr(loss), _ptr(ws),
                                           _ws_bytes(ws, pred.device), _stream(pred)))
    return loss, dpred


def unpack_disp(pred, out=None):
    """pred [N, D, H, W, Cp] -> displacement [N, 3, D, H, W] (ffdp_unpack_disp)."""
    _out(pred, "pred", pred.shape, pred.device)
    N = pred.shape[0]
    Cp = pred.shape[-1]
    if Cp < 3:
        raise ValueError("pred needs at least 3 channels")
    nvox = pred.numel() // (N * Cp)
    if out is None:
        out = torch.empty((N, 3) + tuple(pred.shape[1:-1]), dtype=torch.float32, device=pred.device)
    else:
        _out(out, "out", (N, 3) + tuple(pred.shape[1:-1]), pred.device)
    check("ffdp_unpack_disp", _lib.lib().ffdp_unpack_disp(_ptr(pred), Cp, nvox, N, _ptr(out), _stream(pred)))
    return out
