"""ctypes binding of libffdp.so (argument marshalling only).

Every computation happens in the library's HIP kernels; this module only
turns torch tensors into device pointers, sizes and the current HIP stream.
It raises if the library has not been built — there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libffdp.so")

FFDP_OK = 0
FFDP_ERR_NONFINITE = 7
STATUS = {0: "ok", 1: "null pointer", 2: "bad shape or ROI", 3: "bad parameter", 4: "misaligned pointer",
          5: "workspace missing or too small", 6: "HIP runtime error", 7: "non-finite input or loss"}


class Grid(C.Structure):
    _fields_ = [("D", C.c_int64), ("H", C.c_int64), ("W", C.c_int64),
                ("roi_lo", C.c_int64 * 3), ("roi_hi", C.c_int64 * 3)]


class LnccParams(C.Structure):
    _fields_ = [("window", C.c_int32), ("eps", C.c_float), ("ants_approx", C.c_int32), ("pad_mode", C.c_int32),
                ("check_finite", C.c_int32)]


class MiParams(C.Structure):
    _fields_ = [("bins", C.c_int32), ("hard_bins", C.c_int32), ("pad_mode", C.c_int32), ("check_finite", C.c_int32)]


class Affine(C.Structure):
    _fields_ = [("A", C.c_float * 9), ("t", C.c_float * 3), ("S", C.c_float * 9)]


class ConvGeom(C.Structure):
    _fields_ = [("N", C.c_int32), ("Di", C.c_int32), ("Hi", C.c_int32), ("Wi", C.c_int32), ("Ca", C.c_int32),
                ("Cb", C.c_int32), ("Cout", C.c_int32), ("stride", C.c_int32), ("ups", C.c_int32)]


class FfdpError(RuntimeError):
    def __init__(self, fn: str, code: int, text: str):
        super().__init__(f"{fn} failed with status {code} ({STATUS.get(code, '?')}): {text}")
        self.code = code


_lib = None


def lib():
    """Load libffdp.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_25044_amd.build` "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    gp, lp, mp = C.POINTER(Grid), C.POINTER(LnccParams), C.POINTER(MiParams)
    cg = C.POINTER(ConvGeom)
    ap = C.POINTER(Affine)
    sig = {
        "ffdp_version": ([], C.c_int),
        "ffdp_status_string": ([C.c_int], C.c_char_p),
        "ffdp_last_error": ([], C.c_char_p),
        "ffdp_lncc_workspace_bytes": ([gp, lp], sz),
        "ffdp_mi_workspace_bytes": ([gp, mp], sz),
        "ffdp_mi_state_floats": ([i32], sz),
        "ffdp_warp": ([vp, vp, gp, i32, vp, vp], C.c_int),
        "ffdp_resample": ([vp, i64, i64, i64, vp, i64, i64, i64, i32, f32, vp], C.c_int),
        "ffdp_warp_lncc_fwd": ([vp, vp, vp, gp, lp, vp, vp, sz, vp], C.c_int),
        "ffdp_warp_lncc_bwd": ([vp, vp, vp, gp, lp, vp, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_warp_lncc_bwd_noalloc": ([vp, vp, vp, gp, lp, vp, vp, vp, vp], C.c_int),
        "ffdp_warp_mi_fwd": ([vp, vp, vp, gp, mp, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_warp_mi_bwd": ([vp, vp, vp, gp, mp, vp, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_affine_workspace_bytes": ([gp], sz),
        "ffdp_warp_affine": ([vp, vp, gp, ap, i32, vp, vp], C.c_int),
        "ffdp_warp_affine_bwd": ([vp, vp, gp, ap, i32, vp, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_warp_mi_affine_fwd": ([vp, vp, vp, gp, ap, mp, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_warp_mi_affine_bwd": ([vp, vp, vp, gp, ap, mp, vp, vp, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_adam_step": ([vp, vp, vp, vp, i64, f32, f32, f32, f32, i64, vp], C.c_int),
        "ffdp_gaussian_smooth": ([vp, vp, i64, i64, i64, i32, f32, vp], C.c_int),
        "ffdp_smooth_adam_step": ([vp, vp, vp, vp, i64, i64, i64, i32, f32, f32, f32, f32, f32, i64, vp], C.c_int),
        "ffdp_conv3d_fwd": ([vp, vp, vp, vp, cg, i32, f32, vp, vp, vp], C.c_int),
        "ffdp_conv3d_bwd_data": ([vp, vp, f32, vp, cg, vp, i32, vp], C.c_int),
        "ffdp_conv3d_act_grad": ([vp, vp, f32, i64, vp, vp], C.c_int),
        "ffdp_conv3d_bwd_weight_bf16": ([vp, vp, vp, cg, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_conv3d_bwd_data_bf16": ([vp, vp, cg, vp, i32, vp], C.c_int),
        "ffdp_conv3d_bwd_weight_workspace_bytes": ([cg], sz),
        "ffdp_conv3d_bwd_weight": ([vp, vp, vp, vp, f32, cg, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_conv3d_weight_prep": ([vp, i32, i32, vp, vp, vp], C.c_int),
        "ffdp_unet_pack_pair": ([vp, vp, i64, vp, vp], C.c_int),
        "ffdp_concat_grad_split": ([vp, cg, vp, vp, i32, i32, vp], C.c_int),
        "ffdp_mse_workspace_bytes": ([], sz),
        "ffdp_mse_disp": ([vp, i32, vp, i64, i32, vp, vp, vp, sz, vp], C.c_int),
        "ffdp_unpack_disp": ([vp, i32, i64, i32, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(fn: str, code: int):
    if code != FFDP_OK:
        raise FfdpError(fn, code, lib().ffdp_last_error().decode())


def header_functions():
    """Names of the entry points declared in include/ffdp.h."""
    import re
    hdr = os.path.join(os.path.dirname(PKG), "include", "ffdp.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"\b(ffdp_[a-z0-9_]+)\s*\(", txt)))
