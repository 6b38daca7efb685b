"""Parity criteria between the HIP path and the FP64 oracle.

Loss:     |L_gpu - L_ref| <= 1e-5 |L_ref|, or <= 1e-8 when |L_ref| < 1e-3.
Gradient: ||g - g_ref||_2 / ||g_ref||_2 <= 1e-4 and max|g - g_ref| <= 1e-4 max|g_ref|.
Warp at integer shifts: bitwise.
"""
import numpy as np

LOSS_RTOL = 1e-5
LOSS_ATOL_SMALL = 1e-8
GRAD_RTOL = 1e-4


def assert_loss(l_gpu: float, l_ref: float, what: str = ""):
    tol = LOSS_RTOL * abs(l_ref) if abs(l_ref) >= 1e-3 else LOSS_ATOL_SMALL
    assert abs(l_gpu - l_ref) <= tol, f"{what}: loss {l_gpu!r} vs oracle {l_ref!r} (|diff| {abs(l_gpu - l_ref):.3e} > {tol:.3e})"


def grad_errors(g, g_ref):
    g = np.asarray(g, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    nref = np.linalg.norm(g_ref)
    mref = np.abs(g_ref).max()
    d = g - g_ref
    return (np.linalg.norm(d) / nref if nref > 0 else np.linalg.norm(d)), (np.abs(d).max() / mref if mref > 0 else np.abs(d).max())


def assert_grad(g, g_ref, what: str = ""):
    en, em = grad_errors(g, g_ref)
    assert np.all(np.isfinite(g)), f"{what}: non-finite gradient"
    assert en <= GRAD_RTOL and em <= GRAD_RTOL, f"{what}: gradient rel-norm err {en:.3e}, rel-max err {em:.3e}"
