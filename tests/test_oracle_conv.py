"""Pins of the oracle's 3x3x3 convolutions (O6) against torch.nn.functional.conv3d
in float64 and its autograd (library routes the oracle does not take)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as tf

import oracle


def _setup(seed, N, Di, Hi, Wi, Ca, Cb, Cout, ups):
    g = torch.Generator().manual_seed(seed)
    if ups:
        xa = torch.randn(N, Di // 2, Hi // 2, Wi // 2, Ca, generator=g, dtype=torch.float64)
    else:
        xa = torch.randn(N, Di, Hi, Wi, Ca, generator=g, dtype=torch.float64)
    xb = torch.randn(N, Di, Hi, Wi, Cb, generator=g, dtype=torch.float64) if Cb else None
    w = torch.randn(Cout, 27, Ca + Cb, generator=g, dtype=torch.float64) * 0.2
    b = torch.randn(Cout, generator=g, dtype=torch.float64)
    return xa, xb, w, b


def _lib_input(xa, xb, ups):
    a = xa
    if ups:
        a = xa.repeat_interleave(2, 1).repeat_interleave(2, 2).repeat_interleave(2, 3)
    X = a if xb is None else torch.cat([a, xb], dim=-1)
    return X.permute(0, 4, 1, 2, 3).contiguous()  # NCDHW


def _lib_weight(w):
    Cout, _, Cin = w.shape
    return w.reshape(Cout, 3, 3, 3, Cin).permute(0, 4, 1, 2, 3).contiguous()


CASES = [
    (1, 5, 6, 7, 4, 0, 4, 1, False),
    (2, 6, 4, 8, 8, 4, 12, 1, True),
    (1, 7, 6, 5, 4, 0, 8, 2, False),
    (2, 8, 6, 4, 12, 8, 4, 1, True),
]


@pytest.mark.parametrize("N,Di,Hi,Wi,Ca,Cb,Cout,s,ups", CASES)
@pytest.mark.parametrize("act", [False, True])
def test_forward_matches_torch_conv3d(N, Di, Hi, Wi, Ca, Cb, Cout, s, ups, act):
    xa, xb, w, b = _setup(1, N, Di, Hi, Wi, Ca, Cb, Cout, ups)
    y = oracle.conv3d_fwd(xa, xb, w, b, N, Di, Hi, Wi, Ca, Cb, Cout, stride=s, ups=ups, act=act, slope=0.2)
    ref = tf.conv3d(_lib_input(xa, xb, ups), _lib_weight(w), b, stride=s, padding=1)
    if act:
        ref = tf.leaky_relu(ref, 0.2)
    np.testing.assert_allclose(y, ref.permute(0, 2, 3, 4, 1).numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,Di,Hi,Wi,Ca,Cb,Cout,s,ups", CASES)
def test_backward_matches_torch_autograd(N, Di, Hi, Wi, Ca, Cb, Cout, s, ups):
    xa, xb, w, b = _setup(2, N, Di, Hi, Wi, Ca, Cb, Cout, ups)
    X = _lib_input(xa, xb, ups).requires_grad_(True)
    W = _lib_weight(w).requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    y = tf.conv3d(X, W, bb, stride=s, padding=1)
    P = torch.randn(y.shape, generator=torch.Generator().manual_seed(3), dtype=torch.float64)
    (y * P).sum().backward()
    Pcl = P.permute(0, 2, 3, 4, 1).contiguous()
    dx = oracle.conv3d_bwd_data(Pcl, w, N, Di, Hi, Wi, Ca, Cb, Cout, stride=s)
    np.testing.assert_allclose(dx, X.grad.permute(0, 2, 3, 4, 1).numpy(), rtol=1e-12, atol=1e-12)
    dw, db = oracle.conv3d_bwd_weight(xa, xb, Pcl, N, Di, Hi, Wi, Ca, Cb, Cout, stride=s, ups=ups)
    Cin = Ca + Cb
    np.testing.assert_allclose(dw, W.grad.permute(0, 2, 3, 4, 1).reshape(Cout, 27, Cin).numpy(), rtol=1e-11,
                               atol=1e-11)
    np.testing.assert_allclose(db, bb.grad.numpy(), rtol=1e-12, atol=1e-12)
