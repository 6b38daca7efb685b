"""GPU parity of the composite implicit sampler M(A X + t + S u) and of MI
through it (the affine stage): values, the adjoint to u, A and t, and the
identity transform against the identity sampler, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_25044_amd import ops, synth
from paper_2509_25044_amd._lib import FfdpError
from parity_util import assert_grad, assert_loss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _about_centre(shape, R, shift):
    D, H, W = shape
    c = np.array([(W - 1) / 2, (H - 1) / 2, (D - 1) / 2])
    return R, c - R @ c + np.asarray(shift)


def _case(shape, seed):
    spec = synth.PairSpec(shape, (3.0, 6.0), 2.0)
    p = synth.make_pair(spec, seed=seed)
    return p["F"], p["M"], (-0.5 * p["d"]).contiguous()


# the transforms are rounded to fp32 first: both sides then use the same A, t, S
def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


CASES = [
    ("rotation+shift", (0.07, -0.05, 0.11), 1.03, (0.37, -0.61, 0.29), np.diag([1.0, 1.0, 1.0])),
    ("shear+scaled u", (0.0, 0.0, 0.0), 0.97, (-0.23, 0.41, 0.17), np.array([[0.8, 0.1, 0.0], [0.0, 1.2, -0.05], [0.02, 0.0, 0.9]])),
]


@pytest.mark.parametrize("name,angles,scale,shift,S", CASES)
@pytest.mark.parametrize("pad", ["border", "zeros"])
def test_warp_affine_forward_and_adjoint(name, angles, scale, shift, S, pad):
    print(f"[affine warp {name} pad={pad}]", flush=True)
    shape = (21, 26, 33)
    F, M, u = _case(shape, 31)
    A, t = _about_centre(shape, scale * _rot(*angles), shift)
    A, t, S = _f32(A), _f32(t), _f32(S)
    pm = 0 if pad == "border" else 1
    Md, ud = M.to(DEV), u.to(DEV)
    out = ops.warp_affine(Md, ud, A=A, t=t, S=S, pad=pad).cpu().numpy()
    ref = oracle.warp_affine(M.numpy(), u.numpy(), A=A, t=t, S=S, pad=pm)
    assert np.abs(out - ref).max() <= 1e-5 * np.abs(ref).max(), np.abs(out - ref).max()
    rng = np.random.default_rng(7)
    gout = rng.normal(0, 1, shape).astype(np.float32)
    gu, gA, gt = ops.warp_affine_bwd(Md, torch.from_numpy(gout).to(DEV), ud, A=A, t=t, S=S, pad=pad)
    rgu, rgA, rgt = oracle.warp_affine_bwd(M.numpy(), gout.astype(np.float64), u.numpy(), A=A, t=t, S=S, pad=pm)
    assert_grad(gu.cpu().numpy(), rgu, f"{name} grad_u")
    sc = max(np.abs(rgA).max(), 1e-30)
    assert np.abs(gA.cpu().numpy() - rgA).max() <= 1e-4 * sc, (gA.cpu().numpy(), rgA)
    sc = max(np.abs(rgt).max(), 1e-30)
    assert np.abs(gt.cpu().numpy() - rgt).max() <= 1e-4 * sc, (gt.cpu().numpy(), rgt)


def test_identity_transform_is_the_identity_sampler():
    print("[affine identity]", flush=True)
    F, M, u = _case((17, 19, 40), 32)
    Md, ud = M.to(DEV), u.to(DEV)
    assert torch.equal(ops.warp_affine(Md, ud), ops.warp(Md, ud))
    l0, s0 = ops.warp_mi_fwd(F.to(DEV), Md, ud, bins=32)
    l1, s1 = ops.warp_mi_affine_fwd(F.to(DEV), Md, ud, bins=32)
    assert torch.equal(l0, l1) and torch.equal(s0, s1)
    g0 = ops.warp_mi_bwd(F.to(DEV), Md, ud, s0, bins=32)
    g1, gA, gt = ops.warp_mi_affine_bwd(F.to(DEV), Md, ud, s1, bins=32, want_grad_u=True)
    assert torch.equal(g0, g1)
    # with S = I, dL/dt is the sum of dL/du over the volume
    ref = g0.double().reshape(3, -1).sum(1)
    assert float((gt - ref).abs().max()) <= 1e-6 * float(ref.abs().max()) + 1e-12


@pytest.mark.parametrize("hard", [False, "approx"])
def test_mi_through_the_composite_sampler(hard):
    print(f"[affine mi hard={hard}]", flush=True)
    shape = (24, 28, 36)
    F, M, u = _case(shape, 33)
    A, t = _about_centre(shape, 1.02 * _rot(0.05, 0.04, -0.06), (0.31, -0.27, 0.45))
    A, t, S = _f32(A), _f32(t), _f32(np.diag([0.9, 1.1, 1.0]))
    mode = 2 if hard == "approx" else 0
    Fd, Md, ud = F.to(DEV), M.to(DEV), u.to(DEV)
    loss, st = ops.warp_mi_affine_fwd(Fd, Md, ud, A=A, t=t, S=S, bins=32, hard=hard)
    gu, gA, gt = ops.warp_mi_affine_bwd(Fd, Md, ud, st, A=A, t=t, S=S, bins=32, hard=hard, want_grad_u=True)
    rl, rp, rgu, rgA, rgt = oracle.mi_affine(F.numpy(), M.numpy(), u.numpy(), A=A, t=t, S=S, bins=32, hard=mode)
    assert_loss(float(loss.item()), rl, "affine mi loss")
    atol = 1e-9 if mode == 0 else 4.0 / F.numel()
    np.testing.assert_allclose(st[1024:2048].cpu().numpy().reshape(32, 32), rp, rtol=1e-5, atol=atol)
    assert_grad(gu.cpu().numpy(), rgu, "affine mi grad_u")
    assert np.abs(gA.cpu().numpy() - rgA).max() <= 1e-4 * np.abs(rgA).max()
    assert np.abs(gt.cpu().numpy() - rgt).max() <= 1e-4 * np.abs(rgt).max()
    _, gA2, gt2 = ops.warp_mi_affine_bwd(Fd, Md, ud, st, A=A, t=t, S=S, bins=32, hard=hard)
    assert torch.equal(gA, gA2) and torch.equal(gt, gt2)  # without grad_u, bitwise the same sums


def test_validation():
    print("[affine validation]", flush=True)
    M = torch.zeros((4, 5, 6), device=DEV)
    with pytest.raises(FfdpError):
        ops.warp_affine(M, A=[[float("nan"), 0, 0], [0, 1, 0], [0, 0, 1]])
    with pytest.raises(FfdpError):
        ops.warp_affine(M, out=M)
