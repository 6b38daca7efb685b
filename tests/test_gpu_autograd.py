"""GPU: the autograd.Function adjoints against the C-ABI calls, the FP64 oracle
gradient and the oracle's central finite differences on a 32^3 crop of the
512^3 pair."""
import numpy as np
import pytest
import torch
import torch.nn.functional as tf

import oracle
from paper_2509_25044_amd import autograd, ops, synth
from paper_2509_25044_amd.configs import C1, C3
from parity_util import assert_grad, assert_loss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _kink_free(u):
    f = torch.floor(u)
    return (f + 0.1 + 0.8 * (u - f)).contiguous()


@pytest.fixture(scope="module")
def crop32():
    """32^3 crop of the 512^3 pair where F varies most (blob structure)."""
    p = synth.make_pair(C3.pair, seed=2025, device=DEV)
    F, M, d = p["F"], p["M"], p["d"]
    var = tf.avg_pool3d((F * F)[None, None], 32, 32) - tf.avg_pool3d(F[None, None], 32, 32) ** 2
    k = int(torch.argmax(var.flatten()))
    n = 512 // 32
    z, y, x = (k // (n * n)) * 32, ((k // n) % n) * 32, (k % n) * 32
    sl = (slice(z, z + 32), slice(y, y + 32), slice(x, x + 32))
    Fc = F[sl].contiguous()
    Mc = M[sl].contiguous()
    uc = _kink_free(-d[(slice(None),) + sl])
    del p, F, M, d
    torch.cuda.empty_cache()
    return Fc, Mc, uc


def test_autograd_equals_direct_adjoint(crop32):
    F, M, u = crop32
    uu = u.clone().requires_grad_(True)
    loss = autograd.lncc_loss(F, M, uu, window=5)
    loss.backward()
    g, l2 = ops.warp_lncc_bwd(F, M, u, window=5)
    assert torch.equal(uu.grad, g)
    assert float(loss) == float(l2)


def test_autograd_lncc_against_oracle_fd_on_32cube_crop(crop32):
    print("[autograd lncc fd 32^3]", flush=True)
    F, M, u = crop32
    uu = u.clone().requires_grad_(True)
    loss = autograd.lncc_loss(F, M, uu, window=5)
    loss.backward()
    g = uu.grad.cpu().numpy()
    Fn, Mn, un = F.cpu().numpy(), M.cpu().numpy(), u.cpu().numpy()
    lr, gr = oracle.lncc(Fn, Mn, un, window=5, eps=1e-5)
    assert_loss(float(loss), lr, "crop loss")
    assert_grad(g, gr, "crop grad vs oracle")
    rng = np.random.default_rng(7)
    gmax = np.abs(gr).max()
    # finite differences of the FP64 oracle loss where the gradient is largest and at random points
    flat = np.argsort(np.abs(gr).ravel())[::-1][:12]
    pts = [np.unravel_index(i, gr.shape) for i in flat]
    pts += [tuple(int(v) for v in (rng.integers(0, 3), *rng.integers(0, 32, 3))) for _ in range(8)]
    for (c, z, y, x) in pts:
        up, um = un.copy(), un.copy()
        up[c, z, y, x] = np.float32(un[c, z, y, x] + np.float32(2e-3))
        um[c, z, y, x] = np.float32(un[c, z, y, x] - np.float32(2e-3))
        h = float(up[c, z, y, x]) - float(um[c, z, y, x])
        lp, _ = oracle.lncc(Fn, Mn, up, window=5, eps=1e-5, with_grad=False)
        lm, _ = oracle.lncc(Fn, Mn, um, window=5, eps=1e-5, with_grad=False)
        fd = (lp - lm) / h
        assert abs(g[c, z, y, x] - fd) <= 1e-4 * gmax + 1e-4 * abs(fd), ((c, z, y, x), g[c, z, y, x], fd)


def test_autograd_mi_against_oracle_and_fd(crop32):
    print("[autograd mi]", flush=True)
    F, M, u = crop32
    uu = u.clone().requires_grad_(True)
    loss = autograd.mi_loss(F, M, uu, bins=32)
    loss.backward()
    lr, _, gr = oracle.mi(F.cpu().numpy(), M.cpu().numpy(), u.cpu().numpy(), bins=32)
    assert_loss(float(loss), lr, "mi crop loss")
    assert_grad(uu.grad.cpu().numpy(), gr, "mi crop grad")


def test_upstream_scale_and_composition():
    p = synth.make_pair(C1.pair, seed=2025)
    F, M = p["F"].to(DEV), p["M"].to(DEV)
    u = (-0.5 * p["d"]).to(DEV).contiguous()
    uu = u.clone().requires_grad_(True)
    total = 2.0 * autograd.lncc_loss(F, M, uu) + 0.5 * autograd.mi_loss(F, M, uu)
    total.backward()
    gl, _ = ops.warp_lncc_bwd(F, M, u)
    _, st = ops.warp_mi_fwd(F, M, u)
    gm = ops.warp_mi_bwd(F, M, u, st)
    ref = (2.0 * gl.double() + 0.5 * gm.double()).cpu().numpy()
    assert_grad(uu.grad.cpu().numpy(), ref, "composition")


def test_images_are_not_differentiable():
    F = torch.rand(8, 8, 8, device=DEV, requires_grad=True)
    M = torch.rand(8, 8, 8, device=DEV)
    u = torch.zeros(3, 8, 8, 8, device=DEV, requires_grad=True)
    with pytest.raises(NotImplementedError):
        autograd.lncc_loss(F, M, u)
