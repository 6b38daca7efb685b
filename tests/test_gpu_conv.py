"""GPU parity of the BF16-MFMA convolution kernels and the U-Net helper kernels
against the FP64 oracle on the same bf16 operands."""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_25044_amd import ops
from parity_util import assert_grad

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SLOPE = 0.2

CASES = [
    (2, 6, 7, 9, 4, 0, 16, 1, False),
    (1, 8, 6, 10, 16, 0, 32, 2, False),
    (1, 6, 8, 4, 64, 0, 128, 2, False),
    (2, 8, 6, 4, 128, 64, 64, 1, True),
    (1, 4, 6, 8, 32, 16, 16, 1, True),
    (2, 5, 7, 6, 16, 0, 4, 1, False),
    (1, 7, 5, 9, 8, 4, 8, 2, False),
    # rows longer than one 32-voxel segment, ragged tails, two channel chunks
    (1, 4, 6, 70, 32, 16, 16, 1, True),
    (1, 4, 4, 40, 64, 32, 32, 1, True),
    (2, 3, 5, 45, 16, 0, 4, 1, False),
    # voxel-chunk weight gradients: stride 2 with two input-channel tiles, and
    # stride 1 with more than 64 output channels (odd voxel count: padded P^T rows)
    (1, 8, 8, 12, 32, 0, 64, 2, False),
    (1, 3, 5, 7, 16, 0, 80, 1, False),
    # stride 2 over a batch of 2 with odd extents (parity classes of unequal size)
    (2, 5, 7, 9, 16, 0, 32, 2, False),
]


def _bf(t):
    return t.to(torch.bfloat16)


def _case(N, Di, Hi, Wi, Ca, Cb, Cout, s, ups, seed=0):
    g = torch.Generator().manual_seed(seed)
    sa = (N, Di // 2, Hi // 2, Wi // 2, Ca) if ups else (N, Di, Hi, Wi, Ca)
    xa = _bf(torch.randn(sa, generator=g))
    xb = _bf(torch.randn((N, Di, Hi, Wi, Cb), generator=g)) if Cb else None
    w = (torch.randn((Cout, 27, Ca + Cb), generator=g) * (1.0 / np.sqrt(27 * (Ca + Cb)))).contiguous()
    b = torch.randn(Cout, generator=g) * 0.1
    geom = ops.conv_geom(N, Di, Hi, Wi, Ca, Cb, Cout, s, ups)
    return xa, xb, w, b, geom


@pytest.mark.parametrize("case", CASES)
def test_conv_forward(case):
    print(f"[conv fwd {case}]", flush=True)
    N, Di, Hi, Wi, Ca, Cb, Cout, s, ups = case
    xa, xb, w, b, geom = _case(*case)
    wd = w.to(DEV)
    wbf, wt = ops.conv3d_weight_prep(wd)
    assert torch.equal(wbf.cpu(), _bf(w))
    assert torch.equal(wt.cpu(), _bf(w).permute(2, 1, 0).contiguous())
    for act in (False, True):
        ybf, yf = ops.conv3d_fwd(xa.to(DEV), None if xb is None else xb.to(DEV), wbf, b.to(DEV), geom, act=act,
                                 slope=SLOPE, want_f32=True)
        ref = oracle.conv3d_fwd(xa.double(), None if xb is None else xb.double(), wbf.cpu().double(), b.double(), N,
                                Di, Hi, Wi, Ca, Cb, Cout, stride=s, ups=ups, act=act, slope=SLOPE)
        assert_grad(yf.cpu().numpy(), ref, f"fwd act={act}")
        assert torch.equal(ybf.cpu(), _bf(yf.cpu()))


@pytest.mark.parametrize("case", CASES)
def test_conv_backward(case):
    print(f"[conv bwd {case}]", flush=True)
    N, Di, Hi, Wi, Ca, Cb, Cout, s, ups = case
    xa, xb, w, b, geom = _case(*case, seed=1)
    wbf, wt = ops.conv3d_weight_prep(w.to(DEV))
    xad, xbd = xa.to(DEV), (None if xb is None else xb.to(DEV))
    y = ops.conv3d_fwd(xad, xbd, wbf, b.to(DEV), geom, act=True, slope=SLOPE)
    Do, Ho, Wo = ops.conv_out_shape(geom)
    dy = torch.randn((N, Do, Ho, Wo, Cout), generator=torch.Generator().manual_seed(5))
    # the operand both sides use: bf16(dy * act'(y)) with the product in fp32
    P = _bf(dy * torch.where(y.cpu().float() > 0, 1.0, SLOPE)).double()
    dx = ops.conv3d_bwd_data(dy.to(DEV), y, wt, geom, slope=SLOPE)
    ref_dx = oracle.conv3d_bwd_data(P, wbf.cpu().double(), N, Di, Hi, Wi, Ca, Cb, Cout, stride=s)
    assert_grad(dx.cpu().numpy(), ref_dx, "bwd data")
    dx2 = ops.conv3d_bwd_data(dy.to(DEV), y, wt, geom, slope=SLOPE, dx=dx.clone(), accumulate=True)
    assert_grad(dx2.cpu().numpy(), 2 * ref_dx, "bwd data accumulate")
    # the same from P formed once in bf16: P itself bit for bit, dx bit for bit
    pb = ops.conv3d_act_grad(dy.to(DEV), y, slope=SLOPE)
    assert torch.equal(pb.cpu(), _bf(P))
    assert torch.equal(ops.conv3d_bwd_data_bf16(pb, wt, geom), dx)
    assert torch.equal(ops.conv3d_bwd_data_bf16(pb, wt, geom, dx=dx.clone(), accumulate=True), dx2)
    dw, db = ops.conv3d_bwd_weight(xad, xbd, dy.to(DEV), y, geom, slope=SLOPE)
    ref_dw, ref_db = oracle.conv3d_bwd_weight(xa.double(), None if xb is None else xb.double(), P, N, Di, Hi, Wi, Ca,
                                              Cb, Cout, stride=s, ups=ups)
    assert_grad(dw.cpu().numpy(), ref_dw, "bwd weight")
    assert_grad(db.cpu().numpy(), ref_db, "bwd bias")
    dwp, dbp = ops.conv3d_bwd_weight_bf16(xad, xbd, pb, geom)
    assert torch.equal(dwp, dw) and torch.equal(dbp, db)


def test_no_activation_backward():
    case = (2, 5, 7, 6, 16, 0, 4, 1, False)
    N, Di, Hi, Wi, Ca, Cb, Cout, s, ups = case
    xa, xb, w, b, geom = _case(*case, seed=2)
    wbf, wt = ops.conv3d_weight_prep(w.to(DEV))
    dy = torch.randn((N, Di, Hi, Wi, Cout), generator=torch.Generator().manual_seed(6))
    P = _bf(dy).double()
    dx = ops.conv3d_bwd_data(dy.to(DEV), None, wt, geom)
    assert_grad(dx.cpu().numpy(), oracle.conv3d_bwd_data(P, wbf.cpu().double(), N, Di, Hi, Wi, Ca, Cb, Cout), "dx")
    pb = ops.conv3d_act_grad(dy.to(DEV), None)
    assert torch.equal(pb.cpu(), _bf(dy))
    assert torch.equal(ops.conv3d_bwd_data_bf16(pb, wt, geom), dx)
    dw, db = ops.conv3d_bwd_weight(xa.to(DEV), None, dy.to(DEV), None, geom)
    rdw, rdb = oracle.conv3d_bwd_weight(xa.double(), None, P, N, Di, Hi, Wi, Ca, Cb, Cout)
    assert_grad(dw.cpu().numpy(), rdw, "dw")
    assert_grad(db.cpu().numpy(), rdb, "db")
    dwp, dbp = ops.conv3d_bwd_weight_bf16(xa.to(DEV), None, pb, geom)
    assert torch.equal(dwp, dw) and torch.equal(dbp, db)


def test_act_grad_lengths_and_offsets():
    # the 8-wide kernel with a scalar tail, and the scalar kernel alone for
    # operands that are not 16-byte aligned
    g = torch.Generator().manual_seed(11)
    for n in (1, 7, 8, 1003, 4096 + 5):
        dy = torch.randn(n + 1, generator=g)
        y = _bf(torch.randn(n + 1, generator=g))
        dyd, yd = dy.to(DEV), y.to(DEV)
        for off in (0, 1):  # offset 1: views 4 and 2 bytes past a 16-byte boundary
            d, yy = dy[off:off + n], y[off:off + n]
            ref = _bf(d * torch.where(yy.float() > 0, 1.0, SLOPE))
            assert torch.equal(ops.conv3d_act_grad(dyd[off:off + n], yd[off:off + n], slope=SLOPE).cpu(), ref)
            assert torch.equal(ops.conv3d_act_grad(dyd[off:off + n], None).cpu(), _bf(d))


def test_helper_kernels():
    g = torch.Generator().manual_seed(9)
    F = torch.rand((2, 6, 5, 4), generator=g)
    M = torch.rand((2, 6, 5, 4), generator=g)
    x = ops.unet_pack_pair(F.to(DEV), M.to(DEV)).cpu()
    assert torch.equal(x[..., 0], _bf(F)) and torch.equal(x[..., 1], _bf(M)) and float(x[..., 2:].abs().max()) == 0
    geom = ops.conv_geom(2, 6, 4, 8, 8, 4, 4, 1, True)
    dxc = torch.randn((2, 6, 4, 8, 12), generator=g)
    dxa, dxb = ops.concat_grad_split(dxc.to(DEV), geom)
    ref_b = dxc[..., 8:]
    ref_a = dxc[..., :8].reshape(2, 3, 2, 2, 2, 4, 2, 8).sum(dim=(2, 4, 6))
    torch.testing.assert_close(dxb.cpu(), ref_b, rtol=0, atol=0)
    torch.testing.assert_close(dxa.cpu(), ref_a, rtol=1e-6, atol=1e-6)
    # channel groups that do not divide 256 (Ca = 12, Cb = 20), rows longer
    # than one pass of the block, accumulation, and no skip part (Cb = 0)
    for (N, Di, Hi, Wi, Ca, Cb) in [(1, 2, 4, 200, 12, 20), (2, 4, 2, 6, 16, 0)]:
        geom = ops.conv_geom(N, Di, Hi, Wi, Ca, Cb, 4, 1, True)
        dxc = torch.randn((N, Di, Hi, Wi, Ca + Cb), generator=g)
        a0 = torch.randn((N, Di // 2, Hi // 2, Wi // 2, Ca), generator=g)
        b0 = torch.randn((N, Di, Hi, Wi, Cb), generator=g) if Cb else None
        dxa, dxb = ops.concat_grad_split(dxc.to(DEV), geom, dxa=a0.to(DEV), dxb=None if b0 is None else b0.to(DEV),
                                         acc_a=True, acc_b=True)
        ref_a = dxc[..., :Ca].reshape(N, Di // 2, 2, Hi // 2, 2, Wi // 2, 2, Ca).sum(dim=(2, 4, 6))
        torch.testing.assert_close(dxa.cpu(), a0 + ref_a, rtol=1e-6, atol=1e-6)
        if Cb:
            torch.testing.assert_close(dxb.cpu(), b0 + dxc[..., Ca:], rtol=0, atol=0)
        else:
            assert dxb is None
    pred = torch.randn((2, 5, 6, 7, 4), generator=g)
    tgt = torch.randn((2, 3, 5, 6, 7), generator=g)
    loss, dpred = ops.mse_disp(pred.to(DEV), tgt.to(DEV))
    diff = pred[..., :3].double() - tgt.permute(0, 2, 3, 4, 1).double()
    assert abs(float(loss) - float((diff ** 2).mean())) < 1e-6
    ref_g = torch.cat([2 * diff / diff.numel(), torch.zeros(2, 5, 6, 7, 1, dtype=torch.float64)], -1)
    torch.testing.assert_close(dpred.cpu().double(), ref_g, rtol=1e-5, atol=1e-9)
    u = ops.unpack_disp(pred.to(DEV)).cpu()
    torch.testing.assert_close(u, pred[..., :3].permute(0, 4, 1, 2, 3), rtol=0, atol=0)
