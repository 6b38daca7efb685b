"""The binding rejects wrongly shaped, typed or placed buffers before any
launch: a wrong buffer would otherwise become out-of-bounds device reads or
writes.  The validators are checked on the CPU; the GPU half calls every
entry point with one bad buffer at a time and expects the error (nothing is
launched, so nothing runs on the device)."""
import pytest
import torch

from paper_2509_25044_amd import ops


def test_out_validator_checks_shape_dtype_device_layout():
    dev = torch.device("cpu")
    ok = torch.zeros(3, 4, 5)
    assert ops._out(ok, "x", (3, 4, 5), dev) is ok
    with pytest.raises(ValueError, match="shape"):
        ops._out(torch.zeros(3, 4, 6), "x", (3, 4, 5), dev)
    with pytest.raises(TypeError, match="float32"):
        ops._out(torch.zeros(3, 4, 5, dtype=torch.float64), "x", (3, 4, 5), dev)
    with pytest.raises(ValueError, match="contiguous"):
        ops._out(torch.zeros(5, 4, 3).permute(2, 1, 0), "x", (3, 4, 5), dev)
    with pytest.raises(ValueError, match="must be on"):
        ops._out(ok, "x", (3, 4, 5), torch.device("meta"))
    with pytest.raises(TypeError):
        ops._out(ok.numpy(), "x", (3, 4, 5), dev)


def test_scalar_and_workspace_validators():
    dev = torch.device("cpu")
    assert ops._dev_scalar(None, "s", dev) is None
    ops._dev_scalar(torch.zeros(1), "s", dev)
    with pytest.raises(ValueError):
        ops._dev_scalar(torch.zeros(1, dtype=torch.float64), "s", dev)
    with pytest.raises(ValueError, match="at least"):
        ops._dev_scalar(torch.zeros(10), "state", dev, n=11)
    assert ops._ws_bytes(torch.zeros(10, dtype=torch.uint8), dev) == 10
    assert ops._ws_bytes(torch.zeros(10, dtype=torch.float32), dev) == 40  # bytes, not elements
    with pytest.raises(ValueError):
        ops._ws_bytes(torch.zeros(10, dtype=torch.uint8), torch.device("meta"))


@pytest.mark.gpu
def test_entry_points_reject_bad_buffers():
    dev = torch.device("cuda:0")
    D, H, W = 6, 7, 9
    F = torch.rand(D, H, W, device=dev)
    M = torch.rand(D, H, W, device=dev)
    u = torch.zeros(3, D, H, W, device=dev)
    bad_u = torch.zeros(3, D, H, W + 1, device=dev)
    f64 = torch.zeros(3, D, H, W, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        ops.warp(M, bad_u)
    with pytest.raises(ValueError):
        ops.warp(M, u, out=torch.empty(D, H, W + 1, device=dev))
    with pytest.raises(ValueError):
        ops.warp_lncc_bwd(F, M, u, grad_u=torch.empty(3, D, H, W - 1, device=dev))
    with pytest.raises(TypeError):
        ops.warp_lncc_bwd(F, M, u, grad_u=f64)
    with pytest.raises(ValueError):
        ops.warp_lncc_bwd(F, M, u, grad_scale=torch.ones(1, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        ops.warp_lncc_bwd(F, M, u, loss=torch.empty(0, device=dev))
    with pytest.raises(ValueError):
        ops.warp_mi_fwd(F, M, u, bins=32, state=torch.empty(10, device=dev))
    _, st = ops.warp_mi_fwd(F, M, u, bins=16)
    with pytest.raises(ValueError):
        ops.warp_mi_bwd(F, M, u, st, bins=32)  # a 16-bin state is too small for 32 bins
    with pytest.raises(ValueError):
        ops.warp_mi_bwd(F, M, u, st, bins=16, grad_u=torch.empty(3, D, H, device=dev))
    with pytest.raises(ValueError):
        ops.warp_affine(M, bad_u)
    with pytest.raises(ValueError):
        ops.warp_affine_bwd(M, torch.zeros(D, H, W, device=dev), u=bad_u)
    with pytest.raises(ValueError):
        ops.warp_affine_bwd(M, torch.zeros(D, H, W + 1, device=dev), u=u)
    with pytest.raises(ValueError):
        ops.adam_step(u, u, u, torch.zeros(3, D, H, W, device=dev)[:, :, :, :4].contiguous(), lr=0.1)
    with pytest.raises(ValueError):
        ops.gaussian_smooth(u, 1.0, out=torch.empty(3, D, H, W + 1, device=dev))
    g = ops.conv_geom(1, 8, 8, 8, 4, 0, 16)
    xa = torch.zeros(1, 8, 8, 8, 4, dtype=torch.bfloat16, device=dev)
    wb = torch.zeros(16, 27, 4, dtype=torch.bfloat16, device=dev)
    with pytest.raises(ValueError):
        ops.conv3d_fwd(xa[:, :4].contiguous(), None, wb, None, g)
    with pytest.raises(ValueError):
        ops.conv3d_fwd(xa, None, wb[:8].contiguous(), None, g)
    with pytest.raises(TypeError):
        ops.conv3d_fwd(xa.float(), None, wb, None, g)
    with pytest.raises(ValueError):
        ops.mse_disp(torch.zeros(1, 8, 8, 8, 4, device=dev), torch.zeros(1, 3, 8, 8, 7, device=dev))
    torch.cuda.synchronize()
