"""GPU parity of the Gaussian field smoothing (ffdp_gaussian_smooth) against
the oracle's direct (2R+1)^3 sum: ragged shapes spanning several 64 x 16
tiles and z chunks, arrays thinner than the kernel radius, every supported
radius, and sampled crops of a full 512^3 three-channel field; and of the
fused smoothing + Adam step (ffdp_smooth_adam_step)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_25044_amd import ops
from paper_2509_25044_amd._lib import FfdpError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _field(shape, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(shape, generator=g, dtype=torch.float32)


def _tol(x):
    # three passes of at most 13 fp32 fused multiply-adds with taps summing to 1
    return 4e-6 * float(np.abs(x).max())


@pytest.mark.parametrize("shape,sigma", [
    ((3, 37, 45, 131), 1.0),
    ((3, 37, 45, 131), 0.5),
    ((1, 70, 20, 5), 2.0),
    ((2, 2, 1, 3), 1.0),
    ((1, 1, 1, 1), 0.5),
    ((3, 33, 17, 64), 0.3),
])
def test_matches_oracle(shape, sigma):
    print(f"[smooth {shape} sigma {sigma}]", flush=True)
    x = _field(shape, 11 + len(shape))
    y = ops.gaussian_smooth(x.to(DEV), sigma).cpu().numpy()
    ref = oracle.gaussian_smooth(x.numpy(), sigma)
    err = np.abs(y - ref).max()
    assert err <= _tol(ref), err


def test_single_volume_and_determinism():
    print("[smooth 3d input, repeat]", flush=True)
    x = _field((29, 31, 67), 5).to(DEV)
    a = ops.gaussian_smooth(x, 1.0)
    b = ops.gaussian_smooth(x, 1.0)
    assert a.shape == x.shape and torch.equal(a, b)
    ref = oracle.gaussian_smooth(x.cpu().numpy(), 1.0)
    assert np.abs(a.cpu().numpy() - ref).max() <= _tol(ref)


def test_rejects_overlap_and_bad_sigma():
    print("[smooth validation]", flush=True)
    x = torch.zeros((3, 8, 8, 8), device=DEV)
    with pytest.raises(FfdpError):
        ops.gaussian_smooth(x, 1.0, out=x)
    with pytest.raises(FfdpError):
        ops.gaussian_smooth(x, 0.0)
    with pytest.raises(FfdpError):
        ops.gaussian_smooth(x, 2.5)


@pytest.mark.parametrize("shape,sigma,step", [
    ((3, 37, 45, 131), 1.0, 1),
    ((3, 33, 17, 64), 0.5, 7),
    ((1, 70, 20, 5), 2.0, 2),
    ((2, 2, 1, 3), 1.0, 3),
])
def test_smooth_adam_step_is_smooth_then_adam(shape, sigma, step):
    """The fused step equals ffdp_gaussian_smooth followed by ffdp_adam_step
    bitwise, and the oracle's smoothing followed by its Adam step within the
    smoothing tolerance carried through Adam's normalisation."""
    print(f"[smooth+adam shape={shape} sigma={sigma} step={step}]", flush=True)
    g = _field(shape, 11).to(DEV)
    x0 = _field(shape, 12).to(DEV)
    m0 = 0.1 * _field(shape, 13).to(DEV)
    v0 = (1e-4 + 0.01 * _field(shape, 14).abs()).to(DEV)  # away from 0: the step stays well conditioned
    x1, m1, v1 = x0.clone(), m0.clone(), v0.clone()
    ops.smooth_adam_step(x1, g, m1, v1, sigma, lr=0.05, step=step)
    x2, m2, v2 = x0.clone(), m0.clone(), v0.clone()
    ops.adam_step(x2, ops.gaussian_smooth(g, sigma), m2, v2, lr=0.05, step=step)
    assert torch.equal(x1, x2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    sg = oracle.gaussian_smooth(g.cpu().numpy(), sigma)
    xr, mr, vr = (t.cpu().numpy().astype(np.float64) for t in (x0, m0, v0))
    oracle.adam(xr, sg.astype(np.float64), mr, vr, lr=0.05, step=step)
    assert np.abs(m1.cpu().numpy() - mr).max() <= _tol(sg)
    assert np.abs(x1.cpu().numpy() - xr).max() <= 1e-4 * 0.05 * max(1.0, float(np.abs(xr).max()))


def test_smooth_adam_rejects_overlap():
    print("[smooth+adam validation]", flush=True)
    x, g, m, v = (torch.zeros((3, 8, 8, 8), device=DEV) for _ in range(4))
    for args in ((x, x, m, v), (x, g, x, v), (x, g, m, m)):
        with pytest.raises(FfdpError):
            ops.smooth_adam_step(*args, 1.0, lr=0.1)
    with pytest.raises(FfdpError):
        ops.smooth_adam_step(x, g, m, v, 1.0, lr=0.1, step=0)


@pytest.mark.parametrize("sigma", [1.0, 0.5])
def test_full_size_sampled_crops(sigma):
    """512^3 x 3 channels (the displacement of the 512^3 workload): outputs in
    boxes at the corners, a face and the centre, each checked with the oracle
    run on the box plus an R-voxel halo (edge replication inside the array
    is the same on the crop wherever the crop meets the array boundary)."""
    print(f"[smooth 512^3 x3 sigma {sigma}]", flush=True)
    n = 512
    R = int(np.ceil(3 * sigma))
    g = torch.Generator(device=DEV).manual_seed(77)
    x = torch.randn((3, n, n, n), generator=g, device=DEV, dtype=torch.float32)
    y = ops.gaussian_smooth(x, sigma)
    torch.cuda.synchronize()
    boxes = [((0, 0, 0), 12), ((n - 12, n - 12, n - 12), 12), ((250, 0, 300), 16), ((200, 201, 202), 20),
             ((0, 511 - 10, 128), 11)]
    for lo, s in boxes:
        clo = [max(a - R, 0) for a in lo]
        chi = [min(a + s + R, n) for a in lo]
        crop = x[:, clo[0]:chi[0], clo[1]:chi[1], clo[2]:chi[2]].cpu().numpy()
        ref = oracle.gaussian_smooth(crop, sigma)
        o = [a - c for a, c in zip(lo, clo)]
        ref = ref[:, o[0]:o[0] + s, o[1]:o[1] + s, o[2]:o[2] + s]
        got = y[:, lo[0]:lo[0] + s, lo[1]:lo[1] + s, lo[2]:lo[2] + s].cpu().numpy()
        assert got.shape == ref.shape
        err = np.abs(got - ref).max()
        assert err <= _tol(ref), (lo, err)
