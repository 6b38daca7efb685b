"""Pins of the oracle's trilinear sampler (O1) against closed forms and library routines.

Paper passage: eq. (interp) of App. "Ring Sampler" (trilinear sum over the
eight lattice neighbours) and Alg. gridsampler (implicit identity grid plus
displacement, one sample per target voxel).
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from paper_2509_25044_amd import synth


def _rand(shape, seed):
    return synth.random_volume(shape, seed).numpy()


@pytest.mark.parametrize("shift", [(0, 0, 0), (2, -1, 3), (-3, 4, -2), (7, 0, -9)])
def test_integer_shift_is_exact_edge_replicated_copy(orc, shift):
    D, H, W = 7, 9, 11
    M = _rand((D, H, W), 1)
    u = np.zeros((3, D, H, W), np.float32)
    u[0], u[1], u[2] = shift[0], shift[1], shift[2]
    out = orc.warp(M, u, pad=0)
    z = np.clip(np.arange(D) + shift[2], 0, D - 1)
    y = np.clip(np.arange(H) + shift[1], 0, H - 1)
    x = np.clip(np.arange(W) + shift[0], 0, W - 1)
    ref = M[np.ix_(z, y, x)].astype(np.float64)
    assert np.array_equal(out, ref)


def test_random_integer_field_is_exact_gather(orc):
    D, H, W = 6, 8, 10
    M = _rand((D, H, W), 2)
    g = np.random.default_rng(3)
    u = g.integers(-4, 5, (3, D, H, W)).astype(np.float32)
    out = orc.warp(M, u, pad=0)
    zz, yy, xx = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    ref = M[np.clip(zz + u[2].astype(int), 0, D - 1), np.clip(yy + u[1].astype(int), 0, H - 1),
            np.clip(xx + u[0].astype(int), 0, W - 1)]
    assert np.array_equal(out, ref.astype(np.float64))


def test_values_match_scipy_map_coordinates_nearest(orc):
    D, H, W = 9, 10, 12
    M = _rand((D, H, W), 4)
    u = synth.random_disp((D, H, W), 5, 3.0).numpy()
    out = orc.warp(M, u, pad=0)
    zz, yy, xx = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    coords = np.stack([zz + u[2].astype(np.float64), yy + u[1].astype(np.float64), xx + u[0].astype(np.float64)])
    ref = ndi.map_coordinates(M.astype(np.float64), coords, order=1, mode="nearest")
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13)


def _torch_sample(M, u, mode):
    """grid_sample in float64 with align_corners=True, returns (values, dvalue/dp)."""
    D, H, W = M.shape
    Mt = torch.from_numpy(M.astype(np.float64))[None, None]
    zz, yy, xx = torch.meshgrid(torch.arange(D, dtype=torch.float64), torch.arange(H, dtype=torch.float64),
                                torch.arange(W, dtype=torch.float64), indexing="ij")
    ut = torch.from_numpy(u.astype(np.float64))
    p = torch.stack([xx + ut[0], yy + ut[1], zz + ut[2]], dim=-1)
    scale = torch.tensor([2.0 / (W - 1), 2.0 / (H - 1), 2.0 / (D - 1)], dtype=torch.float64)
    grid = (p * scale - 1.0).requires_grad_(True)
    out = torch.nn.functional.grid_sample(Mt, grid[None], mode="bilinear", padding_mode=mode, align_corners=True)
    out.sum().backward()
    dp = (grid.grad * scale).permute(3, 0, 1, 2).numpy()
    return out[0, 0].detach().numpy(), dp


@pytest.mark.parametrize("pad,mode", [(0, "border"), (1, "zeros")])
def test_values_and_derivatives_match_torch_grid_sample(orc, pad, mode):
    D, H, W = 8, 9, 10
    M = _rand((D, H, W), 6)
    u = synth.random_disp((D, H, W), 7, 2.5, avoid_kinks=True).numpy()
    val, dval = orc.warp(M, u, pad=pad, with_grad=True)
    tv, td = _torch_sample(M, u, mode)
    np.testing.assert_allclose(val, tv, rtol=0, atol=1e-13)
    np.testing.assert_allclose(dval, td, rtol=0, atol=1e-12)


def test_border_derivative_convention_matches_torch_at_exact_edges(orc):
    """Points exactly on 0 or n-1 and beyond count as clamped (derivative 0)."""
    D, H, W = 5, 6, 7
    M = _rand((D, H, W), 8)
    u = np.zeros((3, D, H, W), np.float32)
    # x lands exactly on 0 for x=2, exactly on W-1 for x=W-3, beyond for others
    for x in range(W):
        u[0, :, :, x] = {2: -2.0, W - 3: 2.0}.get(x, 0.37 if x % 2 else -9.5)
    val, dval = orc.warp(M, u, pad=0, with_grad=True)
    tv, td = _torch_sample(M, u, "border")
    np.testing.assert_allclose(val, tv, rtol=0, atol=1e-13)
    np.testing.assert_allclose(dval, td, rtol=0, atol=1e-12)
    assert np.all(dval[0][:, :, 2] == 0) and np.all(dval[0][:, :, W - 3] == 0)


def test_zero_displacement_is_identity(orc):
    M = _rand((4, 5, 6), 9)
    assert np.array_equal(orc.warp(M, None), M.astype(np.float64))


def test_resample_matches_torch_interpolate(orc):
    src = synth.random_disp((5, 7, 6), 10, 1.0).numpy()
    out = orc.resample(src, (9, 13, 11), value_scale=2.0)
    ref = torch.nn.functional.interpolate(torch.from_numpy(src.astype(np.float64))[None], size=(9, 13, 11),
                                          mode="trilinear", align_corners=True)[0].numpy() * 2.0
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13)


def test_ring_sampler_slab_identity(orc):
    """The ring sampler's decomposition (Sec. "Ring Sampler", eq. interp-h):
    with zero padding, warping M equals the sum over z-slabs of warping the
    slab alone (M outside the slab set to zero), because the trilinear value
    is linear in M and each corner lies in exactly one slab."""
    shape = (23, 9, 11)
    M = synth.random_volume(shape, 5).numpy()
    u = synth.random_disp(shape, 6, 3.0).numpy()
    full = orc.warp(M, u, pad=1)
    acc = np.zeros_like(full)
    for a, b in ((0, 7), (7, 8), (8, 23)):
        Ms = np.zeros_like(M)
        Ms[a:b] = M[a:b]
        acc += orc.warp(Ms, u, pad=1)
    np.testing.assert_allclose(acc, full, rtol=0, atol=1e-12)
