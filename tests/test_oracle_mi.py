"""Pins of the oracle's Parzen mutual information (O4) and its gradient.

Paper passages: eq. (mi) (kernel density estimates of the marginal and joint
intensity distributions), App. "Vanilla MI implementation" (B bins on [0,1],
Parzen block), the B-spline kernel choice, and the adjoint of App. "Backward
pass" (gradient given dL/dp_IJ and the marginals).

Pins: scipy's cardinal B-spline basis element for kappa and its derivative,
partition of unity, sum p = 1, symmetry, entropy identities (MI(F,F) =
2 H(p_F) - H(p_FF), equality with H(p_F) for the box kernel), near-zero MI
of independent inputs, autograd of an independent torch Parzen-block route,
and central finite differences.
"""
import numpy as np
import pytest
import torch
from scipy.interpolate import BSpline

from paper_2509_25044_amd import synth

_B3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
_dB3 = _B3.derivative()


def _b3(t):
    v = _B3(np.asarray(t, np.float64))
    return np.nan_to_num(v, nan=0.0)


def _db3(t):
    v = _dB3(np.asarray(t, np.float64))
    return np.nan_to_num(v, nan=0.0)


@pytest.mark.parametrize("B", [8, 32, 256])
def test_parzen_weights_match_scipy_bspline_in_the_interior(orc, B):
    rng = np.random.default_rng(30)
    for v in rng.uniform(2.0 / B, 1.0 - 2.0 / B, 50):
        k, o = orc.parzen(v, B)
        s = v * B - 0.5
        m = np.arange(B)
        np.testing.assert_allclose(k, _b3(s - m), rtol=0, atol=1e-15)
        np.testing.assert_allclose(o, B * _db3(s - m), rtol=0, atol=1e-12)


@pytest.mark.parametrize("B", [8, 32, 64, 200, 256])
def test_parzen_partition_of_unity_and_zero_derivative_sum(orc, B):
    for v in np.concatenate([np.linspace(-0.1, 1.1, 241), [0.0, 1.0, 0.5 / B, 1 - 0.5 / B]]):
        k, o = orc.parzen(v, B)
        assert abs(k.sum() - 1.0) < 1e-14
        assert np.all(k >= 0.0)
        assert abs(o.sum()) < 1e-11
        if v < 0.0 or v > 1.0:
            assert np.all(o == 0.0)


def test_parzen_bin_centre_values(orc):
    B = 16
    k, _ = orc.parzen((5 + 0.5) / B, B)
    assert abs(k[5] - 2.0 / 3.0) < 1e-15 and abs(k[4] - 1.0 / 6.0) < 1e-15 and abs(k[6] - 1.0 / 6.0) < 1e-15


def test_hard_bins(orc):
    k, o = orc.parzen(1.0, 8, hard=True)
    assert k[7] == 1.0 and k.sum() == 1.0 and np.all(o == 0)
    k, _ = orc.parzen(0.124, 8, hard=True)
    assert k[0] == 1.0


def test_joint_pmf_sums_to_one_and_is_symmetric(orc):
    F = synth.random_volume((8, 8, 8), 31).numpy()
    M = synth.random_volume((8, 8, 8), 32).numpy()
    l1, p1, _ = orc.mi(F, M, None, bins=16, with_grad=False)
    l2, p2, _ = orc.mi(M, F, None, bins=16, with_grad=False)
    assert abs(p1.sum() - 1.0) < 1e-13
    np.testing.assert_allclose(p1, p2.T, rtol=0, atol=1e-16)
    assert abs(l1 - l2) < 1e-13


def _entropy(p):
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


@pytest.mark.parametrize("B", [8, 32, 256])
def test_self_information_identity_and_bounds(orc, B):
    F = synth.random_volume((10, 9, 8), 33).numpy()
    loss, p, _ = orc.mi(F, F, None, bins=B, with_grad=False)
    pF = p.sum(1)
    H_F, H_FF = _entropy(pF), _entropy(p)
    mi = -loss
    assert abs(mi - (2 * H_F - H_FF)) < 1e-12
    assert 0.0 <= mi <= H_F + 1e-12
    lh, ph, _ = orc.mi(F, F, None, bins=B, hard=True, with_grad=False)
    assert abs(-lh - _entropy(ph.sum(1))) < 1e-12


def test_independent_inputs_have_small_mi(orc):
    F = synth.random_volume((32, 32, 32), 34).numpy()
    M = synth.random_volume((32, 32, 32), 35).numpy()
    loss, _, _ = orc.mi(F, M, None, bins=8, with_grad=False)
    assert 0.0 <= -loss < 2e-3


def _torch_parzen_block(v, B):
    """Independent route: the full Parzen block kappa(b_m - v) for every bin m
    through scipy-checked closed-form B-spline pieces in torch, with the
    edge folding done by explicit extra bins."""
    vc = v.clamp(0.0, 1.0)
    s = vc * B - 0.5
    js = torch.arange(-2, B + 2, dtype=torch.float64)
    t = (s[..., None] - js).abs()
    w = torch.where(t < 1, (4 - 6 * t ** 2 + 3 * t ** 3) / 6, torch.where(t < 2, (2 - t).clamp(min=0) ** 3 / 6,
                                                                         torch.zeros_like(t)))
    left = w[..., :3].sum(-1, keepdim=True)    # j = -2, -1, 0 fold onto bin 0
    right = w[..., -3:].sum(-1, keepdim=True)  # j = B-1, B, B+1 fold onto bin B-1
    return torch.cat([left, w[..., 3:-3], right], dim=-1)


def _grid_sample(M, u):
    D, H, W = M.shape
    zz, yy, xx = torch.meshgrid(torch.arange(D, dtype=torch.float64), torch.arange(H, dtype=torch.float64),
                                torch.arange(W, dtype=torch.float64), indexing="ij")
    p = torch.stack([xx + u[0], yy + u[1], zz + u[2]], dim=-1)
    scale = torch.tensor([2.0 / (W - 1), 2.0 / (H - 1), 2.0 / (D - 1)], dtype=torch.float64)
    return torch.nn.functional.grid_sample(M[None, None], (p * scale - 1.0)[None], mode="bilinear",
                                           padding_mode="border", align_corners=True)[0, 0]


@pytest.mark.parametrize("B,roi", [(8, None), (16, ((1, 6), (0, 7), (2, 8))), (256, None)])
def test_loss_and_gradient_match_autograd_of_parzen_block_route(orc, B, roi):
    D, H, W = 7, 8, 9
    F = synth.random_volume((D, H, W), 36, lo=0.05, hi=0.95).numpy()
    M = synth.random_volume((D, H, W), 37, lo=0.05, hi=0.95).numpy()
    u = synth.random_disp((D, H, W), 38, 1.5, avoid_kinks=True).numpy()
    r6 = None if roi is None else np.array([roi[0][0], roi[0][1], roi[1][0], roi[1][1], roi[2][0], roi[2][1]])
    loss, p, g = orc.mi(F, M, u, roi=r6, bins=B)
    ut = torch.from_numpy(u.astype(np.float64)).requires_grad_(True)
    Mw = _grid_sample(torch.from_numpy(M.astype(np.float64)), ut)
    Ft = torch.from_numpy(F.astype(np.float64))
    if roi is not None:
        (z0, z1), (y0, y1), (x0, x1) = roi
        Ft, Mw = Ft[z0:z1, y0:y1, x0:x1], Mw[z0:z1, y0:y1, x0:x1]
    PF = _torch_parzen_block(Ft.reshape(-1), B)
    PM = _torch_parzen_block(Mw.reshape(-1), B)
    P = PF.T @ PM / PF.shape[0]
    pF, pM = P.sum(1), P.sum(0)
    mask = P > 0
    mi = (P[mask] * torch.log(P[mask] / (pF[:, None] * pM[None, :])[mask])).sum()
    (-mi).backward()
    np.testing.assert_allclose(p, P.detach().numpy(), rtol=0, atol=1e-15)
    assert abs(loss - float(-mi)) < 1e-12
    np.testing.assert_allclose(g, ut.grad.numpy(), rtol=0, atol=1e-10 * np.abs(g).max())


def test_gradient_central_differences(orc):
    D, H, W = 8, 8, 8
    F = synth.random_volume((D, H, W), 39, lo=0.05, hi=0.95).numpy()
    M = synth.random_volume((D, H, W), 40, lo=0.05, hi=0.95).numpy()
    u = synth.random_disp((D, H, W), 41, 1.5, avoid_kinks=True).numpy()
    _, _, g = orc.mi(F, M, u, bins=8)
    rng = np.random.default_rng(42)
    for _ in range(12):
        c, z, y, x = rng.integers(0, 3), rng.integers(0, D), rng.integers(0, H), rng.integers(0, W)
        up, um = u.copy(), u.copy()
        up[c, z, y, x] = np.float32(u[c, z, y, x] + np.float32(1e-3))
        um[c, z, y, x] = np.float32(u[c, z, y, x] - np.float32(1e-3))
        h = float(up[c, z, y, x]) - float(um[c, z, y, x])
        lp, _, _ = orc.mi(F, M, up, bins=8, with_grad=False)
        lm, _, _ = orc.mi(F, M, um, bins=8, with_grad=False)
        fd = (lp - lm) / h
        assert abs(fd - g[c, z, y, x]) <= 2e-5 * np.abs(g).max() + 1e-6 * abs(fd), (c, z, y, x, fd, g[c, z, y, x])


# ---- the approximate estimator (hard-bin counts convolved with the kernel) ----
def _folded_kernel_matrix(B):
    """K[m][j]: weight that a sample at the centre of bin j gives bin m under
    the cubic B-spline of one bin width, support outside [0, B) folded onto
    the edge bins; built from scipy's B-spline, not from the oracle."""
    b3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
    K = np.zeros((B, B))
    for j in range(B):
        for off in range(-2, 3):
            w = b3(float(off))
            w = 0.0 if np.isnan(w) else float(w)
            K[min(max(j + off, 0), B - 1), j] += w
    return K


def test_approx_estimator_counts_and_convolution_brute_force(orc):
    """p = K (counts / N) K^T with numpy counts of floor(v B) (clipped)."""
    B = 16
    rng = np.random.default_rng(41)
    F = rng.uniform(-0.05, 1.05, (6, 7, 8)).astype(np.float32)
    M = rng.uniform(-0.05, 1.05, (6, 7, 8)).astype(np.float32)
    _, p, _ = orc.mi(F, M, None, bins=B, hard=2, with_grad=False)
    bf = np.clip(np.floor(np.clip(F.astype(np.float64), 0, 1) * B), 0, B - 1).astype(int).ravel()
    bm = np.clip(np.floor(np.clip(M.astype(np.float64), 0, 1) * B), 0, B - 1).astype(int).ravel()
    cnt = np.zeros((B, B))
    np.add.at(cnt, (bf, bm), 1.0)
    K = _folded_kernel_matrix(B)
    ref = K @ (cnt / bf.size) @ K.T
    np.testing.assert_allclose(p, ref, rtol=0, atol=1e-15)
    assert abs(p.sum() - 1.0) < 1e-13


def test_approx_estimator_is_exact_on_bin_centres(orc):
    """Samples on bin centres: the soft weights are the bin-centre kernel
    taps, so the approximate PMF, loss and gradient equal the exact ones
    (the gradient formula of the approximate mode is the exact one)."""
    B = 16
    rng = np.random.default_rng(42)
    F = ((rng.integers(0, B, (7, 8, 9)) + 0.5) / B).astype(np.float32)
    M = ((rng.integers(0, B, (7, 8, 9)) + 0.5) / B).astype(np.float32)
    u = np.zeros((3, 7, 8, 9), np.float32)
    le, pe, ge = orc.mi(F, M, u, bins=B, hard=0)
    la, pa, ga = orc.mi(F, M, u, bins=B, hard=2)
    np.testing.assert_allclose(pa, pe, rtol=0, atol=1e-15)
    assert abs(la - le) < 1e-13
    np.testing.assert_allclose(ga, ge, rtol=1e-12, atol=1e-15)


def test_approx_estimator_swap_symmetry_and_closeness(orc):
    """Swapping F and M transposes p and keeps MI; on smooth data the
    approximate MI stays within a few percent of the exact MI."""
    B = 32
    spec = synth.PairSpec((16, 20, 24), (3.0, 6.0), 2.0)
    pr = synth.make_pair(spec, seed=5)
    F, M = pr["F"].numpy(), pr["M"].numpy()
    la, pa, _ = orc.mi(F, M, None, bins=B, hard=2, with_grad=False)
    lb, pb, _ = orc.mi(M, F, None, bins=B, hard=2, with_grad=False)
    np.testing.assert_allclose(pb, pa.T, rtol=0, atol=1e-15)
    assert abs(la - lb) < 1e-12
    le, _, _ = orc.mi(F, M, None, bins=B, hard=0, with_grad=False)
    assert abs(la - le) < 0.05 * abs(le), (la, le)


@pytest.mark.parametrize("hard", [0, 2])
def test_streamed_pmf_and_pointwise_gradient_match_whole_volume_mi(orc, hard):
    """mi_pmf (sampling on the fly, per-thread histograms) equals the PMF of
    mi() (pinned above to brute force and closed forms), and mi_grad_u_at
    given that PMF equals mi()'s gradient at the listed voxels, inside and
    outside an ROI."""
    rng = np.random.default_rng(31)
    D, H, W = 9, 11, 13
    F = rng.random((D, H, W)).astype(np.float32)
    M = rng.random((D, H, W)).astype(np.float32)
    u = (1.7 * rng.standard_normal((3, D, H, W))).astype(np.float32)
    roi = [1, 8, 2, 10, 0, 12]
    loss, p, g = orc.mi(F, M, u, roi=roi, bins=12, hard=hard)
    ps = orc.mi_pmf(F, M, u, roi=roi, bins=12, hard=hard)
    np.testing.assert_allclose(ps, p, rtol=1e-12, atol=1e-15)
    pts = np.array([[z, y, x] for z in (0, 1, 4, 7, 8) for y in (0, 2, 9, 10) for x in (0, 5, 11, 12)])
    gp = orc.mi_grad_u_at(F, M, u, pts, ps, roi=roi, bins=12, hard=hard)
    ref = g[:, pts[:, 0], pts[:, 1], pts[:, 2]].T
    np.testing.assert_allclose(gp, ref, rtol=1e-10, atol=1e-14)
    assert np.abs(ref).max() > 0


def test_pointwise_gradient_is_the_finite_difference_of_the_loss(orc):
    """mi_grad_u_at against central differences of mi()'s loss in one voxel's
    displacement (fractional parts kept away from the trilinear kinks)."""
    rng = np.random.default_rng(32)
    D, H, W = 8, 9, 10
    F = rng.random((D, H, W)).astype(np.float32)
    M = rng.random((D, H, W)).astype(np.float32)
    u = (0.3 + 0.4 * rng.random((3, D, H, W))).astype(np.float32)
    p = orc.mi_pmf(F, M, u, bins=8)
    k = (4, 5, 3)
    g = orc.mi_grad_u_at(F, M, u, [k], p, bins=8)[0]
    h = 1e-3
    for c in range(3):
        up, um = u.copy(), u.copy()
        up[c][k] += h
        um[c][k] -= h
        fd = (orc.mi(F, M, up, bins=8, with_grad=False)[0] - orc.mi(F, M, um, bins=8, with_grad=False)[0]) / (
            float(up[c][k]) - float(um[c][k]))
        assert abs(fd - g[c]) <= 2e-3 * abs(g[c]) + 1e-9, (c, fd, g[c])


def test_streamed_pmf_counts_values_near_bin_edges(orc):
    """The edge count of mi_pmf is the number of ROI voxels whose clamped
    warped value lies within the tolerance of an interior bin edge (counted
    here from the oracle's warp)."""
    rng = np.random.default_rng(33)
    D, H, W = 8, 9, 10
    F = rng.random((D, H, W)).astype(np.float32)
    M = (np.round(rng.random((D, H, W)) * 16) / 16).astype(np.float32)  # many values on edges of 8 or 16 bins
    u = np.zeros((3, D, H, W), np.float32)
    u[0, ::2] = 0.5
    for B, tol in ((8, 1e-6), (16, 1e-6), (16, 0.02)):
        _, ne = orc.mi_pmf(F, M, u, roi=[1, 7, 0, 9, 2, 10], bins=B, edge_tol=tol, with_edges=True)
        mw = np.clip(orc.warp(M, u), 0.0, 1.0)[1:7, 0:9, 2:10] * B
        e = np.floor(mw + 0.5)
        ref = int(((np.abs(mw - e) <= tol * B) & (e > 0) & (e < B)).sum())
        assert ne == ref and (tol < 0.01 or ne > 0), (B, tol, ne, ref)
