"""Pins of the oracle's LNCC loss (O2) and its gradient (O3).

Paper passages: eq. (lncc-loss) and eq. (lncc-a/b/c) with their expanded
forms (App. "Definition of LNCC loss"), Alg. lncc (loss = 1 - mean), the
chain rule of App. "Efficient Backward Pass" and the ANTs approximation.

The pins reach the oracle from routes it does not take: library box means
(avg_pool3d, expanded moments), library sampling (grid_sample) with autograd
for the adjoint, closed forms (LNCC(F, F) = 1 at eps = 0, a single voxel),
invariances, and central finite differences.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as tf

from paper_2509_25044_amd import synth


def _lib_route_loss(F, Mw, w, eps, roi=None):
    """LNCC through library box means (zero-padded, count_include_pad) and the
    expanded moments; all float64 torch so autograd can differentiate it."""
    r = (w - 1) // 2

    def box(t):
        return tf.avg_pool3d(t[None, None], w, stride=1, padding=r, count_include_pad=True)[0, 0]

    muF, muM = box(F), box(Mw)
    A = box(F * Mw) - muF * muM
    B = box(F * F) - muF * muF
    C = box(Mw * Mw) - muM * muM
    n = A * A / (B * C + eps)
    if roi is not None:
        (z0, z1), (y0, y1), (x0, x1) = roi
        n = n[z0:z1, y0:y1, x0:x1]
    return 1.0 - n.mean()


def _grid_sample(M, u):
    D, H, W = M.shape
    zz, yy, xx = torch.meshgrid(torch.arange(D, dtype=torch.float64), torch.arange(H, dtype=torch.float64),
                                torch.arange(W, dtype=torch.float64), indexing="ij")
    p = torch.stack([xx + u[0], yy + u[1], zz + u[2]], dim=-1)
    scale = torch.tensor([2.0 / (W - 1), 2.0 / (H - 1), 2.0 / (D - 1)], dtype=torch.float64)
    return tf.grid_sample(M[None, None], (p * scale - 1.0)[None], mode="bilinear", padding_mode="border",
                          align_corners=True)[0, 0]


def _roi_tuple(roi):
    return None if roi is None else np.array([roi[0][0], roi[0][1], roi[1][0], roi[1][1], roi[2][0], roi[2][1]])


@pytest.mark.parametrize("w", [3, 5, 7])
def test_self_similarity_is_one_at_zero_eps(orc, w):
    F = synth.random_volume((9, 8, 10), 11).numpy()
    loss, _ = orc.lncc(F, F, None, window=w, eps=0.0, with_grad=False)
    assert abs(loss) < 1e-12


def test_self_similarity_with_eps_matches_library_variance(orc):
    F = synth.random_volume((8, 9, 7), 12).numpy()
    eps = 1e-3
    loss, _ = orc.lncc(F, F, None, window=5, eps=eps, with_grad=False)
    t = torch.from_numpy(F.astype(np.float64))
    B = tf.avg_pool3d((t * t)[None, None], 5, 1, 2, count_include_pad=True)[0, 0] - \
        tf.avg_pool3d(t[None, None], 5, 1, 2, count_include_pad=True)[0, 0] ** 2
    ref = 1.0 - float((B * B / (B * B + eps)).mean())
    assert abs(loss - ref) < 1e-12


def test_single_voxel_closed_form(orc):
    """One voxel, w = 3: the window holds the voxel and 26 padded zeros, so
    A = f m 26/729, B = f^2 26/729, C = m^2 26/729."""
    f, m, eps = 0.75, 0.5, 1e-4
    F = np.full((1, 1, 1), f, np.float32)
    M = np.full((1, 1, 1), m, np.float32)
    loss, _ = orc.lncc(F, M, None, window=3, eps=eps, with_grad=False)
    k = 26.0 / 729.0
    n = (f * m * k) ** 2 / ((f * f * k) * (m * m * k) + eps)
    assert abs(loss - (1.0 - n)) < 1e-15


@pytest.mark.parametrize("w,roi", [(3, None), (5, None), (5, ((2, 7), (1, 8), (3, 9))), (7, None)])
def test_loss_matches_library_box_means(orc, w, roi):
    D, H, W = 9, 10, 11
    F = synth.random_volume((D, H, W), 13).numpy()
    M = synth.random_volume((D, H, W), 14).numpy()
    u = synth.random_disp((D, H, W), 15, 2.0).numpy()
    loss, _ = orc.lncc(F, M, u, roi=_roi_tuple(roi), window=w, eps=1e-5, with_grad=False)
    Mw = _grid_sample(torch.from_numpy(M.astype(np.float64)), torch.from_numpy(u.astype(np.float64)))
    ref = float(_lib_route_loss(torch.from_numpy(F.astype(np.float64)), Mw, w, 1e-5, roi))
    assert abs(loss - ref) < 1e-12 * max(1.0, abs(ref))


def test_intensity_scale_invariance_and_interior_shift_invariance(orc):
    D, H, W = 10, 10, 10
    # values on a 2^-12 lattice so that the shifts below are exact in fp32
    F = np.round(synth.random_volume((D, H, W), 16).numpy() * 4096) / 4096
    M = np.round(synth.random_volume((D, H, W), 17).numpy() * 4096) / 4096
    eps = 1e-4
    base, _ = orc.lncc(F, M, None, window=3, eps=eps, with_grad=False)
    a, c = 2.0, 0.5  # exact in binary
    scaled, _ = orc.lncc(a * F, c * M, None, window=3, eps=eps * a * a * c * c, with_grad=False)
    assert abs(base - scaled) < 1e-12
    roi = np.array([1, 9, 1, 9, 1, 9])  # windows never touch the zero padding
    b0, _ = orc.lncc(F, M, None, roi=roi, window=3, eps=eps, with_grad=False)
    b1, _ = orc.lncc(F + 0.25, M - 0.125, None, roi=roi, window=3, eps=eps, with_grad=False)
    assert abs(b0 - b1) < 1e-10


@pytest.mark.parametrize("w,roi", [(3, None), (5, None), (5, ((1, 7), (2, 8), (0, 9)))])
def test_gradient_matches_autograd_of_library_route(orc, w, roi):
    D, H, W = 8, 9, 10
    F = synth.random_volume((D, H, W), 18).numpy()
    M = synth.random_volume((D, H, W), 19).numpy()
    u = synth.random_disp((D, H, W), 20, 1.5, avoid_kinks=True).numpy()
    eps = 1e-3
    loss, g = orc.lncc(F, M, u, roi=_roi_tuple(roi), window=w, eps=eps)
    ut = torch.from_numpy(u.astype(np.float64)).requires_grad_(True)
    Mw = _grid_sample(torch.from_numpy(M.astype(np.float64)), ut)
    ref = _lib_route_loss(torch.from_numpy(F.astype(np.float64)), Mw, w, eps, roi)
    ref.backward()
    assert abs(loss - float(ref)) < 1e-12
    np.testing.assert_allclose(g, ut.grad.numpy(), rtol=0, atol=1e-10 * np.abs(g).max())


def test_gradient_central_differences(orc):
    D, H, W = 8, 8, 8
    F = synth.random_volume((D, H, W), 21).numpy()
    M = synth.random_volume((D, H, W), 22).numpy()
    u = synth.random_disp((D, H, W), 23, 1.5, avoid_kinks=True).numpy()
    eps = 1e-5
    _, g = orc.lncc(F, M, u, window=5, eps=eps)
    rng = np.random.default_rng(24)
    for _ in range(12):
        c, z, y, x = rng.integers(0, 3), rng.integers(0, D), rng.integers(0, H), rng.integers(0, W)
        up, um = u.copy(), u.copy()
        up[c, z, y, x] = np.float32(u[c, z, y, x] + np.float32(1e-3))
        um[c, z, y, x] = np.float32(u[c, z, y, x] - np.float32(1e-3))
        h = float(up[c, z, y, x]) - float(um[c, z, y, x])
        lp, _ = orc.lncc(F, M, up, window=5, eps=eps, with_grad=False)
        lm, _ = orc.lncc(F, M, um, window=5, eps=eps, with_grad=False)
        fd = (lp - lm) / h
        assert abs(fd - g[c, z, y, x]) <= 1e-5 * np.abs(g).max() + 1e-7 * abs(fd), (c, z, y, x, fd, g[c, z, y, x])


def test_sampled_gradient_agrees_with_full_gradient(orc):
    D, H, W = 10, 9, 8
    F = synth.random_volume((D, H, W), 25).numpy()
    M = synth.random_volume((D, H, W), 26).numpy()
    u = synth.random_disp((D, H, W), 27, 2.0).numpy()
    roi = np.array([1, 9, 2, 7, 0, 8])
    for ants in (False, True):
        _, g = orc.lncc(F, M, u, roi=roi, window=5, eps=1e-5, ants=ants)
        idx = np.array([[0, 0, 0], [9, 8, 7], [5, 4, 3], [1, 2, 0], [8, 6, 7], [4, 0, 5]])
        s = orc.lncc_grad_u_at(F, M, u, idx, roi=roi, window=5, eps=1e-5, ants=ants)
        for j, (z, y, x) in enumerate(idx):
            np.testing.assert_allclose(s[j], g[:, z, y, x], rtol=1e-12, atol=1e-18)


def test_gradient_vanishes_far_from_roi(orc):
    D, H, W = 12, 6, 6
    F = synth.random_volume((D, H, W), 28).numpy()
    M = synth.random_volume((D, H, W), 29).numpy()
    roi = np.array([0, 4, 0, 6, 0, 6])
    _, g = orc.lncc(F, M, None, roi=roi, window=3, eps=1e-5)
    assert np.all(g[:, 5:] == 0.0) and np.any(g[:, 4] != 0.0)


# ---------------------------------------------------------------- ANTs mode --
# App. "ANTs gradient approximation": the backward skips the window sums of
# the gamma family, i.e. dL/dMw_k = F_k gamma_k - Mw_k gamma_AC,k + gamma_MF,k
# with voxel k's own factors.  Written out, that is a_k (F_k - muF_k) -
# c_k (Mw_k - muM_k) with a_k = 2 g A_k / D_k, c_k = 2 g A_k^2 B_k / D_k^2,
# which is exactly g w^3 dn_k/dMw_k: w^3 times the derivative of voxel k's
# own LNCC term with respect to its own warped value (the other voxels'
# terms, which the exact gradient sums over the window, are left out).

def _ants_case(seed, shape=(8, 8, 8), scale=2.0):
    F = synth.random_volume(shape, seed).numpy()
    M = synth.random_volume(shape, seed + 1).numpy()
    u = synth.random_disp(shape, seed + 2, scale).numpy()
    return F, M, u


@pytest.mark.parametrize("w,roi", [(3, None), (5, ((1, 7), (2, 8), (0, 8))), (7, None)])
def test_ants_gradient_is_self_term_derivative(orc, w, roi):
    """Central differences of the single-voxel-ROI loss 1 - n_k in Mw_k
    (the forward map, pinned above against library box means) give
    dn_k/dMw_k; the ANTs gradient must be -w^3/N_roi times it, times the
    sampler derivative dMw/dp."""
    F, M, u = _ants_case(300 + w)
    D, H, W = F.shape
    eps = 1e-3
    rt = _roi_tuple(roi)
    _, g = orc.lncc(F, M, u, roi=rt, window=w, eps=eps, ants=True)
    Mw, dMw = orc.warp(M, u, with_grad=True)
    nroi = D * H * W if roi is None else np.prod([b - a for a, b in roi])
    rng = np.random.default_rng(310 + w)
    inside = 0
    for _ in range(24):
        z, y, x = (int(rng.integers(0, n)) for n in (D, H, W))
        in_roi = roi is None or all(a <= c < b for c, (a, b) in zip((z, y, x), roi))
        if not in_roi:
            assert np.all(g[:, z, y, x] == 0.0)
            continue
        inside += 1
        one = np.array([z, z + 1, y, y + 1, x, x + 1])
        h = 1e-4
        mp, mm = Mw.copy(), Mw.copy()
        mp[z, y, x] += h
        mm[z, y, x] -= h
        dl = (orc.lncc_loss_mw(F, mp, roi=one, window=w, eps=eps) -
              orc.lncc_loss_mw(F, mm, roi=one, window=w, eps=eps)) / (2 * h)  # = -dn_k/dMw_k
        s = (w ** 3) * dl / nroi  # = -(1/N_roi) w^3 dn_k/dMw_k
        ref = s * dMw[:, z, y, x]
        np.testing.assert_allclose(g[:, z, y, x], ref, rtol=1e-6, atol=1e-9 * np.abs(g).max())
    assert inside >= 8


def test_ants_gradient_matches_library_box_means(orc):
    """The same mode through avg_pool3d statistics and grid_sample's
    derivative: a_k (F_k - muF_k) - c_k (Mw_k - muM_k) on the ROI, zero off it."""
    F, M, u = _ants_case(320, shape=(8, 9, 10))
    w, eps = 5, 1e-4
    roi = ((1, 7), (0, 8), (2, 9))
    _, g = orc.lncc(F, M, u, roi=_roi_tuple(roi), window=w, eps=eps, ants=True)
    r = (w - 1) // 2

    def box(t):
        return tf.avg_pool3d(t[None, None], w, stride=1, padding=r, count_include_pad=True)[0, 0]

    Ft = torch.from_numpy(F.astype(np.float64))
    ut = torch.from_numpy(u.astype(np.float64)).requires_grad_(True)
    Mw = _grid_sample(torch.from_numpy(M.astype(np.float64)), ut)
    dMw = torch.stack(torch.autograd.grad(Mw.sum(), ut)[0].unbind(0))  # dMw/dp per channel (voxel-local)
    Mw = Mw.detach()
    muF, muM = box(Ft), box(Mw)
    A = box(Ft * Mw) - muF * muM
    B = box(Ft * Ft) - muF * muF
    C = box(Mw * Mw) - muM * muM
    Dn = B * C + eps
    nroi = np.prod([b - a for a, b in roi])
    gi = -1.0 / nroi
    s = 2 * gi * A / Dn * (Ft - muF) - 2 * gi * A * A * B / (Dn * Dn) * (Mw - muM)
    mask = torch.zeros_like(s)
    mask[tuple(slice(a, b) for a, b in roi)] = 1.0
    ref = (s * mask)[None] * dMw
    np.testing.assert_allclose(g, ref.numpy(), rtol=0, atol=1e-10 * np.abs(g).max())
