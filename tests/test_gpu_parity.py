"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Sizes stay where the oracle finishes in seconds but span several 64 x 16
tiles, z-chunks and ragged tails; edge cases cover single voxels, ROIs, the
zero-padding sampler, NaN propagation and determinism.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2509_25044_amd import ops, synth
from paper_2509_25044_amd.configs import C1, C2
from parity_util import assert_grad, assert_loss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(t):
    return t.to(DEV).contiguous()


def _np(t):
    return t.detach().cpu().numpy()


def _roi6(roi):
    return None if roi is None else np.array([roi[0][0], roi[0][1], roi[1][0], roi[1][1], roi[2][0], roi[2][1]])


@pytest.fixture(scope="module")
def c1():
    p = synth.make_pair(C1.pair, seed=2025)
    u = (-0.6 * p["d"]).contiguous()
    return p["F"], p["M"], u


@pytest.fixture(scope="module")
def c2():
    p = synth.make_pair(C2.pair, seed=2025)
    u = (-0.6 * p["d"]).contiguous()
    return p["F"], p["M"], u


def _rand_case(shape, seed, scale=2.0):
    F = synth.random_volume(shape, seed)
    M = synth.random_volume(shape, seed + 1)
    u = synth.random_disp(shape, seed + 2, scale)
    return F, M, u


# ------------------------------------------------------------------ warp ----
@pytest.mark.parametrize("shift", [(0, 0, 0), (3, -2, 1), (-7, 5, 11)])
def test_warp_integer_shift_bitwise(shift):
    print(f"[warp int shift {shift}]", flush=True)
    F, M, _ = _rand_case((19, 23, 70), 100)
    u = torch.zeros((3, 19, 23, 70))
    for c in range(3):
        u[c] = shift[c]
    out = _np(ops.warp(_dev(M), _dev(u)))
    ref = oracle.warp(M.numpy(), u.numpy())
    assert np.array_equal(out.astype(np.float64), ref)


@pytest.mark.parametrize("pad", ["border", "zeros"])
def test_warp_random_field(pad):
    print(f"[warp random {pad}]", flush=True)
    F, M, u = _rand_case((21, 33, 130), 110, scale=4.0)
    out = _np(ops.warp(_dev(M), _dev(u), pad=pad))
    ref = oracle.warp(M.numpy(), u.numpy(), pad=1 if pad == "zeros" else 0)
    np.testing.assert_allclose(out, ref, rtol=0, atol=2e-6)


def test_resample_matches_oracle():
    print("[resample]", flush=True)
    src = synth.random_disp((10, 12, 14), 120, 3.0)
    out = _np(ops.resample(_dev(src), (20, 24, 28), value_scale=2.0))
    ref = oracle.resample(src.numpy(), (20, 24, 28), value_scale=2.0)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-5)
    down = _np(ops.resample(_dev(src), (5, 6, 7), value_scale=0.5))
    np.testing.assert_allclose(down, oracle.resample(src.numpy(), (5, 6, 7), 0.5), rtol=0, atol=1e-5)


# ------------------------------------------------------------------ LNCC ----
def _lncc_case(F, M, u, window=5, eps=1e-5, ants=False, pad="border", roi=None, what=""):
    print(f"[lncc {what} shape={tuple(F.shape)} w={window} ants={ants} pad={pad} roi={roi}]", flush=True)
    Fd, Md = _dev(F), _dev(M)
    ud = None if u is None else _dev(u)
    nws = ops.lncc_workspace_bytes(F.shape, roi, window)
    wsf = torch.zeros(nws, dtype=torch.uint8, device=DEV)
    wsb = torch.zeros(nws, dtype=torch.uint8, device=DEV)
    lf = float(ops.warp_lncc_fwd(Fd, Md, ud, window=window, eps=eps, pad=pad, roi=roi, ws=wsf).item())
    g, lb = ops.warp_lncc_bwd(Fd, Md, ud, window=window, eps=eps, ants=ants, pad=pad, roi=roi, ws=wsb)
    lb = float(lb.item())
    lr, gr = oracle.lncc(F.numpy(), M.numpy(), None if u is None else u.numpy(), roi=_roi6(roi), window=window,
                         eps=eps, ants=ants, pad=1 if pad == "zeros" else 0)
    assert_loss(lf, lr, f"{what} fwd")
    assert_loss(lb, lr, f"{what} bwd")
    # the FP64 block partials hold sum n_i: the mean similarity 1 - L without
    # the fp32 rounding of L (the strong form of the check where L is near 1)
    nroi = np.prod([b - a for a, b in roi]) if roi is not None else F.numel()
    # fused windows: the workspace is the block partials (and a zero flag);
    # wide windows: 8 N doubles of window sums and fields come first
    first = 8 * F.numel() if window > 9 else 0
    for name, ws in (("fwd", wsf), ("bwd", wsb)):
        sim = float(ws.view(torch.float64)[first:(nws - 16) // 8].sum().item()) / nroi
        assert abs(sim - (1.0 - lr)) <= 1e-5 * abs(1.0 - lr) + 1e-9, f"{what} {name} similarity {sim} vs {1.0 - lr}"
    assert_grad(_np(g), gr, f"{what} grad")


@pytest.mark.parametrize("window", [3, 5, 7, 9])
def test_lncc_c1_pair(c1, window):
    F, M, u = c1
    _lncc_case(F, M, u, window=window, what="c1")


def test_lncc_c1_zero_displacement_and_self(c1):
    F, M, u = c1
    _lncc_case(F, M, None, window=5, what="c1 u=None")
    # F against itself at u = 0 and eps = 0: LNCC = 1 everywhere -> loss 0
    l = float(ops.warp_lncc_fwd(_dev(F), _dev(F), None, window=5, eps=0.0).item())
    assert abs(l) < 1e-5


def test_lncc_c1_ants(c1):
    F, M, u = c1
    _lncc_case(F, M, u, window=5, ants=True, what="c1 ants")


def test_lncc_c1_zeros_pad_and_roi(c1):
    F, M, u = c1
    _lncc_case(F, M, u * 3.0, window=5, pad="zeros", what="c1 zeros")
    _lncc_case(F, M, u, window=5, roi=((8, 56), (3, 61), (10, 50)), what="c1 roi")


def test_lncc_c2_clinical_window7(c2):
    F, M, u = c2
    _lncc_case(F, M, u, window=7, what="c2")


@pytest.mark.parametrize("window", [11, 13, 15])
def test_lncc_wide_windows_c1(c1, window):
    """Windows past the fused kernel's register rings: the separable FP64
    passes, forward and exact adjoint."""
    F, M, u = c1
    _lncc_case(F, M, u, window=window, what="c1 wide")


def test_lncc_wide_window_modes(c1):
    F, M, u = c1
    _lncc_case(F, M, u, window=13, ants=True, what="c1 wide ants")
    _lncc_case(F, M, u * 3.0, window=11, pad="zeros", what="c1 wide zeros")
    _lncc_case(F, M, u, window=15, roi=((8, 56), (3, 61), (10, 50)), what="c1 wide roi")
    _lncc_case(F, M, None, window=15, what="c1 wide u=None")
    l = float(ops.warp_lncc_fwd(_dev(F), _dev(F), None, window=15, eps=0.0).item())
    assert abs(l) < 1e-6


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 7), (37, 45, 70), (20, 17, 130)])
def test_lncc_wide_ragged_shapes(shape):
    F, M, u = _rand_case(shape, 130)
    _lncc_case(F, M, u, window=15, eps=1e-5, what="ragged w15")
    _lncc_case(F, M, u, window=11, eps=1e-3, ants=True, what="ragged w11 ants")


def _wide_zchunk(shape):
    """z-chunk of the wide-window column passes (64 x 4 columns per block,
    about 4096 blocks, chunks of at least 32 slices): the library's planner,
    restated only to put sampled voxels on the chunk seams."""
    D, H, W = shape
    cols = -(-W // 64) * -(-H // 4)
    want = max(1, min(-(-4096 // cols), max(1, D // 32)))
    return -(-D // want)


def test_lncc_wide_window_clinical_samples(c2):
    """w = 15 on the clinical pair: dloss/du at voxels on the slice-tile seams
    (32 x 32 tiles of the sampling pass, 32 x 16 of the a, c, e pass), the
    column passes' z-chunk seams, the faces and random voxels
    against the oracle's per-voxel adjoint on the whole arrays; the loss of a
    sub-ROI box against the oracle on the warped volume."""
    F, M, u = c2
    D, H, W = F.shape
    zc = _wide_zchunk(F.shape)
    rng = np.random.default_rng(77)
    pts = set()
    xs = [0, 31, 32, 63, 64, 127, 128, W - 1]
    ys = [0, 15, 16, 31, 32, 95, 96, 111, 112, H - 1]
    zs = sorted({0, D - 1, D // 2} | {v for k in (1, 2) for v in (k * zc - 1, k * zc) if 0 <= v < D})
    for i, z in enumerate(zs):
        for j, x in enumerate(xs):
            pts.add((z, ys[(i + j) % len(ys)], x))
    for _ in range(16):
        pts.add((int(rng.integers(D)), int(rng.integers(H)), int(rng.integers(W))))
    pts = sorted(pts)
    print(f"[lncc wide clinical: {len(pts)} samples, z-chunk {zc}]", flush=True)
    Fd, Md, ud = _dev(F), _dev(M), _dev(u)
    g, _ = ops.warp_lncc_bwd(Fd, Md, ud, window=15)
    got = g[:, [p[0] for p in pts], [p[1] for p in pts], [p[2] for p in pts]].double().cpu().numpy().T
    ref = oracle.lncc_grad_u_at(F.numpy(), M.numpy(), u.numpy(), pts, window=15)
    sc = np.abs(ref).max()
    assert sc > 0
    err = np.abs(got - ref).max(axis=1)
    bad = [(pts[i], got[i], ref[i]) for i in np.nonzero(err > 1e-4 * sc)[0]]
    assert not bad, bad[:5]
    box = ((60, 84), (90, 114), (100, 124))
    l_gpu = float(ops.warp_lncc_fwd(Fd, Md, ud, window=15, roi=box).item())
    mw = oracle.warp(M.numpy(), u.numpy())
    l_ref = oracle.lncc_loss_mw(F.numpy(), mw, roi=_roi6(box), window=15)
    assert_loss(l_gpu, l_ref, "clinical w15 sub-ROI")


@pytest.mark.parametrize("shape", [(1, 1, 1), (6, 7, 1), (6, 7, 2), (3, 5, 7), (2, 40, 3), (37, 45, 70), (20, 17, 130)])
def test_lncc_ragged_shapes(shape):
    F, M, u = _rand_case(shape, 130)
    _lncc_case(F, M, u, window=5, eps=1e-3, what="ragged")
    _lncc_case(F, M, u, window=5, eps=1e-5, what="ragged eps 1e-5")
    _lncc_case(F, M, u, window=7, eps=1e-5, what="ragged w7")
    _lncc_case(F, M, u, window=3, eps=1e-3, ants=True, what="ragged ants")


def test_lncc_deterministic(c1):
    F, M, u = (_dev(t) for t in c1)
    g1, l1 = ops.warp_lncc_bwd(F, M, u)
    g2, l2 = ops.warp_lncc_bwd(F, M, u)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_lncc_grad_scale_and_nan(c1):
    F, M, u = (_dev(t) for t in c1)
    g1, _ = ops.warp_lncc_bwd(F, M, u)
    s = torch.tensor([2.5], device=DEV)
    g2, _ = ops.warp_lncc_bwd(F, M, u, grad_scale=s)
    # the scale enters as dL/dn_i, so rounding differs from scaling afterwards
    assert_grad(_np(g2), _np(g1).astype(np.float64) * 2.5, "grad_scale")
    Fn = F.clone()
    Fn[10, 10, 10] = float("nan")
    l = ops.warp_lncc_fwd(Fn, M, u)
    assert torch.isnan(l).all()


# -------------------------------------------------------------------- MI ----
def _mi_case(F, M, u, bins=32, hard=False, pad="border", roi=None, what=""):
    print(f"[mi {what} shape={tuple(F.shape)} bins={bins} hard={hard} pad={pad} roi={roi}]", flush=True)
    Fd, Md = _dev(F), _dev(M)
    ud = None if u is None else _dev(u)
    loss, state = ops.warp_mi_fwd(Fd, Md, ud, bins=bins, hard=hard, pad=pad, roi=roi)
    g = ops.warp_mi_bwd(Fd, Md, ud, state, bins=bins, hard=hard, pad=pad, roi=roi)
    mode = 2 if hard == "approx" else int(bool(hard))
    lr, pr, gr = oracle.mi(F.numpy(), M.numpy(), None if u is None else u.numpy(), roi=_roi6(roi), bins=bins,
                           hard=mode, pad=1 if pad == "zeros" else 0)
    st = _np(state)
    B = bins
    nroi = np.prod([b - a for a, b in roi]) if roi is not None else F.numel()
    # Hard bins (box kernel, approximate estimator): both sides take the bin
    # of their own value exactly (floor of the exact product v B), so F's
    # bins agree.  The warped value is fp32 on the device and float64 in the
    # oracle; a voxel whose oracle value lies within the fp32 sampler's
    # rounding of a bin edge may land in the neighbouring bin.  Such voxels
    # are counted from the oracle's own values; each moves at most 2/N_roi of
    # mass between p entries and changes MI by at most ~100/N_roi (six p log p
    # terms with p >= 1/N_roi).  With none of them, parity is exact.
    namb = _edge_voxels(M, u, pad, roi, B) if (mode in (1, 2) and u is not None) else 0
    if namb:
        print(f"  {what}: {namb} ROI voxels within fp32 rounding of a bin edge", flush=True)
    lt = abs(float(loss.item()) - lr)
    if namb == 0:
        assert_loss(float(loss.item()), lr, f"{what} loss")
    else:
        assert lt <= 1e-5 * abs(lr) + 100.0 * namb / nroi, f"{what} loss {float(loss.item())} vs {lr}"
    atol = 1e-9 + 2.0 * namb / nroi
    np.testing.assert_allclose(st[B * B:2 * B * B].reshape(B, B), pr, rtol=1e-5, atol=atol)
    if mode == 1:
        assert float(g.abs().max()) == 0.0
    elif mode == 2 and u is not None:
        _mi_approx_grad(F, M, u, pad, roi, B, st, pr, _np(g), gr, nroi, what)
    else:
        assert_grad(_np(g), gr, f"{what} grad")


def _edge_voxels(M, u, pad, roi, B):
    """ROI voxels whose float64 warped value (clamped to [0, 1]) lies within
    16 fp32 ulps of 1 of an interior bin edge m / B: the fp32 trilinear
    value (seven rounded interpolations of values in [0, 1]) can differ from
    the float64 one by less than that."""
    mw = np.clip(oracle.warp(M.numpy(), u.numpy(), pad=1 if pad == "zeros" else 0), 0.0, 1.0)
    if roi is not None:
        mw = mw[tuple(slice(a, b) for a, b in roi)]
    t = mw * B
    k = np.round(t)
    near = (np.abs(t - k) <= 16 * 2.0 ** -24 * B) & (k > 0) & (k < B)
    return int(near.sum())


def _mi_approx_grad(F, M, u, pad, roi, B, st, pr, g, gr, nroi, what):
    """Approximate-mode gradient with a warped image.  A voxel whose warped
    value lies within fp32 rounding of a bin edge may be counted in the
    neighbouring bin on one side (the kernel forms the value in fp32, the
    oracle in float64), and each such decision changes p, and so the log
    table T = log p - log p_M, in the 3x3 bins around the two bins it moves
    between.  Both tables are then correct for their own counts.  The
    gradient is compared on the voxels where the two tables could move it by
    less than a tenth of the tolerance; the decisions that differ must be
    few, those voxels few, and every gradient finite."""
    dp = np.abs(st[B * B:2 * B * B].reshape(B, B).astype(np.float64) - pr)
    moved = 0.5 * dp.sum() * nroi  # voxels whose count moved, at least
    namb = _edge_voxels(M, u, pad, roi, B)
    assert moved <= namb + 1e-3, f"{what}: {moved:.1f} voxels change bins, {namb} lie near an edge"
    pm = pr.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t_orc = np.where(pr > 0, np.log(pr) - np.log(pm)[None, :], 0.0)
    dt = np.abs(st[:B * B].reshape(B, B).astype(np.float64) - t_orc)
    # bound on |g_gpu - g_ref| from dt alone at each voxel:
    # |dMw/dp| / N_roi * sum_ab kappa_a(F) |dkappa_b/dv(Mw)| dt[a, b]
    # over the 4x4 cubic B-spline patch (the kernel's form of the sum)
    mw, dmw = oracle.warp(M.numpy(), u.numpy(), pad=1 if pad == "zeros" else 0, with_grad=True)
    def patch(v):
        vc = np.clip(v, 0.0, 1.0)
        sv = vc * B - 0.5
        f = np.floor(sv)
        t = sv - f
        q = 1.0 - t
        w = np.stack([q ** 3 / 6, 0.5 * t ** 3 - t * t + 2.0 / 3, 0.5 * q ** 3 - q * q + 2.0 / 3, t ** 3 / 6])
        ds = np.where((v >= 0.0) & (v <= 1.0), float(B), 0.0)
        dw = np.abs(np.stack([-0.5 * q * q, 1.5 * t * t - 2 * t, -1.5 * q * q + 2 * q, 0.5 * t * t])) * ds
        return f.astype(np.int64) - 1, w, dw
    jf, wf, _ = patch(F.numpy().astype(np.float64))
    jm, _, dm = patch(mw)
    bound = np.zeros(F.shape)
    for a in range(4):
        for b in range(4):
            bound += wf[a] * dm[b] * dt[np.clip(jf + a, 0, B - 1), np.clip(jm + b, 0, B - 1)]
    bound *= np.abs(dmw).max(axis=0) / nroi
    if roi is not None:
        inside = np.zeros(F.shape, dtype=bool)
        inside[tuple(slice(a, b) for a, b in roi)] = True
        bound *= inside
    touch = bound > 1e-5 * np.abs(gr).max()
    assert np.all(np.isfinite(g)), f"{what}: non-finite gradient"
    frac = touch.mean()
    print(f"  {what}: >= {moved:.1f} voxels moved bins, {int((dt > 1e-5).sum())} log-table entries differ, "
          f"{frac:.5f} of the voxels could see it", flush=True)
    assert frac <= 0.02, f"{what}: {frac:.4f} of the voxels read a log-table entry that differs"
    keep = ~touch
    assert_grad(g * keep[None], gr * keep[None], f"{what} grad (voxels with agreeing tables, {1 - frac:.5f})")


def test_mi_c1_pair(c1):
    F, M, u = c1
    _mi_case(F, M, u, bins=32, what="c1")
    _mi_case(F, M, None, bins=8, what="c1 b8 u=None")


def test_mi_c2_multimodal(c2):
    F, M, u = c2
    _mi_case(F, M, u, bins=32, what="c2")


def test_mi_roi_zeros_hard(c1):
    F, M, u = c1
    _mi_case(F, M, u, bins=16, roi=((5, 60), (0, 64), (7, 33)), what="c1 roi")
    _mi_case(F, M, u * 3, bins=32, pad="zeros", what="c1 zeros")
    _mi_case(F, M, u, bins=32, hard=True, what="c1 hard")


def test_mi_approx_estimator(c1, c2):
    """The approximate histogram estimator: exact counts where the warped
    image is M itself (u = None), bin-edge tolerance otherwise, and the
    exact-kernel gradient at the approximate p."""
    F, M, u = c1
    _mi_case(F, M, None, bins=32, hard="approx", what="c1 approx u=None")
    _mi_case(F, M, None, bins=48, hard="approx", what="c1 approx u=None b48")
    _mi_case(F, M, u, bins=32, hard="approx", what="c1 approx")
    _mi_case(F, M, u, bins=16, hard="approx", roi=((5, 60), (0, 64), (7, 33)), what="c1 approx roi")
    _mi_case(F, M, u * 3, bins=32, hard="approx", pad="zeros", what="c1 approx zeros")
    F2, M2, u2 = c2
    _mi_case(F2, M2, u2, bins=32, hard="approx", what="c2 approx")


@pytest.mark.parametrize("bins", [8, 45, 47, 48, 64, 68, 69])
def test_mi_bin_counts_and_histogram_copies(c1, bins):
    """Bin counts on both sides of the LDS layout changes (4 histogram copies
    up to 47 bins, 2 copies up to 68, 1 above, 79 KB of LDS at 47 bins)."""
    F, M, u = c1
    _mi_case(F, M, u, bins=bins, what=f"c1 b{bins}")
    if bins in (45, 64):
        _mi_case(F, M, u, bins=bins, hard="approx", what=f"c1 approx b{bins}")


@pytest.mark.parametrize("bins", [90, 98, 99, 128, 129, 200, 256])
def test_mi_wide_histograms(bins):
    """Bin counts beyond the LDS-resident layouts: one u64 LDS histogram up to
    98 bins, global u64 atomics above; the approximate estimator's u32
    counts in LDS up to 128 bins, global above; the adjoint's log table in
    LDS up to 128 bins, read through the caches above."""
    F, M, u = _rand_case((24, 28, 36), 160 + bins)
    _mi_case(F, M, u, bins=bins, what=f"wide b{bins}")
    if bins in (90, 129, 200):  # the oracle's approximate p is a B^4 sum
        _mi_case(F, M, u, bins=bins, hard="approx", what=f"wide approx b{bins}")


def test_checked_mode(c1):
    """check_finite = 1: the same results on finite inputs; FFDP_ERR_NONFINITE
    for a NaN or infinite value in F, M, u or grad_scale, and for a NaN loss
    from finite inputs (eps = 0 on a constant image)."""
    from paper_2509_25044_amd._lib import FfdpError
    F, M, u = (_dev(t) for t in c1)
    g0, l0 = ops.warp_lncc_bwd(F, M, u)
    g1, l1 = ops.warp_lncc_bwd(F, M, u, check_finite=True)
    assert torch.equal(g0, g1) and torch.equal(l0, l1)
    assert torch.equal(ops.warp_lncc_fwd(F, M, u, check_finite=True), l0)
    m0, s0 = ops.warp_mi_fwd(F, M, u)
    m1, s1 = ops.warp_mi_fwd(F, M, u, check_finite=True)
    assert torch.equal(m0, m1) and torch.equal(s0, s1)
    assert torch.equal(ops.warp_mi_bwd(F, M, u, s1, check_finite=True), ops.warp_mi_bwd(F, M, u, s1))

    def refused(fn):
        with pytest.raises(FfdpError) as e:
            fn()
        assert e.value.code == 7, e.value
    Fn = F.clone()
    Fn[3, 4, 5] = float("nan")
    un = u.clone()
    un[1, 10, 11, 12] = float("inf")
    Mn = M.clone()
    Mn[60, 1, 2] = -float("inf")
    refused(lambda: ops.warp_lncc_fwd(Fn, M, u, check_finite=True))
    refused(lambda: ops.warp_lncc_bwd(F, M, un, check_finite=True))
    refused(lambda: ops.warp_lncc_bwd(F, M, u, grad_scale=torch.tensor([float("nan")], device=DEV),
                                      check_finite=True))
    refused(lambda: ops.warp_mi_fwd(F, Mn, u, check_finite=True))
    refused(lambda: ops.warp_mi_bwd(F, M, un, s1, check_finite=True))
    C = torch.full_like(F, 0.5)
    l_nan = ops.warp_lncc_fwd(C, C, None, eps=0.0)  # unchecked: a NaN loss, no error
    assert torch.isnan(l_nan).all()
    refused(lambda: ops.warp_lncc_fwd(C, C, None, eps=0.0, check_finite=True))


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 9, 1), (4, 6, 2), (3, 5, 7), (37, 45, 70)])
def test_mi_ragged_shapes(shape):
    F, M, u = _rand_case(shape, 140)
    _mi_case(F, M, u, bins=16, what="ragged")


def test_mi_self_information_and_determinism(c1):
    F = _dev(c1[0])
    loss, state = ops.warp_mi_fwd(F, F, None, bins=32, hard=True)
    B = 32
    pF = _np(state)[2 * B * B:2 * B * B + B].astype(np.float64)
    H = -(pF[pF > 0] * np.log(pF[pF > 0])).sum()
    assert abs(-float(loss.item()) - H) < 1e-5 * H
    F, M, u = (_dev(t) for t in c1)
    l1, s1 = ops.warp_mi_fwd(F, M, u)
    l2, s2 = ops.warp_mi_fwd(F, M, u)
    assert torch.equal(l1, l2) and torch.equal(s1, s2)
    g1 = ops.warp_mi_bwd(F, M, u, s1)
    g2 = ops.warp_mi_bwd(F, M, u, s1)
    assert torch.equal(g1, g2)


# ------------------------------------------------------------------ Adam ----
@pytest.mark.parametrize("n,offset", [(1_000_003, 0), (4099, 1), (7, 0)])
def test_adam_matches_oracle(n, offset):
    print(f"[adam n={n} offset={offset}]", flush=True)
    rng = np.random.default_rng(150)
    x0 = rng.normal(size=n + offset).astype(np.float32)
    xd = torch.from_numpy(x0).to(DEV)
    md = torch.zeros_like(xd)
    vd = torch.zeros_like(xd)
    xr, mr, vr = x0[offset:].astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = (rng.normal(size=n + offset) * 10.0 ** rng.integers(-3, 2)).astype(np.float32)
        gd = torch.from_numpy(g).to(DEV)
        ops.adam_step(xd[offset:], gd[offset:], md[offset:], vd[offset:], lr=0.1, step=step)
        oracle.adam(xr, g[offset:].astype(np.float64), mr, vr, lr=0.1, step=step)
    np.testing.assert_allclose(_np(xd)[offset:], xr, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(_np(md)[offset:], mr, rtol=2e-6, atol=1e-6 * np.abs(mr).max())
