"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: the 512^3 pair and the 1040^3 pair with its 8-voxel halo
(ROI [8, 1032)^3, the windowed 32-bit addressing path).  The oracle cannot
take these volumes whole in seconds, so it checks

* the LNCC dloss/du at 64+ sampled voxels (w = 5; w = 7 and w = 11, the
  latter through the separable FP64 passes, at 16 of them), from crops: the adjoint at voxel
  k depends on F, M and u within 2r + |u| + 1 of k and is linear in
  1/N_roi, so the oracle run on a crop (with the crop's share of the ROI)
  times N_roi(crop) / N_roi(full) is the full-volume value.  The samples
  sit on the 32 x 16 tile seams, the z-chunk seams of the launch, the array
  faces and the ROI faces, plus seeded random voxels;
* the MI dloss/du (exact Parzen and approximate estimators) at sampled
  voxels: the oracle forms the joint PMF of the whole ROI by sampling on the
  fly (mi_pmf) and evaluates the adjoint formula at each sampled voxel with
  it; the full-ROI PMF itself is compared too;
* the loss and the joint PMF of sub-ROI boxes, against the oracle on a crop
  holding the box plus the window and displacement reach, the LNCC loss
  through its FP64 block partials (the mean of n_i, which is 1 - L) so that
  the check keeps its strength where L is close to 1;
and, at any size, that the full-ROI LNCC loss and MI histogram are the
voxel-weighted combinations of those of the eight ROI octants."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2509_25044_amd import ops, synth
from paper_2509_25044_amd.configs import C3, C5
from parity_util import assert_loss

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
REACH = 12  # >= max displacement (8) + 1 + the window radius (2)


def _roi6(roi):
    return np.array([roi[0][0], roi[0][1], roi[1][0], roi[1][1], roi[2][0], roi[2][1]], dtype=np.int64)


def _nvox(roi):
    return int(np.prod([b - a for a, b in roi]))


def _crop(t, lo, hi):
    return t[..., lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].cpu().numpy()


def _crop_bounds(lo_box, hi_box, shape, reach):
    lo = [max(a - reach, 0) for a in lo_box]
    hi = [min(b + reach, n) for b, n in zip(hi_box, shape)]
    return lo, hi


def _rel_roi(roi, lo, hi):
    """The part of roi inside the crop [lo, hi), in crop coordinates."""
    return tuple((max(a, l) - l, min(b, h) - l) for (a, b), l, h in zip(roi, lo, hi))


def _pair(wl):
    g = synth.make_pair(wl.pair, seed=2025, device=DEV)
    F, M = g["F"], g["M"]
    u = (-0.6 * g["d"]).contiguous()
    del g
    torch.cuda.synchronize()
    return F, M, u


def _octants(roi):
    mids = [(a + b) // 2 for a, b in roi]
    out = []
    for kz in range(2):
        for ky in range(2):
            for kx in range(2):
                out.append(tuple(((a, m) if k == 0 else (m, b)) for (a, b), m, k in zip(roi, mids, (kz, ky, kx))))
    return out


def _adjoint_zchunk(shape, window=5):
    """z-chunk length of the fused adjoint's launch: the library's planner
    (32 x 16 tiles, two resident blocks per CU on 256 CUs for windows up to 5,
    the chunk count minimising rounds x (chunk + 2 * 2r) over chunks of >= 16
    slices), restated only to put sampled voxels on the chunk seams."""
    D, H, W = shape
    r = (window - 1) // 2
    tiles = math.ceil(W / 32) * math.ceil(H / 16)
    slots = 256 * (2 if window <= 5 else 1)
    best, bz = None, D
    for c in range(1, min(max(1, D // 16), 64) + 1):
        zc = math.ceil(D / c)
        nc = math.ceil(D / zc)
        cost = math.ceil(tiles * nc / slots) * (zc + 4 * r)
        if best is None or cost < best:
            best, bz = cost, zc
    return bz


def _samples(shape, roi, n_random, seed):
    """Sampled voxels: tile seams in x (32k - 1, 32k) and y (16k - 1, 16k),
    z-chunk seams, array and ROI faces, corners, and seeded random voxels."""
    D, H, W = shape
    zc = _adjoint_zchunk(shape)
    xs = sorted({v for k in (1, 2, W // 64, W // 32 - 1) for v in (32 * k - 1, 32 * k) if 0 <= v < W} |
                {0, W - 1, roi[2][0], roi[2][1] - 1})
    ys = sorted({v for k in (1, 2, H // 32, H // 16 - 1) for v in (16 * k - 1, 16 * k) if 0 <= v < H} |
                {0, H - 1, roi[1][0], roi[1][1] - 1})
    zs = sorted({v for k in range(1, 4) for v in (k * zc - 1, k * zc) if 0 <= v < D} |
                {0, D - 1, roi[0][0], roi[0][1] - 1, D // 2})
    rng = np.random.default_rng(seed)
    pts = set()
    for z in zs:  # every z seam with x and y seams, cycled
        for i, x in enumerate(xs):
            pts.add((z, ys[(i + len(pts)) % len(ys)], x))
    for _ in range(n_random):
        pts.add((int(rng.integers(D)), int(rng.integers(H)), int(rng.integers(W))))
    for c in ((0, 0, 0), (D - 1, H - 1, W - 1), (0, H - 1, W // 2), (D - 1, 0, 31)):
        pts.add(c)
    return sorted(pts), zc


def _table_slack(Fh, Mh, uh, k, dt, n_full, B=32):
    """Bound on the MI gradient difference at voxel k that log-table
    differences dt can cause (the oracle's warp of a crop around k)."""
    lo, hi = _crop_bounds(k, [c + 1 for c in k], Fh.shape, REACH)
    sl = tuple(slice(a, b) for a, b in zip(lo, hi))
    mw, dmw = oracle.warp(np.ascontiguousarray(Mh[sl]), np.ascontiguousarray(uh[(slice(None),) + sl]),
                          with_grad=True)
    j = tuple(c - a for c, a in zip(k, lo))
    kf, _ = oracle.parzen(float(Fh[k]), B)
    _, om = oracle.parzen(float(mw[j]), B)
    return np.abs(dmw[(slice(None),) + j]).max() / n_full * float(kf @ dt @ np.abs(om))


def _similarity_mean(F, M, u, roi, window=5):
    """Mean of n_i over the ROI from the forward call's FP64 block partials
    (1 - L without the fp32 rounding of L)."""
    ws = torch.zeros(ops.lncc_workspace_bytes(F.shape, roi, window), dtype=torch.uint8, device=DEV)
    ops.warp_lncc_fwd(F, M, u, window=window, roi=roi, ws=ws)
    torch.cuda.synchronize()
    return float(ws.view(torch.float64).sum().item()) / _nvox(roi)


def _check(wl, box, n_random):
    shape = wl.shape
    roi = wl.roi if wl.roi is not None else tuple((0, n) for n in shape)
    print(f"[fullsize {wl.name}: generating]", flush=True)
    F, M, u = _pair(wl)
    n_full = _nvox(roi)
    samples, zc = _samples(shape, roi, n_random, seed=len(shape) + shape[0])
    assert len(samples) >= 64

    print(f"[fullsize {wl.name}: lncc adjoint at {len(samples)} sampled voxels, z-chunk {zc}]", flush=True)
    g, loss = ops.warp_lncc_bwd(F, M, u, window=5, roi=roi)
    got_all = g[:, [k[0] for k in samples], [k[1] for k in samples], [k[2] for k in samples]].double().cpu().numpy().T
    del g
    refs = []
    for k in samples:
        lo, hi = _crop_bounds(k, [c + 1 for c in k], shape, 2 * REACH)
        croi = _rel_roi(roi, lo, hi)
        if any(b <= a for a, b in croi):  # the crop holds none of the ROI: no window of it reaches k
            refs.append(np.zeros(3))
            continue
        ref = oracle.lncc_grad_u_at(_crop(F, lo, hi), _crop(M, lo, hi), _crop(u, lo, hi),
                                    [[k[0] - lo[0], k[1] - lo[1], k[2] - lo[2]]], roi=_roi6(croi), window=5)[0]
        refs.append(ref * _nvox(croi) / n_full)
    refs = np.array(refs)
    scale = np.abs(refs).max()
    assert scale > 0
    err = np.abs(got_all - refs).max(axis=1)
    bad = [(samples[i], got_all[i], refs[i]) for i in np.nonzero(err > 1e-4 * scale)[0]]
    assert not bad, bad[:5]

    # w = 7 (the 32 x 24-tile adjoint) and w = 11 (the separable FP64
    # passes of the wide windows) at 16 of the samples, the crops widened by
    # the larger window radius
    sw = samples[:: max(1, len(samples) // 16)]
    for win in (7, 11):
        print(f"[fullsize {wl.name}: w = {win} adjoint at {len(sw)} sampled voxels]", flush=True)
        g, _ = ops.warp_lncc_bwd(F, M, u, window=win, roi=roi)
        got_w = g[:, [k[0] for k in sw], [k[1] for k in sw], [k[2] for k in sw]].double().cpu().numpy().T
        del g
        torch.cuda.empty_cache()
        refs = []
        for k in sw:
            lo, hi = _crop_bounds(k, [c + 1 for c in k], shape, 2 * (REACH + (win - 5) // 2))
            croi = _rel_roi(roi, lo, hi)
            if any(b <= a for a, b in croi):
                refs.append(np.zeros(3))
                continue
            ref = oracle.lncc_grad_u_at(_crop(F, lo, hi), _crop(M, lo, hi), _crop(u, lo, hi),
                                        [[k[0] - lo[0], k[1] - lo[1], k[2] - lo[2]]], roi=_roi6(croi), window=win)[0]
            refs.append(ref * _nvox(croi) / n_full)
        refs = np.array(refs)
        scale = np.abs(refs).max()
        assert scale > 0
        err = np.abs(got_w - refs).max(axis=1)
        bad = [(sw[i], got_w[i], refs[i]) for i in np.nonzero(err > 1e-4 * scale)[0]]
        assert not bad, (win, bad[:5])

    print(f"[fullsize {wl.name}: MI adjoint at sampled voxels, full-ROI PMF]", flush=True)
    Fh, Mh, uh = F.cpu().numpy(), M.cpu().numpy(), u.cpu().numpy()
    for mode, name in ((0, False), (2, "approx")):
        ml, st = ops.warp_mi_fwd(F, M, u, bins=32, roi=roi, hard=name)
        gm = ops.warp_mi_bwd(F, M, u, st, bins=32, roi=roi, hard=name)
        got = gm[:, [k[0] for k in samples], [k[1] for k in samples], [k[2] for k in samples]].double().cpu().numpy().T
        del gm
        p_gpu = st[1024:2048].double().cpu().numpy().reshape(32, 32)
        # 16 fp32 ulps of 1: the fp32 trilinear value can differ from the
        # float64 one by less than that (reading P1)
        p_ref, n_edge = oracle.mi_pmf(Fh, Mh, uh, roi=_roi6(roi), bins=32, hard=mode, edge_tol=16 * 2.0 ** -24,
                                      with_edges=True)
        ref = oracle.mi_grad_u_at(Fh, Mh, uh, samples, p_ref, roi=_roi6(roi), bins=32, hard=mode)
        if mode == 0:
            np.testing.assert_allclose(p_gpu, p_ref, rtol=1e-5, atol=1e-9)
            slack = np.zeros(len(samples))
        else:
            # each voxel near a bin edge moves at most 1/N_roi of count
            print(f"  approx: {n_edge} ROI voxels within fp32 rounding of a bin edge", flush=True)
            np.testing.assert_allclose(p_gpu, p_ref, rtol=1e-5, atol=1e-9 + 2.0 * n_edge / n_full)
            # the log tables T = log p - log p_M of the two sides then differ
            # by dt; the gradient at voxel k can differ by at most
            # |dMw/dp| / N_roi * sum_ab kappa_a(F_k) |omega_b(Mw_k)| dt[a, b]
            t_gpu = st[:1024].double().cpu().numpy().reshape(32, 32)
            pm = p_ref.sum(axis=0)
            with np.errstate(divide="ignore", invalid="ignore"):
                t_ref = np.where(p_ref > 0, np.log(p_ref) - np.log(pm)[None, :], 0.0)
            dt = np.abs(t_gpu - t_ref)
            slack = np.array([_table_slack(Fh, Mh, uh, k, dt, n_full) for k in samples])
        sc = np.abs(ref).max()
        assert sc > 0
        err = np.abs(got - ref).max(axis=1)
        bad = [(samples[i], got[i], ref[i], slack[i]) for i in np.nonzero(err > 1e-4 * sc + slack)[0]]
        assert not bad, (name, bad[:5])
        if mode == 2:
            assert (slack > 1e-4 * sc).mean() <= 0.1, "too many samples read log-table entries that differ"
    del Fh, Mh, uh

    print(f"[fullsize {wl.name}: sub-ROI loss and PMF]", flush=True)
    lo_b, hi_b = box
    sub = tuple(zip(lo_b, hi_b))
    lo, hi = _crop_bounds(lo_b, hi_b, shape, REACH)
    croi = _roi6(_rel_roi(sub, lo, hi))
    Fc, Mc, uc = _crop(F, lo, hi), _crop(M, lo, hi), _crop(u, lo, hi)
    l_gpu = float(ops.warp_lncc_fwd(F, M, u, window=5, roi=sub).item())
    l_ref, _ = oracle.lncc(Fc, Mc, uc, roi=croi, window=5, with_grad=False)
    assert_loss(l_gpu, l_ref, f"{wl.name} sub-ROI lncc")
    s_gpu = _similarity_mean(F, M, u, sub)
    assert abs(s_gpu - (1.0 - l_ref)) <= 1e-5 * abs(1.0 - l_ref), (s_gpu, 1.0 - l_ref)
    for mode, name in ((0, False), (2, "approx")):
        ml, st = ops.warp_mi_fwd(F, M, u, bins=32, roi=sub, hard=name)
        mr, pr, _ = oracle.mi(Fc, Mc, uc, roi=croi, bins=32, hard=mode, with_grad=False)
        assert_loss(float(ml.item()), mr, f"{wl.name} sub-ROI mi mode {mode}")
        atol = 1e-9 if mode == 0 else 4.0 / _nvox(sub)
        np.testing.assert_allclose(st[1024:2048].double().cpu().numpy().reshape(32, 32), pr, rtol=1e-5, atol=atol)

    print(f"[fullsize {wl.name}: octant additivity]", flush=True)
    octs = _octants(roi)
    w = np.array([_nvox(o) for o in octs], dtype=np.float64) / n_full
    parts = [_similarity_mean(F, M, u, o) for o in octs]
    s_full = _similarity_mean(F, M, u, roi)
    assert abs(float(np.dot(w, parts)) - s_full) <= 1e-9 * abs(s_full), (float(np.dot(w, parts)), s_full)
    assert abs((1.0 - s_full) - float(loss.item())) <= 1e-6 * abs(float(loss.item()))
    _, st_full = ops.warp_mi_fwd(F, M, u, bins=32, roi=roi)
    p_full = st_full[1024:2048].double()
    p_oct = sum(wi * ops.warp_mi_fwd(F, M, u, bins=32, roi=o)[1][1024:2048].double() for wi, o in zip(w, octs))
    assert float((p_full - p_oct).abs().max()) <= 1e-6 * float(p_full.max())


def test_fullsize_512cube():
    _check(C3, ((224, 240, 200), (288, 304, 264)), n_random=40)


def test_fullsize_1040cube_halo_roi():
    _check(C5, ((480, 500, 520), (544, 564, 584)), n_random=24)
