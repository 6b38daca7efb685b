"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: the 512^3 pair and the 1040^3 pair with its 8-voxel halo
(ROI [8, 1032)^3, the 64-bit gather path).  The oracle cannot take these
volumes whole in seconds, so it checks

* dloss/du at sampled voxels, from crops: the adjoint at voxel k depends on
  F, M and u within 2r + |u| + 1 of k and is linear in 1/N_roi, so the
  oracle run on a crop (with the crop's share of the ROI) times
  N_roi(crop) / N_roi(full) is the full-volume value;
* the loss and the joint PMF of sub-ROI boxes, against the oracle on a crop
  holding the box plus the window and displacement reach;
and, at any size, that the full-ROI LNCC loss and MI histogram are the
voxel-weighted combinations of those of the eight ROI octants."""
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


def _check(wl, samples, box):
    shape = wl.shape
    roi = wl.roi if wl.roi is not None else tuple((0, n) for n in shape)
    print(f"[fullsize {wl.name}: generating]", flush=True)
    F, M, u = _pair(wl)
    n_full = _nvox(roi)

    print(f"[fullsize {wl.name}: lncc adjoint at {len(samples)} sampled voxels]", flush=True)
    g, loss = ops.warp_lncc_bwd(F, M, u, window=5, roi=roi)
    for k in samples:
        lo, hi = _crop_bounds(k, [c + 1 for c in k], shape, 2 * REACH)
        croi = _rel_roi(roi, lo, hi)
        ref = oracle.lncc_grad_u_at(_crop(F, lo, hi), _crop(M, lo, hi), _crop(u, lo, hi),
                                    [[k[0] - lo[0], k[1] - lo[1], k[2] - lo[2]]], roi=_roi6(croi), window=5)[0]
        ref = ref * _nvox(croi) / n_full
        got = g[:, k[0], k[1], k[2]].double().cpu().numpy()
        scale = max(np.abs(ref).max(), 1e-30)
        assert np.abs(got - ref).max() <= 1e-4 * scale + 1e-12, (k, got, ref)

    print(f"[fullsize {wl.name}: sub-ROI loss and PMF]", flush=True)
    lo_b, hi_b = box
    sub = tuple(zip(lo_b, hi_b))
    lo, hi = _crop_bounds(lo_b, hi_b, shape, REACH)
    croi = _roi6(_rel_roi(sub, lo, hi))
    Fc, Mc, uc = _crop(F, lo, hi), _crop(M, lo, hi), _crop(u, lo, hi)
    l_gpu = float(ops.warp_lncc_fwd(F, M, u, window=5, roi=sub).item())
    l_ref, _ = oracle.lncc(Fc, Mc, uc, roi=croi, window=5, with_grad=False)
    assert_loss(l_gpu, l_ref, f"{wl.name} sub-ROI lncc")
    for mode, name in ((0, False), (2, "approx")):
        ml, st = ops.warp_mi_fwd(F, M, u, bins=32, roi=sub, hard=name)
        mr, pr, _ = oracle.mi(Fc, Mc, uc, roi=croi, bins=32, hard=mode, with_grad=False)
        assert_loss(float(ml.item()), mr, f"{wl.name} sub-ROI mi mode {mode}")
        atol = 1e-9 if mode == 0 else 4.0 / _nvox(sub)
        np.testing.assert_allclose(st[1024:2048].double().cpu().numpy().reshape(32, 32), pr, rtol=1e-5, atol=atol)

    print(f"[fullsize {wl.name}: octant additivity]", flush=True)
    octs = _octants(roi)
    parts = [float(ops.warp_lncc_fwd(F, M, u, window=5, roi=o).item()) for o in octs]
    w = np.array([_nvox(o) for o in octs], dtype=np.float64) / n_full
    combined = 1.0 - float(np.dot(w, 1.0 - np.array(parts)))
    assert abs(combined - float(loss.item())) <= 1e-5 * abs(float(loss.item())), (combined, float(loss.item()))
    _, st_full = ops.warp_mi_fwd(F, M, u, bins=32, roi=roi)
    p_full = st_full[1024:2048].double()
    p_oct = sum(wi * ops.warp_mi_fwd(F, M, u, bins=32, roi=o)[1][1024:2048].double() for wi, o in zip(w, octs))
    assert float((p_full - p_oct).abs().max()) <= 1e-6 * float(p_full.max())


def test_fullsize_512cube():
    n = 512
    samples = [(0, 0, 0), (n - 1, n - 1, n - 1), (255, 256, 257), (3, 500, 129), (511, 17, 300), (100, 0, 511)]
    _check(C3, samples, ((224, 240, 200), (288, 304, 264)))


def test_fullsize_1040cube_halo_roi():
    samples = [(8, 8, 8), (1031, 1031, 1031), (7, 500, 500), (520, 519, 518), (1000, 9, 1030), (300, 1039, 700)]
    _check(C5, samples, ((480, 500, 520), (544, 564, 584)))
