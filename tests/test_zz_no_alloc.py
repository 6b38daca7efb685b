"""The entry point for callers that cannot allocate (ffdp_warp_lncc_bwd_noalloc),
called through the C ABI: its outputs equal those of ffdp_warp_lncc_bwd with a
caller workspace, bit for bit, on two calls in a row (the second on a smaller
grid, which reuses the library-owned scratch the first call left behind);
grids that need more block partials than the scratch holds are rejected
before anything runs.  A wide window (w = 15) on a small grid keeps its FP64
fields in the same scratch."""
import ctypes as C

import pytest
import torch

from paper_2509_25044_amd import _lib, ops, synth

DEV = "cuda:0"


def _grid(shape, roi=None):
    return ops.make_grid(shape, roi)


def test_noalloc_rejects_grids_beyond_its_scratch():
    L = _lib.lib()
    g = _grid((16, 8192, 8192))  # 256 x 512 tiles: more partials than the scratch holds
    p = ops.lncc_params(5)
    fake = C.c_void_p(0x10000)
    need = L.ffdp_lncc_workspace_bytes(C.byref(g), C.byref(p)) // 8
    assert need > 65536
    rc = L.ffdp_warp_lncc_bwd_noalloc(fake, fake, fake, C.byref(g), C.byref(p), None, fake, fake, None)
    assert rc == 5, rc
    assert b"scratch" in L.ffdp_last_error()
    # wide windows keep 64 bytes per voxel in the workspace: 64^3 does not fit
    g = _grid((64, 64, 64))
    p = ops.lncc_params(15)
    assert L.ffdp_lncc_workspace_bytes(C.byref(g), C.byref(p)) > 8 * 65538
    rc = L.ffdp_warp_lncc_bwd_noalloc(fake, fake, fake, C.byref(g), C.byref(p), None, fake, fake, None)
    assert rc == 5, rc
    assert b"scratch" in L.ffdp_last_error()


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry_point_twice():
    L = _lib.lib()
    stream = torch.cuda.current_stream(torch.device(DEV)).cuda_stream
    for k, (shape, roi, window, ants) in enumerate([((40, 56, 72), ((3, 37), (2, 50), (5, 70)), 5, 0),
                                                    ((30, 40, 50), None, 7, 0),
                                                    ((24, 32, 40), None, 3, 0),
                                                    ((12, 14, 16), None, 15, 0)]):
        p = synth.make_pair(synth.PairSpec(shape, (3.0, 6.0), 3.0), seed=synth.BASE_SEED + 40 + k, device=DEV)
        F, M, u = p["F"], p["M"], (-0.8 * p["d"]).contiguous()
        print(f"[noalloc] call {k} shape {shape} roi {roi} window {window}", flush=True)
        g = _grid(shape, roi)
        lp = ops.lncc_params(window, 1e-5, bool(ants), "border")
        nws = L.ffdp_lncc_workspace_bytes(C.byref(g), C.byref(lp))
        ws = torch.empty(nws, dtype=torch.uint8, device=DEV)
        scale = torch.tensor([0.75], device=DEV)
        ref_g = torch.full((3,) + shape, float("nan"), device=DEV)
        ref_l = torch.full((1,), float("nan"), device=DEV)
        got_g = torch.full((3,) + shape, float("nan"), device=DEV)
        got_l = torch.full((1,), float("nan"), device=DEV)
        rc = L.ffdp_warp_lncc_bwd(F.data_ptr(), M.data_ptr(), u.data_ptr(), C.byref(g), C.byref(lp),
                                  scale.data_ptr(), ref_g.data_ptr(), ref_l.data_ptr(), ws.data_ptr(), nws, stream)
        assert rc == 0, L.ffdp_last_error()
        rc = L.ffdp_warp_lncc_bwd_noalloc(F.data_ptr(), M.data_ptr(), u.data_ptr(), C.byref(g), C.byref(lp),
                                          scale.data_ptr(), got_g.data_ptr(), got_l.data_ptr(), stream)
        assert rc == 0, L.ffdp_last_error()
        torch.cuda.synchronize()
        assert torch.isfinite(ref_g).all() and torch.isfinite(ref_l).all()
        assert torch.equal(got_g, ref_g), float((got_g - ref_g).abs().max())
        assert torch.equal(got_l, ref_l), (float(got_l), float(ref_l))
        # the binding's wrapper (argument marshalling only) gives the same
        g2, l2 = ops.warp_lncc_bwd_noalloc(F, M, u, torch.empty_like(u), torch.empty(1, device=DEV), window=window,
                                           roi=roi, grad_scale=scale)
        torch.cuda.synchronize()
        assert torch.equal(g2, ref_g) and torch.equal(l2, ref_l)
