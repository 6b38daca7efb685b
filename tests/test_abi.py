"""The C-ABI library: it loads, exports every declared entry point, and its
host-side validation rejects bad arguments before any launch (no GPU needed:
every call below fails validation, so nothing reaches the HIP runtime)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2509_25044_amd import _lib
from paper_2509_25044_amd._lib import Grid, LnccParams, MiParams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_every_header_function_is_exported(L):
    names = _lib.header_functions()
    assert len(names) >= 13
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)


def test_library_is_gfx950_code_object():
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def _grid(D=8, H=8, W=8, roi=None):
    g = Grid()
    g.D, g.H, g.W = D, H, W
    roi = roi or ((0, D), (0, H), (0, W))
    for k in range(3):
        g.roi_lo[k], g.roi_hi[k] = roi[k]
    return g


def _lp(window=5, eps=1e-5, ants=0, pad=0, check=0):
    p = LnccParams()
    p.window, p.eps, p.ants_approx, p.pad_mode, p.check_finite = window, eps, ants, pad, check
    return p


def _mp(bins=32, hard=0, pad=0, check=0):
    p = MiParams()
    p.bins, p.hard_bins, p.pad_mode, p.check_finite = bins, hard, pad, check
    return p


FAKE = C.c_void_p(0x10000)       # 4-byte aligned, never dereferenced (validation fails first)
FAKE_MIS = C.c_void_p(0x10002)   # misaligned


def test_status_strings_and_version(L):
    assert L.ffdp_version() >= 100
    assert L.ffdp_status_string(0) == b"ok"
    assert L.ffdp_status_string(5).startswith(b"workspace")
    assert L.ffdp_status_string(7).startswith(b"non-finite")
    assert L.ffdp_status_string(99) == b"unknown status"


def test_workspace_queries_grow_with_blocks_not_voxels(L):
    lp = _lp()
    small = L.ffdp_lncc_workspace_bytes(C.byref(_grid(64, 64, 64)), C.byref(lp))
    big = L.ffdp_lncc_workspace_bytes(C.byref(_grid(512, 512, 512)), C.byref(lp))
    assert 0 < small <= big <= 64 * 1024      # O(#blocks) doubles, far below N
    assert (small - 16) % 8 == 0 and (big - 16) % 8 == 0  # block partials, then the checked-mode flag
    assert L.ffdp_mi_workspace_bytes(C.byref(_grid()), C.byref(_mp(32))) == (32 * 32 + 2) * 8
    assert L.ffdp_mi_workspace_bytes(C.byref(_grid()), C.byref(_mp(256))) == (256 * 256 + 2) * 8
    assert L.ffdp_mi_workspace_bytes(C.byref(_grid()), None) == (256 * 256 + 2) * 8  # any valid bins
    # no (valid) parameters: enough for every window
    n = [L.ffdp_lncc_workspace_bytes(C.byref(_grid(100, 200, 300)), C.byref(_lp(window=w))) for w in range(3, 16, 2)]
    assert L.ffdp_lncc_workspace_bytes(C.byref(_grid(100, 200, 300)), None) == max(n)
    assert L.ffdp_lncc_workspace_bytes(C.byref(_grid(100, 200, 300)), C.byref(_lp(window=18))) == max(n)


@pytest.mark.parametrize("w", [11, 13, 15])
def test_wide_window_workspace_holds_fp64_fields(L, w):
    """Windows past 9 run separable passes: 8 doubles per voxel (window sums
    of the five products, then of a, c, e; the fields a, c, e), the block
    partials of the 64 x 4-column passes, and the checked-mode flag."""
    for shape in ((100, 200, 300), (7, 9, 11), (1, 1, 1)):
        D, H, W = shape
        n = L.ffdp_lncc_workspace_bytes(C.byref(_grid(*shape)), C.byref(_lp(window=w)))
        blocks = (n - 16 - 64 * D * H * W) // 8
        cols = -(-W // 64) * -(-H // 4)
        assert (n - 16) % 8 == 0 and blocks >= cols and blocks % cols == 0, (shape, n, blocks, cols)
        assert blocks <= max(cols, 4096 + cols)
    assert L.ffdp_mi_state_floats(32) == 2 * 32 * 32 + 2 * 32 + 16


@pytest.mark.parametrize("kw,code", [
    (dict(F=None), 1),
    (dict(M=None), 1),
    (dict(grid=None), 1),
    (dict(params=None), 1),
    (dict(F=FAKE_MIS), 4),
    (dict(u=FAKE_MIS), 4),
    (dict(grid=_grid(0, 8, 8)), 2),
    (dict(grid=_grid(8, 8, 8, ((0, 9), (0, 8), (0, 8)))), 2),
    (dict(grid=_grid(8, 8, 8, ((3, 3), (0, 8), (0, 8)))), 2),
    (dict(grid=_grid(2048, 2048, 1024)), 2),
    (dict(grid=_grid(8, 70000, 8)), 2),
    (dict(params=_lp(window=4)), 3),
    (dict(params=_lp(window=17)), 3),
    (dict(params=_lp(window=12)), 3),
    (dict(params=_lp(window=1)), 3),
    (dict(params=_lp(eps=-1.0)), 3),
    (dict(params=_lp(eps=float("nan"))), 3),
    (dict(params=_lp(pad=2)), 3),
    (dict(params=_lp(ants=3)), 3),
    (dict(params=_lp(check=2)), 3),
    (dict(ws=None), 5),
    (dict(ws_bytes=1), 5),
    (dict(loss=None), 1),
])
def test_lncc_fwd_validation(L, kw, code):
    a = dict(F=FAKE, M=FAKE, u=None, grid=_grid(), params=_lp(), loss=FAKE, ws=FAKE, ws_bytes=1 << 20)
    a.update(kw)
    g = C.byref(a["grid"]) if a["grid"] is not None else None
    p = C.byref(a["params"]) if a["params"] is not None else None
    s = L.ffdp_warp_lncc_fwd(a["F"], a["M"], a["u"], g, p, a["loss"], a["ws"], a["ws_bytes"], None)
    assert s == code, L.ffdp_last_error()
    assert len(L.ffdp_last_error()) > 0


def test_lncc_bwd_validation(L):
    g, p = _grid(), _lp()
    assert L.ffdp_warp_lncc_bwd(FAKE, FAKE, None, C.byref(g), C.byref(p), None, None, None, FAKE, 1 << 20, None) == 1
    assert L.ffdp_warp_lncc_bwd(FAKE, FAKE, None, C.byref(g), C.byref(p), FAKE_MIS, FAKE, None, FAKE, 1 << 20,
                                None) == 4
    assert L.ffdp_warp_lncc_bwd(FAKE, FAKE, None, C.byref(g), C.byref(_lp(window=2)), None, FAKE, None, FAKE,
                                1 << 20, None) == 3


@pytest.mark.parametrize("mp,code", [(_mp(bins=7), 3), (_mp(bins=257), 3), (_mp(hard=3), 3), (_mp(hard=-1), 3),
                                     (_mp(pad=5), 3), (_mp(check=2), 3), (_mp(check=-1), 3)])
def test_mi_validation(L, mp, code):
    g = _grid()
    s = L.ffdp_warp_mi_fwd(FAKE, FAKE, None, C.byref(g), C.byref(mp), FAKE, FAKE, FAKE, 1 << 20, None)
    assert s == code
    s = L.ffdp_warp_mi_bwd(FAKE, FAKE, None, C.byref(g), C.byref(mp), FAKE, None, FAKE, FAKE, 1 << 20, None)
    assert s == code


def test_mi_bins_beyond_64_pass_validation_to_the_workspace_check(L):
    g = _grid()
    for b in (65, 128, 200, 256):
        need = L.ffdp_mi_workspace_bytes(C.byref(g), C.byref(_mp(b)))
        assert L.ffdp_warp_mi_fwd(FAKE, FAKE, None, C.byref(g), C.byref(_mp(b)), FAKE, FAKE, FAKE, need - 8,
                                  None) == 5
        assert b"workspace" in L.ffdp_last_error()


def test_checked_mode_is_refused_by_the_composite_sampler_calls(L):
    from paper_2509_25044_amd._lib import Affine
    g, aff = _grid(), Affine()
    for i in range(3):
        aff.A[4 * i] = 1.0
        aff.S[4 * i] = 1.0
    mp = _mp(check=1)
    assert L.ffdp_warp_mi_affine_fwd(FAKE, FAKE, None, C.byref(g), C.byref(aff), C.byref(mp), FAKE, FAKE, FAKE,
                                     1 << 20, None) == 3
    assert b"check_finite" in L.ffdp_last_error()


def test_mi_workspace_and_null_checks(L):
    g, mp = _grid(), _mp()
    assert L.ffdp_warp_mi_fwd(FAKE, FAKE, None, C.byref(g), C.byref(mp), FAKE, FAKE, FAKE, 8, None) == 5
    assert L.ffdp_warp_mi_fwd(FAKE, FAKE, None, C.byref(g), C.byref(mp), FAKE, None, FAKE, 1 << 20, None) == 1
    assert L.ffdp_warp_mi_bwd(FAKE, FAKE, None, C.byref(g), C.byref(mp), None, None, FAKE, FAKE, 1 << 20, None) == 1


def test_adam_validation(L):
    assert L.ffdp_adam_step(FAKE, FAKE, FAKE, FAKE, 0, 0.1, 0.9, 0.999, 1e-8, 1, None) == 0  # n = 0: no-op
    assert L.ffdp_adam_step(FAKE, FAKE, FAKE, FAKE, -1, 0.1, 0.9, 0.999, 1e-8, 1, None) == 2
    assert L.ffdp_adam_step(None, FAKE, FAKE, FAKE, 8, 0.1, 0.9, 0.999, 1e-8, 1, None) == 1
    assert L.ffdp_adam_step(FAKE, FAKE, FAKE, FAKE, 8, 0.1, 0.9, 0.999, 1e-8, 0, None) == 3
    assert L.ffdp_adam_step(FAKE, FAKE, FAKE, FAKE, 8, 0.1, 1.0, 0.999, 1e-8, 1, None) == 3
    assert L.ffdp_adam_step(FAKE, FAKE, FAKE, FAKE, 8, 0.1, 0.9, 0.999, 0.0, 1, None) == 3
    assert L.ffdp_adam_step(FAKE, FAKE_MIS, FAKE, FAKE, 8, 0.1, 0.9, 0.999, 1e-8, 1, None) == 4


def test_warp_and_resample_validation(L):
    g = _grid()
    assert L.ffdp_warp(None, None, C.byref(g), 0, FAKE, None) == 1
    assert L.ffdp_warp(FAKE, None, C.byref(g), 3, FAKE, None) == 3
    assert L.ffdp_warp(FAKE, None, C.byref(g), 0, FAKE, None) == 3  # out aliases M
    assert L.ffdp_resample(FAKE, 4, 4, 4, FAKE, 8, 8, 8, 1, 2.0, None) == 3  # overlap
    assert L.ffdp_resample(FAKE, 0, 4, 4, C.c_void_p(0x900000), 8, 8, 8, 1, 2.0, None) == 2
    assert L.ffdp_resample(FAKE, 4, 4, 4, C.c_void_p(0x900000), 8, 8, 8, 0, 2.0, None) == 3


def test_smoothing_validation(L):
    a, b = C.c_void_p(0x100000), C.c_void_p(0x900000)
    assert L.ffdp_gaussian_smooth(a, a, 8, 8, 8, 3, 1.0, None) == 3            # in and out overlap
    assert L.ffdp_gaussian_smooth(a, b, 8, 8, 8, 3, 0.0, None) == 3            # sigma out of (0, 2]
    assert L.ffdp_gaussian_smooth(a, b, 8, 8, 8, 3, 2.5, None) == 3
    assert L.ffdp_gaussian_smooth(a, b, 8, 8, 8, 0, 1.0, None) == 3            # channels
    assert L.ffdp_gaussian_smooth(a, b, 0, 8, 8, 3, 1.0, None) == 2            # shape
    assert L.ffdp_gaussian_smooth(None, b, 8, 8, 8, 3, 1.0, None) == 1
    assert L.ffdp_gaussian_smooth(FAKE_MIS, b, 8, 8, 8, 3, 1.0, None) == 4


def test_smooth_adam_validation(L):
    # four disjoint 3 x 8^3 float arrays (6 KiB apart)
    x, g, m, v = (C.c_void_p(0x100000 + k * 0x2000) for k in range(4))
    args = (8, 8, 8, 3, 1.0, 0.1, 0.9, 0.999, 1e-8)
    assert L.ffdp_smooth_adam_step(x, g, m, v, *args, 0, None) == 3             # step 0
    assert L.ffdp_smooth_adam_step(x, x, m, v, *args, 1, None) == 3             # g overlaps x
    assert L.ffdp_smooth_adam_step(x, g, m, m, *args, 1, None) == 3             # m overlaps v
    assert L.ffdp_smooth_adam_step(x, g, m, C.c_void_p(0x100000 + 0x1000), *args, 1, None) == 3  # v inside x
    assert L.ffdp_smooth_adam_step(None, g, m, v, *args, 1, None) == 1
    assert L.ffdp_smooth_adam_step(x, g, m, v, 8, 8, 8, 3, 3.0, 0.1, 0.9, 0.999, 1e-8, 1, None) == 3  # sigma
    assert L.ffdp_smooth_adam_step(x, g, m, v, 8, 8, 8, 3, 1.0, 0.1, 1.0, 0.999, 1e-8, 1, None) == 3  # beta1
    assert L.ffdp_smooth_adam_step(x, g, m, v, 8, 0, 8, 3, 1.0, 0.1, 0.9, 0.999, 1e-8, 1, None) == 2  # shape


def _cg(N=1, Di=4, Hi=4, Wi=4, Ca=16, Cb=0, Cout=16, stride=1, ups=0):
    g = _lib.ConvGeom()
    g.N, g.Di, g.Hi, g.Wi, g.Ca, g.Cb, g.Cout, g.stride, g.ups = N, Di, Hi, Wi, Ca, Cb, Cout, stride, ups
    return g


def test_conv_backward_from_p_validation(L):
    a16, b16 = C.c_void_p(0x100000), C.c_void_p(0x900000)
    # the P pass: n < 0, NULL operands with n > 0, n = 0 a no-op
    assert L.ffdp_conv3d_act_grad(a16, None, 0.2, -1, b16, None) == 2
    assert L.ffdp_conv3d_act_grad(None, None, 0.2, 8, b16, None) == 1
    assert L.ffdp_conv3d_act_grad(a16, None, 0.2, 8, None, None) == 1
    assert L.ffdp_conv3d_act_grad(FAKE_MIS, None, 0.2, 8, b16, None) == 4
    assert L.ffdp_conv3d_act_grad(None, None, 0.2, 0, None, None) == 0
    g = _cg()
    # backward-data from P: geometry, P alignment (16 bytes), accumulate flag
    assert L.ffdp_conv3d_bwd_data_bf16(a16, b16, C.byref(_cg(Ca=3)), a16, 0, None) == 3
    assert L.ffdp_conv3d_bwd_data_bf16(C.c_void_p(0x100008), b16, C.byref(g), a16, 0, None) == 4
    assert L.ffdp_conv3d_bwd_data_bf16(None, b16, C.byref(g), a16, 0, None) == 1
    assert L.ffdp_conv3d_bwd_data_bf16(a16, b16, C.byref(g), a16, 2, None) == 3
    # backward-weight from P: NULL P, missing skip input, workspace size
    assert L.ffdp_conv3d_bwd_weight_bf16(a16, None, None, C.byref(g), b16, None, a16, 1 << 30, None) == 1
    assert L.ffdp_conv3d_bwd_weight_bf16(a16, None, b16, C.byref(_cg(Cb=8)), b16, None, a16, 1 << 30, None) == 1
    assert L.ffdp_conv3d_bwd_weight_bf16(a16, None, b16, C.byref(g), b16, None, a16, 8, None) == 5
    # the concatenated-gradient split needs ups = 1 and 16-byte aligned buffers
    assert L.ffdp_concat_grad_split(a16, C.byref(g), b16, None, 0, 0, None) == 3
    gu = _cg(Cb=8, ups=1)
    assert L.ffdp_concat_grad_split(C.c_void_p(0x100004), C.byref(gu), b16, C.c_void_p(0x500000), 0, 0, None) == 4
