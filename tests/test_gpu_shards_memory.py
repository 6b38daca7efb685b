"""Two claims of the design on one GPU.

* Slab decomposition (Sec. "Grid Parallel"): the fused LNCC loss and
  gradient of a volume equal those assembled from z-slabs, each computed on
  its slab plus a halo with the slab as ROI and the global 1/N_roi as the
  gradient scale, the halo contributions added back to their owners.  This
  is the arithmetic a sharded run performs around its halo exchange (no
  second GPU is involved).
* No device allocation inside the library: with caller-owned outputs and
  workspaces, repeated calls leave torch's allocator and the device's free
  memory unchanged (the caller-owned-workspace contract of the C ABI).
"""
import math

import numpy as np
import pytest
import torch

from paper_2509_25044_amd import ops, synth
from parity_util import assert_grad

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _pair(shape, max_disp, seed):
    p = synth.make_pair(synth.PairSpec(shape, (3.0, 8.0), max_disp), seed=seed, device=DEV)
    return p["F"], p["M"], (-0.6 * p["d"]).contiguous()


@pytest.mark.parametrize("window,bounds", [(5, (0, 21, 43, 64)), (7, (0, 9, 30, 31, 64))])
def test_lncc_slab_decomposition(window, bounds):
    print(f"[lncc slabs w={window} bounds={bounds}]", flush=True)
    F, M, u = _pair((64, 40, 36), 2.5, 2025)
    D = F.shape[0]
    n_full = F.numel()
    g_full, l_full = ops.warp_lncc_bwd(F, M, u, window=window)
    r = (window - 1) // 2
    # a halo wide enough that no window or sample of a slab's voxels, or of the
    # voxels its adjoint reaches, sees the crop's faces
    halo = 2 * r + math.ceil(float(u.abs().max())) + 2
    g_sum = torch.zeros_like(g_full)
    parts = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        lo, hi = max(0, a - halo), min(D, b + halo)
        Fc, Mc, uc = F[lo:hi].contiguous(), M[lo:hi].contiguous(), u[:, lo:hi].contiguous()
        roi = ((a - lo, b - lo), (0, F.shape[1]), (0, F.shape[2]))
        n_s = (b - a) * F.shape[1] * F.shape[2]
        scale = torch.tensor([n_s / n_full], dtype=torch.float32, device=DEV)
        g, l = ops.warp_lncc_bwd(Fc, Mc, uc, window=window, roi=roi, grad_scale=scale)
        g_sum[:, lo:hi] += g
        parts.append((n_s, float(l.item())))
    l_sum = 1.0 - sum(n * (1.0 - l) for n, l in parts) / n_full
    assert abs(l_sum - float(l_full.item())) <= 1e-5 * abs(float(l_full.item()))
    assert_grad(g_sum.double().cpu().numpy(), g_full.double().cpu().numpy(), f"slabs w={window}")


def test_adam_slab_decomposition():
    """Adam is elementwise: slabs of the field updated separately give the same field bitwise."""
    g = torch.Generator(device=DEV).manual_seed(5)
    shape = (3, 40, 24, 20)
    x, grad, m, v = (torch.randn(shape, generator=g, device=DEV) for _ in range(4))
    v = v.abs()
    xs, ms, vs = x.clone(), m.clone(), v.clone()
    ops.adam_step(x, grad, m, v, lr=0.1, step=3)
    for a, b in ((0, 13), (13, 40)):
        sl = (slice(None), slice(a, b))
        xa, ga, ma, va = (t[sl].contiguous() for t in (xs, grad, ms, vs))
        ops.adam_step(xa, ga, ma, va, lr=0.1, step=3)
        xs[sl], ms[sl], vs[sl] = xa, ma, va
    assert torch.equal(x, xs) and torch.equal(m, ms) and torch.equal(v, vs)


def test_calls_allocate_no_device_memory():
    print("[no allocation with caller-owned buffers]", flush=True)
    F, M, u = _pair((48, 40, 36), 2.5, 2026)
    g = torch.empty_like(u)
    m, v = torch.zeros_like(u), torch.zeros_like(u)
    sm = torch.empty_like(u)
    loss = torch.empty(1, device=DEV)
    ws_l = torch.empty(ops.lncc_workspace_bytes(F.shape, None, 5), dtype=torch.uint8, device=DEV)
    ws_m = torch.empty(ops.mi_workspace_bytes(32), dtype=torch.uint8, device=DEV)
    state = torch.empty(ops.mi_state_floats(32), device=DEV)

    def calls():
        ops.warp_lncc_bwd(F, M, u, window=5, grad_u=g, loss=loss, ws=ws_l)
        ops.warp_lncc_fwd(F, M, u, window=5, loss=loss, ws=ws_l)
        ops.warp_mi_fwd(F, M, u, bins=32, state=state, loss=loss, ws=ws_m)
        ops.warp_mi_bwd(F, M, u, state, bins=32, grad_u=g, ws=ws_m)
        ops.gaussian_smooth(g, 1.0, out=sm)
        ops.adam_step(u, sm, m, v, lr=0.01, step=1)

    calls()  # first launches load the code objects
    torch.cuda.synchronize()
    alloc0 = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        calls()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert torch.cuda.memory_allocated() == alloc0
    assert torch.cuda.max_memory_allocated() == alloc0
    # the device's free memory: no library-side allocation across 30 calls
    assert free0 - free1 <= (2 << 20), (free0, free1)
