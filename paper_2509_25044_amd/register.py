"""Deformable registration driver: multi-scale pyramid, fused loss + adjoint,
per-voxel Adam on the displacement, checkpoint/resume.

The loop is the paper's registration iteration (Sec. "Grid Parallel" keeps
optimiser states m1, m2 per voxel of the displacement and smooths the
gradient and the displacement; the experiments run per-scale iteration lists
on image pyramids with sigma_grad = 1 and sigma_warp = 0.5 voxels).  Every
iteration is library calls on the current HIP stream -- the fused
loss+adjoint kernel, the Adam kernel (fused with the Gaussian smoothing of the
gradient when that is on), the optional smoothing of the displacement -- and the loss of
each iteration is written into a device buffer, so the loop never waits on
the host.  Smoothing is off by default (sigma 0).

Pyramid: level factors f (e.g. 0.25, 0.5, 1.0) give shapes round(f * shape);
images are resampled with the library's corner-aligned trilinear resize;
the displacement moves to the next level by the same resize with each
channel scaled by that axis's (n_fine - 1)/(n_coarse - 1); Adam state starts
fresh on each level.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import ops


@dataclasses.dataclass
class RegConfig:
    loss: str = "lncc"                  # "lncc" or "mi"
    window: int = 5
    eps: float = 1e-5
    ants: bool = False
    bins: int = 32
    levels: Tuple[float, ...] = (1.0,)
    iters: Tuple[int, ...] = (50,)       # per level (one value is used for every level)
    lr: float = 0.1
    betas: Tuple[float, float] = (0.9, 0.999)
    adam_eps: float = 1e-8
    pad: str = "border"
    roi: Optional[tuple] = None          # full-resolution ROI; coarser levels use the full array
    sigma_grad: float = 0.0              # Gaussian smoothing of dL/du before Adam (0 = off)
    sigma_warp: float = 0.0              # Gaussian smoothing of u after Adam (0 = off)


def level_shapes(shape: Sequence[int], levels: Sequence[float]) -> List[Tuple[int, int, int]]:
    out = []
    for f in levels:
        out.append(tuple(max(1, int(round(s * f))) for s in shape))
    return out


def axis_scales(src: Sequence[int], dst: Sequence[int]) -> Tuple[float, float, float]:
    """Displacement scale per channel (x, y, z) when resampling src -> dst with corner alignment."""
    def f(a, b):
        return (b - 1) / (a - 1) if a > 1 else 1.0
    D0, H0, W0 = src
    D1, H1, W1 = dst
    return f(W0, W1), f(H0, H1), f(D0, D1)


def resample_disp(u: torch.Tensor, shape: Sequence[int]) -> torch.Tensor:
    """Move a displacement [3, D, H, W] (voxel units) to another grid."""
    out = torch.empty((3,) + tuple(shape), dtype=torch.float32, device=u.device)
    sx, sy, sz = axis_scales(u.shape[1:], shape)
    for c, s in enumerate((sx, sy, sz)):
        ops.resample(u[c], shape, value_scale=s, out=out[c])
    return out


@dataclasses.dataclass
class RegState:
    """Everything needed to resume a registration exactly."""
    level: int
    step: int                 # Adam steps done on this level
    u: torch.Tensor
    m: torch.Tensor
    v: torch.Tensor
    losses: List[torch.Tensor]

    def save(self, path: str):
        torch.save({"level": self.level, "step": self.step, "u": self.u.cpu(), "m": self.m.cpu(),
                    "v": self.v.cpu(), "losses": [l.cpu() for l in self.losses]}, path)

    @staticmethod
    def load(path: str, device) -> "RegState":
        d = torch.load(path, map_location="cpu", weights_only=True)
        return RegState(d["level"], d["step"], d["u"].to(device), d["m"].to(device), d["v"].to(device),
                        [l.to(device) for l in d["losses"]])


class Registration:
    """Plain deformable registration of F to M (u such that M(x + u) ~ F)."""

    def __init__(self, F: torch.Tensor, M: torch.Tensor, cfg: RegConfig):
        if cfg.loss not in ("lncc", "mi"):
            raise ValueError("loss must be 'lncc' or 'mi'")
        self.cfg = cfg
        self.shapes = level_shapes(F.shape, cfg.levels)
        self._tmp = {}  # smoothing output buffers, one per level shape
        self.F = []
        self.M = []
        for shp in self.shapes:
            if tuple(shp) == tuple(F.shape):
                self.F.append(F)
                self.M.append(M)
            else:
                self.F.append(ops.resample(F, shp))
                self.M.append(ops.resample(M, shp))

    def iters(self, level: int) -> int:
        it = self.cfg.iters
        return it[level] if len(it) > 1 else it[0]

    def init_state(self, u0: Optional[torch.Tensor] = None, level: int = 0) -> RegState:
        shp = self.shapes[level]
        dev = self.F[level].device
        if u0 is None:
            u = torch.zeros((3,) + tuple(shp), dtype=torch.float32, device=dev)
        elif tuple(u0.shape[1:]) != tuple(shp):
            u = resample_disp(u0.contiguous(), shp)
        else:
            u = u0.clone().contiguous()
        return RegState(level, 0, u, torch.zeros_like(u), torch.zeros_like(u), [])

    def _roi(self, level):
        return self.cfg.roi if tuple(self.shapes[level]) == tuple(self.F[-1].shape) else None

    def step(self, st: RegState, loss_out: torch.Tensor, grad: Optional[torch.Tensor] = None) -> torch.Tensor:
        """One iteration: fused loss + adjoint, then Adam.  loss_out: device float [1]."""
        c = self.cfg
        lv = st.level
        F, M = self.F[lv], self.M[lv]
        if c.loss == "lncc":
            grad, _ = ops.warp_lncc_bwd(F, M, st.u, window=c.window, eps=c.eps, ants=c.ants, pad=c.pad,
                                        roi=self._roi(lv), grad_u=grad, loss=loss_out)
        else:
            _, state = ops.warp_mi_fwd(F, M, st.u, bins=c.bins, pad=c.pad, roi=self._roi(lv), loss=loss_out)
            grad = ops.warp_mi_bwd(F, M, st.u, state, bins=c.bins, pad=c.pad, roi=self._roi(lv), grad_u=grad)
        st.step += 1
        if c.sigma_grad > 0:  # smoothed gradient and Adam in one pass (bitwise smooth, then step)
            ops.smooth_adam_step(st.u, grad, st.m, st.v, c.sigma_grad, lr=c.lr, beta1=c.betas[0], beta2=c.betas[1],
                                 eps=c.adam_eps, step=st.step)
        else:
            ops.adam_step(st.u, grad, st.m, st.v, lr=c.lr, beta1=c.betas[0], beta2=c.betas[1], eps=c.adam_eps,
                          step=st.step)
        if c.sigma_warp > 0:
            key = tuple(st.u.shape)
            su = ops.gaussian_smooth(st.u, c.sigma_warp, out=self._buffer(st.u))
            self._tmp[key], st.u = st.u, su
        return grad

    def _buffer(self, like: torch.Tensor) -> torch.Tensor:
        key = tuple(like.shape)
        b = self._tmp.get(key)
        if b is None:
            b = self._tmp[key] = torch.empty_like(like)
        return b

    def evaluate(self, u: torch.Tensor, level: int = -1) -> float:
        """Loss of the current displacement at a level (host sync)."""
        c = self.cfg
        lv = level % len(self.shapes)
        if c.loss == "lncc":
            l = ops.warp_lncc_fwd(self.F[lv], self.M[lv], u, window=c.window, eps=c.eps, pad=c.pad,
                                  roi=self._roi(lv))
        else:
            l, _ = ops.warp_mi_fwd(self.F[lv], self.M[lv], u, bins=c.bins, pad=c.pad, roi=self._roi(lv))
        return float(l.item())

    def run(self, u0: Optional[torch.Tensor] = None, state: Optional[RegState] = None,
            stop_after: Optional[int] = None,
            until: Optional[Callable[[int, int, torch.Tensor], bool]] = None) -> RegState:
        """Run (or resume) the pyramid.  stop_after: total iterations to run in
        this call (for checkpointing); until(level, step, loss_dev) -> True
        stops early (it may synchronise)."""
        st = state if state is not None else self.init_state(u0, 0)
        done = 0
        while True:
            lv = st.level
            n = self.iters(lv)
            hist = torch.empty(n, dtype=torch.float32, device=st.u.device)
            if len(st.losses) > lv:  # resuming inside this level
                hist[: st.step] = st.losses[lv][: st.step]
                st.losses[lv] = hist
            else:
                st.losses.append(hist)
            grad = None
            while st.step < n:
                if stop_after is not None and done >= stop_after:
                    return st
                grad = self.step(st, hist[st.step: st.step + 1], grad)
                done += 1
                if until is not None and until(lv, st.step, hist[st.step - 1: st.step]):
                    return st
            if lv + 1 >= len(self.shapes):
                return st
            nxt = self.init_state(st.u, lv + 1)
            nxt.losses = st.losses
            st = nxt


def register(F: torch.Tensor, M: torch.Tensor, cfg: RegConfig, u0: Optional[torch.Tensor] = None) -> RegState:
    """Register F and M; returns the final state (u at full resolution, losses per level)."""
    return Registration(F, M, cfg).run(u0=u0)


# ------------------------------------------------------------ affine MI stage --
@dataclasses.dataclass
class AffineConfig:
    """Affine MI registration settings (the paper's affine stage runs MI on a
    pyramid before the deformable stage)."""
    bins: int = 32
    hard: object = False                 # MI estimator: False (Parzen) or "approx"
    levels: Tuple[float, ...] = (0.5, 1.0)
    iters: Tuple[int, ...] = (100,)      # per level (one value is used for every level)
    lr_A: float = 0.005
    lr_t: float = 0.2
    pad: str = "border"


def _centre(shape):
    D, H, W = shape
    return np.array([(W - 1) / 2.0, (H - 1) / 2.0, (D - 1) / 2.0])


def register_affine(F: torch.Tensor, M: torch.Tensor, cfg: AffineConfig):
    """Affine MI registration of F and M: (A, t, losses) with M(A X + t) ~ F
    in F's voxel coordinates X = (x, y, z).  The transform is optimised as
    p = A (X - c) + c + t' about the volume centre c (so that rotation and
    translation decouple); every loss and gradient comes from the
    composite-sampler MI kernels, the 12 parameters take Adam steps on the
    device, and each level starts from the previous one's transform."""
    shapes = level_shapes(F.shape, cfg.levels)
    dev = F.device
    prm = torch.zeros(12, dtype=torch.float32, device=dev)  # A - I (row-major), t'
    losses = []
    prev = None
    for lv, shp in enumerate(shapes):
        Fl = F if tuple(shp) == tuple(F.shape) else ops.resample(F, shp)
        Ml = M if tuple(shp) == tuple(M.shape) else ops.resample(M, shp)
        if prev is not None:  # move (A, t') to this grid: A' = s A s^-1, t'' = s t'
            s = np.array(axis_scales(prev, shp))
            h = prm.double().cpu().numpy()
            A = np.eye(3) + h[:9].reshape(3, 3)
            A = (s[:, None] * A) / s[None, :]
            prm = torch.tensor(np.concatenate([(A - np.eye(3)).reshape(-1), s * h[9:]]), dtype=torch.float32,
                               device=dev)
        c = _centre(shp)
        m = torch.zeros_like(prm)
        v = torch.zeros_like(prm)
        g = torch.zeros_like(prm)
        n = cfg.iters[lv] if len(cfg.iters) > 1 else cfg.iters[0]
        hist = []
        for it in range(1, n + 1):
            h = prm.double().cpu().numpy()
            A = np.eye(3) + h[:9].reshape(3, 3)
            t = h[9:] + c - A @ c
            loss, state = ops.warp_mi_affine_fwd(Fl, Ml, None, A=A, t=t, bins=cfg.bins, hard=cfg.hard, pad=cfg.pad)
            _, gA, gt = ops.warp_mi_affine_bwd(Fl, Ml, None, state, A=A, t=t, bins=cfg.bins, hard=cfg.hard,
                                               pad=cfg.pad)
            # t depends on A through t = t' + c - A c
            gAc = gA - torch.outer(gt, torch.tensor(c, dtype=torch.float64, device=dev))
            g.copy_(torch.cat([gAc.reshape(-1), gt]).float())
            ops.adam_step(prm[:9], g[:9], m[:9], v[:9], lr=cfg.lr_A, step=it)
            ops.adam_step(prm[9:], g[9:], m[9:], v[9:], lr=cfg.lr_t, step=it)
            hist.append(loss)
        losses.append(torch.cat(hist))
        prev = shp
    h = prm.double().cpu().numpy()
    A = np.eye(3) + h[:9].reshape(3, 3)
    c = _centre(F.shape)
    return A, h[9:] + c - A @ c, losses


# ------------------------------------------------------- workload registrations --
def _main():
    """Run one workload's registration on its seeded synthetic pair and print
    a JSON summary: the loss every `--every` iterations per level, wall-clock
    seconds (device synchronised, pair generation excluded) and the rms
    distance of u from the pair's true inverse displacement."""
    import argparse
    import json
    import time

    from . import synth
    from .configs import ALL

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, help="workload name or prefix (c1, c2, c3, c5)")
    ap.add_argument("--loss", choices=("lncc", "mi"), default="lncc")
    ap.add_argument("--iters", type=int, default=None, help="iterations per level (default: the workload's)")
    ap.add_argument("--levels", type=float, nargs="+", default=None, help="pyramid levels (default: the workload's)")
    ap.add_argument("--sigma-grad", type=float, default=0.0)
    ap.add_argument("--sigma-warp", type=float, default=0.0)
    ap.add_argument("--every", type=int, default=25)
    ap.add_argument("--seed", type=int, default=synth.BASE_SEED)
    args = ap.parse_args()
    wl = ALL.get(args.workload) or next(w for w in ALL.values() if w.name.startswith(args.workload))
    dev = torch.device("cuda:0")
    p = synth.make_pair(wl.pair, seed=args.seed, device=dev)
    F, M, d = p["F"], p["M"], p["d"]
    del p
    cfg = RegConfig(loss=args.loss, window=wl.lncc_window, bins=wl.mi_bins,
                    levels=tuple(args.levels) if args.levels else wl.levels,
                    iters=(args.iters if args.iters else wl.iters,), lr=wl.lr, roi=wl.roi,
                    sigma_grad=args.sigma_grad, sigma_warp=args.sigma_warp)
    reg = Registration(F, M, cfg)
    u_zero = torch.zeros((3,) + tuple(F.shape), device=dev)
    l_zero = reg.evaluate(u_zero)
    del u_zero
    reg.run(u0=None, stop_after=1)  # first use of every kernel, untimed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = reg.run()
    final = reg.evaluate(st.u)  # synchronises
    secs = time.perf_counter() - t0
    from .warmstart import inverse_target
    tgt = inverse_target(d)
    rms = lambda x: float(torch.sqrt((x ** 2).mean()))
    curves = [[round(float(v), 6) for v in h.cpu()[:: args.every].tolist()] for h in st.losses]
    print(json.dumps({"workload": wl.name, "shape": list(F.shape), "loss": args.loss,
                      "window": cfg.window if args.loss == "lncc" else None,
                      "bins": cfg.bins if args.loss == "mi" else None, "levels": list(cfg.levels),
                      "iters_per_level": cfg.iters[0], "sigma_grad": cfg.sigma_grad, "sigma_warp": cfg.sigma_warp,
                      "loss_at_u0": l_zero, "final_loss": final, "seconds": round(secs, 4),
                      "ms_per_iteration": round(secs * 1e3 / (cfg.iters[0] * len(cfg.levels)), 3),
                      "rms_u_minus_inverse": rms(st.u - tgt), "rms_inverse": rms(tgt),
                      "loss_every": args.every, "loss_curves": curves}), flush=True)


if __name__ == "__main__":
    _main()
