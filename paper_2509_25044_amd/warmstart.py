"""Learned warm start: train the U-Net on generated pairs, then compare
time-to-target of warm-started and plain registration.

    python -m paper_2509_25044_amd.warmstart [--pairs 2000] [--batch 4] [--shape 160 192 224] ...
    python -m paper_2509_25044_amd.warmstart --c5 [--pairs 400] [--batch 2] ...

Training pairs are seeds 2025 .. 2025 + pairs - 1 of the clinical-shape
recipe (random smooth deformations); the target of a pair is the field u with
M(x + u) = F(x), i.e. the fixed point u = -d(x + u) of the known displacement
d, solved with the library's warp.  Every `converged_every`-th pair instead
takes the displacement the plain optimiser converges to (the optimiser's own
fields, as the recipe asks).  Held-out pairs follow the training range.

Time-to-target: the plain method runs its full schedule from u = 0 and its
final LNCC loss L* is the target; the warm-started method runs the network,
then Adam with fresh state at full resolution until its loss is <= L*.  Both
are timed end to end with device synchronisation; network training is
excluded and reported separately.

--c5: the same study on one GPU's share of the gigavoxel problem (1040^3,
LNCC w = 5 on the interior [8, 1032)^3, 100 full-resolution iterations for the
plain method).  The network works at 4x downsampling: the pair is smoothed
(sigma 2 voxels, against aliasing of the fine texture), resampled to 260^3,
padded to 264^3 (edge replication; the U-Net needs sides divisible by 8), and
the prediction is cropped and resampled back to 1040^3 with each channel
scaled by its axis's grid ratio.  Training pairs are the same continuous pairs
without the texture evaluated directly on the 260^3 grid (synth.make_pair
with grid=...), so no 1040^3 volume is generated for training.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time
from typing import Optional

import torch

import torch.nn.functional as tnf

from . import ops, synth
from .configs import C5
from .register import RegConfig, Registration, resample_disp
from .unet import UNet3D


def inverse_target(d: torch.Tensor, iters: int = 4) -> torch.Tensor:
    """u with u(x) = -d(x + u(x)) by fixed-point iteration (warp of each channel of d)."""
    u = (-d).contiguous()
    for _ in range(iters):
        u = torch.stack([-ops.warp(d[c].contiguous(), u) for c in range(3)]).contiguous()
    return u


def training_pair(spec: synth.PairSpec, seed: int, device, converged: bool = False,
                  reg_cfg: Optional[RegConfig] = None):
    p = synth.make_pair(spec, seed=seed, device=device, noise_on_device=True)
    F, M = p["F"], p["M"]
    if converged:
        T = Registration(F, M, reg_cfg).run().u
    else:
        T = inverse_target(p["d"])
    return F, M, T


def train(model: UNet3D, spec: synth.PairSpec, pairs: int, batch: int = 4, lr: float = 1e-3, seed0: int = 2025,
          converged_every: int = 16, reg_cfg: Optional[RegConfig] = None, log_every: int = 25, log=print,
          make=None, lr_final: Optional[float] = None):
    """make(seed) -> (F, M, T) replaces the default pair recipe when given;
    lr_final: the learning rate decays linearly from lr to lr_final."""
    dev = model.device
    steps = pairs // batch
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        Fs, Ms, Ts = [], [], []
        for i in range(batch):
            idx = s * batch + i
            conv = converged_every > 0 and idx % converged_every == converged_every - 1
            if make is not None:
                F, M, T = make(seed0 + idx)
            else:
                F, M, T = training_pair(spec, seed0 + idx, dev, conv, reg_cfg)
            Fs.append(F); Ms.append(M); Ts.append(T)
        lr_s = lr if lr_final is None else lr + (lr_final - lr) * s / max(1, steps - 1)
        loss = model.train_step(torch.stack(Fs), torch.stack(Ms), torch.stack(Ts), lr=lr_s)
        if s % log_every == 0 or s == steps - 1:
            l = float(loss.item())
            hist.append((s, l))
            log(f"train step {s + 1}/{steps} mse {l:.5f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize(dev)
    return {"steps": steps, "pairs": steps * batch, "seconds": time.perf_counter() - t0, "history": hist}


WARM_SCHEDULES = {
    # name: (levels, iterations per level) of the warm-started run; None: the plain run's own schedule
    "same": None,
    "fine": ((1.0,), (600,)),
    "half+fine": ((0.5, 1.0), (100, 600)),
    "half50+fine": ((0.5, 1.0), (50, 600)),
    "half25+fine": ((0.5, 1.0), (25, 600)),
}


def time_to_target(model: UNet3D, F: torch.Tensor, M: torch.Tensor, plain_cfg: RegConfig, check_every: int = 5,
                   schedules=None, predict=None, table=None, controls: bool = False):
    """Wall-clock seconds for the plain pyramid to finish, and for runs started
    from the network's prediction to reach the plain run's final loss
    (checked every check_every iterations on their finest level; the network's
    forward pass is included in every warm time).  schedules: names in table
    (default WARM_SCHEDULES; all of them).  predict(F, M) -> u0 replaces the
    network's full-resolution prediction when given.  controls: also run each
    schedule other than the plain one from u0 = 0 (result "zero"), which
    separates the network's share of a speed-up from the schedule's."""
    table = WARM_SCHEDULES if table is None else table
    predict = model.predict if predict is None else predict
    dev = F.device
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    plain = Registration(F, M, plain_cfg)
    st = plain.run()
    target = plain.evaluate(st.u)  # synchronises
    t_plain = time.perf_counter() - t0
    plain_iters = sum(plain.iters(l) for l in range(len(plain.shapes)))
    del st
    u0 = predict(F, M)
    out = {"target_loss": target, "plain_iters": plain_iters, "plain_seconds": t_plain,
           "zero_loss": plain.evaluate(torch.zeros_like(u0)), "warm_u0_loss": plain.evaluate(u0), "warm": {}}
    if controls:
        out["zero"] = {}
    del plain, u0

    def attempt(cfg, init):
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        u0 = init(F, M)
        warm = Registration(F, M, cfg)
        last = len(warm.shapes) - 1
        done = {"iters": 0, "reached": False}

        def until(level, step, loss_dev):
            done["iters"] += 1
            if level != last or step % check_every:
                return False
            if float(loss_dev.item()) <= target:  # loss of the iterate before this step
                done["reached"] = True
                return True
            return False

        st2 = warm.run(u0=u0, until=until)
        final = warm.evaluate(st2.u)
        torch.cuda.synchronize(dev)
        return {"iters": done["iters"], "seconds": time.perf_counter() - t1,
                "reached": done["reached"] or final <= target, "final_loss": final}

    def zeros(F_, M_):
        return None  # Registration starts from u = 0

    for name in (schedules or list(table)):
        sched = table[name]
        cfg = plain_cfg if sched is None else dataclasses.replace(plain_cfg, levels=sched[0], iters=sched[1])
        out["warm"][name] = attempt(cfg, predict)
        if controls and sched is not None:
            out["zero"][name] = attempt(cfg, zeros)
    return out


# ------------------------------------------------- gigavoxel share (C5) --
C5_GRID = (260, 260, 260)  # 1040^3 at 4x downsampling
C5_NET = (264, 264, 264)   # padded to sides divisible by 8
C5_SCHEDULES = {
    "same": None,
    "fine": ((1.0,), (300,)),
    "half+fine": ((0.5, 1.0), (50, 300)),
}


def pad_edge(x: torch.Tensor, shape) -> torch.Tensor:
    """Pad the trailing faces of [D, H, W] or [C, D, H, W] to shape (D', H', W') by edge replication."""
    D, H, W = x.shape[-3:]
    p = (0, shape[2] - W, 0, shape[1] - H, 0, shape[0] - D)
    y = tnf.pad(x.reshape((1, -1, D, H, W)), p, mode="replicate")
    return y.reshape(tuple(x.shape[:-3]) + tuple(shape)).contiguous()


# Gaussian applied before the 4x downsampling (voxels of the full grid): the
# 3-8 voxel texture would otherwise alias into the 260^3 images; the
# training pairs are generated without it, as the filtered images show it.
C5_ANTIALIAS = 2.0


def c5_training_pair(seed: int, device):
    spec = dataclasses.replace(C5.pair, texture_std=0.0)
    p = synth.make_pair(spec, seed=seed, device=device, noise_on_device=True, grid=C5_GRID)
    T = inverse_target(p["d"])
    return pad_edge(p["F"], C5_NET), pad_edge(p["M"], C5_NET), pad_edge(T, C5_NET)


def c5_predict(model: UNet3D, F: torch.Tensor, M: torch.Tensor) -> torch.Tensor:
    """Full-resolution u0 from the network run at 4x downsampling (filtered first)."""
    Fl = pad_edge(ops.resample(ops.gaussian_smooth(F, C5_ANTIALIAS), C5_GRID), C5_NET)
    Ml = pad_edge(ops.resample(ops.gaussian_smooth(M, C5_ANTIALIAS), C5_GRID), C5_NET)
    g = C5_GRID
    u = model.predict(Fl, Ml)[:, :g[0], :g[1], :g[2]].contiguous()
    return resample_disp(u, F.shape)


def c5_main(args):
    dev = torch.device("cuda:0")
    sm = dict(sigma_grad=args.sigma_grad, sigma_warp=args.sigma_warp)
    plain_cfg = RegConfig(loss="lncc", window=C5.lncc_window, levels=(1.0,), iters=(C5.iters,), lr=C5.lr,
                          roi=C5.roi, **sm)
    model = UNet3D(dev, seed=0)
    if args.load:
        model.load_state_dict(torch.load(args.load, map_location="cpu", weights_only=True))
        tr = {"steps": 0, "pairs": 0, "seconds": 0.0, "history": []}
    else:
        tr = train(model, C5.pair, args.pairs, args.batch, args.lr, converged_every=0,
                   log=lambda s: print(s, flush=True), make=lambda seed: c5_training_pair(seed, dev))
        if args.save:
            torch.save(model.state_dict(), args.save)
        if args.save_weights:
            model.save_weights(args.save_weights)
    print(f"trained {tr['pairs']} pairs in {tr['seconds']:.1f} s", flush=True)
    res = []
    for k in range(args.eval_pairs):
        t0 = time.perf_counter()
        p = synth.make_pair(C5.pair, seed=synth.BASE_SEED + args.pairs + k, device=dev, noise_on_device=True)
        F, M = p["F"], p["M"]
        tgt = inverse_target(p["d"])
        del p
        torch.cuda.synchronize(dev)
        print(f"eval pair {k}: generated in {time.perf_counter() - t0:.1f} s", flush=True)
        u0 = c5_predict(model, F, M)
        rm = {"u0_rmse_vs_inverse": float(torch.sqrt(((u0 - tgt) ** 2).mean())),
              "zero_rmse_vs_inverse": float(torch.sqrt((tgt ** 2).mean()))}
        del u0, tgt
        r = time_to_target(model, F, M, plain_cfg, predict=lambda a, b: c5_predict(model, a, b),
                           table=C5_SCHEDULES, controls=True)
        r.update(rm)
        print(json.dumps(r), flush=True)
        res.append(r)
        del F, M
    return tr, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--shape", type=int, nargs=3, default=(160, 192, 224))
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--eval-pairs", type=int, default=4)
    ap.add_argument("--plain-iters", type=int, default=200)
    ap.add_argument("--converged-every", type=int, default=16)
    ap.add_argument("--texture", type=float, default=0.05, help="std of the band-passed texture in each pair")
    ap.add_argument("--sigma-grad", type=float, default=0.0)
    ap.add_argument("--sigma-warp", type=float, default=0.0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None, help="write the trained network's weights here")
    ap.add_argument("--load", default=None, help="skip training and load weights from here")
    ap.add_argument("--save-weights", default=None, help="also write the trained weights alone (safetensors)")
    ap.add_argument("--load-weights", default=None, help="skip training and load weights alone (safetensors)")
    ap.add_argument("--resume", action="store_true", help="with --load: keep training the loaded weights")
    ap.add_argument("--train-pairs", type=int, default=None,
                    help="pairs to train on (default --pairs); with --resume drawn from --seed0 on")
    ap.add_argument("--seed0", type=int, default=synth.BASE_SEED, help="seed of the first training pair")
    ap.add_argument("--lr-final", type=float, default=None, help="linear decay of the learning rate to this value")
    ap.add_argument("--c5", action="store_true", help="the 1040^3 share with the network at 4x downsampling")
    args = ap.parse_args()
    if args.c5:
        tr, res = c5_main(args)
        _report(args, list(C5.shape), tr, res, C5_SCHEDULES)
        return
    dev = torch.device("cuda:0")
    spec = synth.PairSpec(tuple(args.shape), (4.0, 12.0), 3.0, texture_std=args.texture)
    sm = dict(sigma_grad=args.sigma_grad, sigma_warp=args.sigma_warp)
    plain_cfg = RegConfig(loss="lncc", window=7, levels=(0.25, 0.5, 1.0), iters=(args.plain_iters,), lr=0.1, **sm)
    conv_cfg = RegConfig(loss="lncc", window=7, levels=(0.25, 0.5, 1.0), iters=(50,), lr=0.1, **sm)
    model = UNet3D(dev, seed=0)
    tr = {"steps": 0, "pairs": 0, "seconds": 0.0, "history": []}
    if args.load:
        model.load_state_dict(torch.load(args.load, map_location="cpu", weights_only=True))
    if args.load_weights:
        model.load_weights(args.load_weights)
    if not (args.load or args.load_weights) or args.resume:
        n_train = args.pairs if args.train_pairs is None else args.train_pairs
        tr = train(model, spec, n_train, args.batch, args.lr, seed0=args.seed0,
                   converged_every=args.converged_every, reg_cfg=conv_cfg, log=lambda s: print(s, flush=True),
                   lr_final=args.lr_final)
        if args.save:
            torch.save(model.state_dict(), args.save)
        if args.save_weights:
            model.save_weights(args.save_weights)
    print(f"trained {tr['pairs']} pairs in {tr['seconds']:.1f} s", flush=True)
    res = []
    for k in range(args.eval_pairs):
        p = synth.make_pair(spec, seed=synth.BASE_SEED + args.pairs + k, device=dev)
        r = time_to_target(model, p["F"], p["M"], plain_cfg, controls=True)
        u0 = model.predict(p["F"], p["M"])
        tgt = inverse_target(p["d"])
        r["u0_rmse_vs_inverse"] = float(torch.sqrt(((u0 - tgt) ** 2).mean()))
        r["zero_rmse_vs_inverse"] = float(torch.sqrt((tgt ** 2).mean()))
        print(json.dumps(r), flush=True)
        res.append(r)
    _report(args, list(args.shape), tr, res, WARM_SCHEDULES)


def _report(args, shape, tr, res, table):
    out = {"shape": shape, "train": {k: v for k, v in tr.items() if k != "history"},
           "train_history": tr["history"], "eval": res}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    if not res:
        return
    summ = {"plain_seconds_mean": sum(r["plain_seconds"] for r in res) / len(res), "plain_iters": res[0]["plain_iters"]}
    for name in table:
        for init in ("warm", "zero"):
            rs = [r[init][name] for r in res if name in r.get(init, {})]
            if rs:
                summ[f"{init}_{name}_seconds_mean"] = sum(x["seconds"] for x in rs) / len(rs)
                summ[f"{init}_{name}_iters_mean"] = sum(x["iters"] for x in rs) / len(rs)
                summ[f"{init}_{name}_reached"] = sum(bool(x["reached"]) for x in rs)
    print(json.dumps({"summary": summ}), flush=True)


if __name__ == "__main__":
    main()
