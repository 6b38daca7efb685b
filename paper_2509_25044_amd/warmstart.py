"""Learned warm start: train the U-Net on generated pairs, then compare
time-to-target of warm-started and plain registration.

    python -m paper_2509_25044_amd.warmstart [--pairs 2000] [--batch 4] [--shape 160 192 224] ...

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
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time
from typing import Optional

import torch

from . import ops, synth
from .register import RegConfig, Registration
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
          converged_every: int = 16, reg_cfg: Optional[RegConfig] = None, log_every: int = 25, log=print):
    dev = model.device
    steps = pairs // batch
    hist = []
    t0 = time.perf_counter()
    for s in range(steps):
        Fs, Ms, Ts = [], [], []
        for i in range(batch):
            idx = s * batch + i
            conv = converged_every > 0 and idx % converged_every == converged_every - 1
            F, M, T = training_pair(spec, seed0 + idx, dev, conv, reg_cfg)
            Fs.append(F); Ms.append(M); Ts.append(T)
        loss = model.train_step(torch.stack(Fs), torch.stack(Ms), torch.stack(Ts), lr=lr)
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
}


def time_to_target(model: UNet3D, F: torch.Tensor, M: torch.Tensor, plain_cfg: RegConfig, check_every: int = 5,
                   schedules=None):
    """Wall-clock seconds for the plain pyramid to finish, and for runs started
    from the network's prediction to reach the plain run's final loss
    (checked every check_every iterations on their finest level; the network's
    forward pass is included in every warm time).  schedules: names of
    WARM_SCHEDULES (default: all)."""
    dev = F.device
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    plain = Registration(F, M, plain_cfg)
    st = plain.run()
    target = plain.evaluate(st.u)  # synchronises
    t_plain = time.perf_counter() - t0
    plain_iters = sum(plain.iters(l) for l in range(len(plain.shapes)))
    u0 = model.predict(F, M)
    out = {"target_loss": target, "plain_iters": plain_iters, "plain_seconds": t_plain,
           "zero_loss": plain.evaluate(torch.zeros_like(u0)), "warm_u0_loss": plain.evaluate(u0), "warm": {}}
    for name in (schedules or list(WARM_SCHEDULES)):
        sched = WARM_SCHEDULES[name]
        cfg = plain_cfg if sched is None else dataclasses.replace(plain_cfg, levels=sched[0], iters=sched[1])
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        u0 = model.predict(F, M)
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
        out["warm"][name] = {"iters": done["iters"], "seconds": time.perf_counter() - t1,
                             "reached": done["reached"] or final <= target, "final_loss": final}
    return out


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
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    spec = synth.PairSpec(tuple(args.shape), (4.0, 12.0), 3.0, texture_std=args.texture)
    sm = dict(sigma_grad=args.sigma_grad, sigma_warp=args.sigma_warp)
    plain_cfg = RegConfig(loss="lncc", window=7, levels=(0.25, 0.5, 1.0), iters=(args.plain_iters,), lr=0.1, **sm)
    conv_cfg = RegConfig(loss="lncc", window=7, levels=(0.25, 0.5, 1.0), iters=(50,), lr=0.1, **sm)
    model = UNet3D(dev, seed=0)
    if args.load:
        model.load_state_dict(torch.load(args.load, map_location="cpu", weights_only=True))
        tr = {"steps": 0, "pairs": 0, "seconds": 0.0, "history": []}
    else:
        tr = train(model, spec, args.pairs, args.batch, args.lr, converged_every=args.converged_every,
                   reg_cfg=conv_cfg, log=lambda s: print(s, flush=True))
        if args.save:
            torch.save(model.state_dict(), args.save)
    print(f"trained {tr['pairs']} pairs in {tr['seconds']:.1f} s", flush=True)
    res = []
    for k in range(args.eval_pairs):
        p = synth.make_pair(spec, seed=synth.BASE_SEED + args.pairs + k, device=dev)
        r = time_to_target(model, p["F"], p["M"], plain_cfg)
        u0 = model.predict(p["F"], p["M"])
        tgt = inverse_target(p["d"])
        r["u0_rmse_vs_inverse"] = float(torch.sqrt(((u0 - tgt) ** 2).mean()))
        r["zero_rmse_vs_inverse"] = float(torch.sqrt((tgt ** 2).mean()))
        print(json.dumps(r), flush=True)
        res.append(r)
    out = {"shape": list(args.shape), "train": {k: v for k, v in tr.items() if k != "history"},
           "train_history": tr["history"], "eval": res}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    summ = {"plain_seconds_mean": sum(r["plain_seconds"] for r in res) / len(res), "plain_iters": res[0]["plain_iters"]}
    for name in WARM_SCHEDULES:
        summ[f"warm_{name}_seconds_mean"] = sum(r["warm"][name]["seconds"] for r in res) / len(res)
        summ[f"warm_{name}_reached"] = sum(bool(r["warm"][name]["reached"]) for r in res)
    print(json.dumps({"summary": summ}), flush=True)


if __name__ == "__main__":
    main()
