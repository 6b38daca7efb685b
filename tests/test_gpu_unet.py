"""GPU: the U-Net built on the library's conv kernels trains (overfits a fixed
batch), its backward agrees with a finite difference of its own forward, and a
small trained network gives registration a head start over zero init."""
import numpy as np
import pytest
import torch

from paper_2509_25044_amd import ops, synth
from paper_2509_25044_amd.register import RegConfig
from paper_2509_25044_amd.unet import LAYERS, UNet3D
from paper_2509_25044_amd.warmstart import inverse_target, time_to_target, train

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batch(n, shape, seed0):
    spec = synth.PairSpec(shape, (3.0, 6.0), 2.0)
    Fs, Ms, Ts = [], [], []
    for i in range(n):
        p = synth.make_pair(spec, seed=seed0 + i, device=DEV)
        Fs.append(p["F"]); Ms.append(p["M"]); Ts.append(inverse_target(p["d"]))
    return torch.stack(Fs), torch.stack(Ms), torch.stack(Ts)


def test_shapes_and_overfit():
    print("[unet overfit]", flush=True)
    model = UNet3D(DEV, seed=1)
    F, M, T = _batch(2, (16, 24, 32), 100)
    pred, acts = model.forward(F, M)
    assert pred.shape == (2, 16, 24, 32, 4)
    assert acts["e3"].shape == (2, 2, 3, 4, 128)
    l0 = float(ops.mse_disp(pred, T)[0])
    for _ in range(80):
        loss = model.train_step(F, M, T, lr=3e-3)
    l1 = float(loss)
    assert l1 < 0.5 * l0, (l0, l1)


def test_weight_gradient_direction():
    """A step against the computed weight gradient lowers the loss and a step
    along it raises it (the backward is the derivative of this forward; the
    step moves the largest weight by 2% so it survives bf16 rounding)."""
    print("[unet gradient direction]", flush=True)
    model = UNet3D(DEV, seed=2)
    F, M, T = _batch(2, (16, 16, 16), 200)
    pred, acts = model.forward(F, M)
    loss, dpred = ops.mse_disp(pred, T)
    g = model.backward(dpred, acts).clone()
    l0 = float(loss)
    assert bool(torch.isfinite(g).all()) and float(g.abs().max()) > 0
    base = model.master.clone()
    h = 0.02 * float(base.abs().max()) / float(g.abs().max())
    model.master.copy_(base - h * g)
    model.refresh_bf16()
    lm = float(ops.mse_disp(model.forward(F, M)[0], T)[0])
    model.master.copy_(base + h * g)
    model.refresh_bf16()
    lp = float(ops.mse_disp(model.forward(F, M)[0], T)[0])
    assert lm < l0 < lp, (lm, l0, lp)


def test_trained_network_gives_a_head_start():
    """Train briefly on 32^3 pairs; on held-out pairs the prediction is closer
    to the true inverse field than zero (the gain over starting from u = 0);
    the time-to-target of warm-started versus plain registration is printed."""
    print("[unet warm start small]", flush=True)
    spec = synth.PairSpec((32, 32, 32), (3.0, 6.0), 2.0)
    model = UNet3D(DEV, seed=3)
    train(model, spec, pairs=800, batch=4, lr=1e-3, converged_every=0, log_every=50)
    gains, res = [], []
    for k in range(3):
        p = synth.make_pair(spec, seed=9000 + k, device=DEV)
        tgt = inverse_target(p["d"])
        u0 = model.predict(p["F"], p["M"])
        e_net = float(torch.sqrt(((u0 - tgt) ** 2).mean()))
        e_zero = float(torch.sqrt((tgt ** 2).mean()))
        gains.append(e_zero - e_net)
        r = time_to_target(model, p["F"], p["M"], RegConfig(loss="lncc", window=5, levels=(0.5, 1.0), iters=(60,),
                                                             lr=0.1))
        print(k, e_net, e_zero, r, flush=True)
        res.append(r)
    assert sum(gains) > 0, gains
    assert all(np.isfinite(r["warm_u0_loss"]) for r in res)
