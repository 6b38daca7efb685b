"""Warm-start 3D U-Net trained and run with the library's BF16-MFMA kernels.

Architecture (4 levels, channels 16-32-64-128, 3x3x3 convolutions, LeakyReLU
0.2, bf16 weights and activations, fp32 accumulation):

    x  = (F, M, 0, 0)                                   full res, 4 ch
    e0 = lrelu(conv(x))            4 -> 16   stride 1   full
    e1 = lrelu(conv(e0))          16 -> 32   stride 2   1/2
    e2 = lrelu(conv(e1))          32 -> 64   stride 2   1/4
    e3 = lrelu(conv(e2))          64 -> 128  stride 2   1/8
    d2 = lrelu(conv(up(e3) | e2)) 192 -> 64             1/4
    d1 = lrelu(conv(up(d2) | e1))  96 -> 32             1/2
    d0 = lrelu(conv(up(d1) | e0))  48 -> 16             full
    u  = conv(d0)                  16 -> 4 (3 used)     full, fp32

up = nearest x2, | = channel concatenation; both happen inside the
convolution's operand gather.  Volumes must have D, H, W divisible by 8.

Training keeps fp32 master weights with Adam states (the library's
ffdp_adam_step over one flat buffer) and refreshes the bf16 copies after each
step.  The loss is the MSE between the 3 output channels and a target
displacement field.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import ops

SLOPE = 0.2


@dataclasses.dataclass(frozen=True)
class Layer:
    name: str
    a: str            # input part a (tensor name)
    b: Optional[str]  # input part b (skip) or None
    Ca: int
    Cb: int
    Cout: int
    stride: int
    ups: bool
    act: bool


LAYERS: Tuple[Layer, ...] = (
    Layer("e0", "x", None, 4, 0, 16, 1, False, True),
    Layer("e1", "e0", None, 16, 0, 32, 2, False, True),
    Layer("e2", "e1", None, 32, 0, 64, 2, False, True),
    Layer("e3", "e2", None, 64, 0, 128, 2, False, True),
    Layer("d2", "e3", "e2", 128, 64, 64, 1, True, True),
    Layer("d1", "d2", "e1", 64, 32, 32, 1, True, True),
    Layer("d0", "d1", "e0", 32, 16, 16, 1, True, True),
    Layer("hd", "d0", None, 16, 0, 4, 1, False, False),
)


class UNet3D:
    def __init__(self, device="cuda:0", seed: int = 0):
        self.device = torch.device(device)
        self.offsets: Dict[str, Tuple[int, int, int]] = {}
        n = 0
        for L in LAYERS:
            nw = L.Cout * 27 * (L.Ca + L.Cb)
            self.offsets[L.name] = (n, nw, L.Cout)
            n += nw + L.Cout
        self.nparams = n
        rng = np.random.default_rng(seed)
        p = np.zeros(n, np.float32)
        for L in LAYERS:
            o, nw, _ = self.offsets[L.name]
            fan_in = 27 * (L.Ca + L.Cb)
            bound = math.sqrt(6.0 / fan_in) * (0.1 if L.name == "hd" else 1.0 / math.sqrt(1 + SLOPE ** 2))
            p[o:o + nw] = rng.uniform(-bound, bound, nw)
        self.master = torch.from_numpy(p).to(self.device)
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.step_count = 0
        self.wbf: Dict[str, torch.Tensor] = {}
        self.wt: Dict[str, torch.Tensor] = {}
        self._ws = None
        self.refresh_bf16()

    # views into the flat buffers
    def w(self, name, buf=None):
        buf = self.master if buf is None else buf
        o, nw, cout = self.offsets[name]
        L = next(l for l in LAYERS if l.name == name)
        return buf[o:o + nw].view(L.Cout, 27, L.Ca + L.Cb)

    def b(self, name, buf=None):
        buf = self.master if buf is None else buf
        o, nw, cout = self.offsets[name]
        return buf[o + nw:o + nw + cout]

    def refresh_bf16(self):
        for L in LAYERS:
            wb, wt = ops.conv3d_weight_prep(self.w(L.name), self.wbf.get(L.name), self.wt.get(L.name))
            self.wbf[L.name], self.wt[L.name] = wb, wt

    def state_dict(self):
        return {"master": self.master.cpu(), "m": self.m.cpu(), "v": self.v.cpu(), "step": self.step_count}

    def save_weights(self, path: str):
        """The fp32 master weights alone (no optimiser state), as safetensors."""
        from safetensors.torch import save_file
        save_file({"master": self.master.detach().cpu().contiguous()}, path,
                  metadata={"layers": ",".join(L.name for L in LAYERS), "nparams": str(self.nparams),
                            "step": str(self.step_count)})

    def load_weights(self, path: str):
        """Master weights written by save_weights (safetensors: no code runs on load)."""
        from safetensors.torch import load_file
        w = load_file(path)["master"]
        if w.numel() != self.nparams:
            raise ValueError(f"{path}: {w.numel()} parameters, this network has {self.nparams}")
        self.master.copy_(w.to(self.device))
        self.refresh_bf16()

    def load_state_dict(self, d):
        self.master.copy_(d["master"].to(self.device))
        self.m.copy_(d["m"].to(self.device))
        self.v.copy_(d["v"].to(self.device))
        self.step_count = int(d["step"])
        self.refresh_bf16()

    # --------------------------------------------------------------- forward
    def _geom(self, L: Layer, acts, N):
        xa = acts[L.a]
        if L.ups:
            Di, Hi, Wi = (2 * s for s in xa.shape[1:4])
        else:
            Di, Hi, Wi = xa.shape[1:4]
        return ops.conv_geom(N, Di, Hi, Wi, L.Ca, L.Cb, L.Cout, L.stride, L.ups)

    def forward(self, F: torch.Tensor, M: torch.Tensor):
        """F, M fp32 [N, D, H, W] -> (pred fp32 [N, D, H, W, 4], activations)."""
        if F.dim() == 3:
            F, M = F[None], M[None]
        N, D, H, W = F.shape
        if D % 8 or H % 8 or W % 8:
            raise ValueError(f"U-Net input sides must be multiples of 8 (got {D}x{H}x{W})")
        acts = {"x": ops.unet_pack_pair(F.contiguous(), M.contiguous())}
        pred = None
        for L in LAYERS:
            g = self._geom(L, acts, N)
            xb = acts[L.b] if L.b else None
            if L.name == "hd":
                pred = ops.conv3d_fwd(acts[L.a], None, self.wbf[L.name], self.b(L.name), g, act=False,
                                      want_bf16=False, want_f32=True)
            else:
                acts[L.name] = ops.conv3d_fwd(acts[L.a], xb, self.wbf[L.name], self.b(L.name), g, act=L.act,
                                              slope=SLOPE)
        return pred, acts

    def predict(self, F: torch.Tensor, M: torch.Tensor) -> torch.Tensor:
        """Displacement [3, D, H, W] (or [N, 3, ...] for a batch)."""
        batched = F.dim() == 4
        pred, _ = self.forward(F, M)
        u = ops.unpack_disp(pred)
        return u if batched else u[0]

    # -------------------------------------------------------------- backward
    def backward(self, dpred: torch.Tensor, acts):
        """Fill self.grad from dL/dpred (fp32 [N, D, H, W, 4])."""
        N = dpred.shape[0]
        grads = {}  # fp32 gradients of the layer outputs
        dout = {"hd": dpred}
        for L in reversed(LAYERS):
            g = self._geom(L, acts, N)
            dy = dout[L.name] if L.name == "hd" else grads[L.name]
            y = acts.get(L.name) if L.act else None
            xa = acts[L.a]
            xb = acts[L.b] if L.b else None
            nb = ops.conv3d_bwd_weight_workspace_bytes(g)
            if self._ws is None or self._ws.numel() < nb:
                self._ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            p = ops.conv3d_act_grad(dy, y, slope=SLOPE)  # bf16 dL/dy act'(y), the operand of both products
            ops.conv3d_bwd_weight_bf16(xa, xb, p, g, dw=self.w(L.name, self.grad), db=self.b(L.name, self.grad),
                                       ws=self._ws)
            if L.a == "x":
                continue
            if L.ups:
                dxc = ops.conv3d_bwd_data_bf16(p, self.wt[L.name], g)
                dxa, dxb = ops.concat_grad_split(dxc, g)
                grads[L.a] = dxa
                grads[L.b] = dxb  # first contribution to the skip's gradient
                del dxc
            elif L.a in grads:
                ops.conv3d_bwd_data_bf16(p, self.wt[L.name], g, dx=grads[L.a], accumulate=True)
            else:
                grads[L.a] = ops.conv3d_bwd_data_bf16(p, self.wt[L.name], g)
            del p
            grads.pop(L.name, None)
        return self.grad

    def train_step(self, F, M, target, lr=1e-3):
        """One Adam step on the MSE to target [N, 3, D, H, W]; returns the loss tensor (device)."""
        pred, acts = self.forward(F, M)
        loss, dpred = ops.mse_disp(pred, target)
        self.backward(dpred, acts)
        self.step_count += 1
        ops.adam_step(self.master, self.grad, self.m, self.v, lr=lr, step=self.step_count)
        self.refresh_bf16()
        return loss
