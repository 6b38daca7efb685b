"""Seeded synthetic registration pairs (input generation only).

This module builds the fixed/moving volumes, the known displacement and the
optional multimodal remap used by the tests, the benchmark and the oracle's
timing leg.  It contains none of the registration method's arithmetic: no
trilinear sampling, no window statistics, no histograms.  The moving image is
obtained by evaluating the *continuous* blob model at displaced points, so
M = F o (x + d) holds exactly for the smooth part without any interpolation.

Recipe (stand-in for the paper's clinical 1 mm and 100 um brain volumes, which
are not available; shapes follow the paper's workloads):

* base seed 2025 (the paper's faux-OASIS base seed, App. "faux-OASIS"),
  seed = 2025 + pair index; numpy PCG64 with SeedSequence.spawn sub-streams
  for blobs, noise, displacement, remap and texture.
* F(x) = G(x) + n_F(x),  G = sum of ``n_blobs`` isotropic Gaussians with
  centres uniform in the array, sigma ~ U[sigma_lo, sigma_hi], amplitude ~ U[0,1].
* d(x): each of the three components is a sum of K random Fourier modes whose
  wave vectors are drawn from the spectrum of white noise smoothed by a
  Gaussian of std ``disp_sigma`` voxels; the field is scaled so that
  max_x ||d(x)||_2 equals ``max_disp`` voxels.
* M(x) = G(x + d(x)) + n_M(x).  Noise n_F, n_M ~ N(0, noise_std^2) i.i.d.
  (std, not variance), drawn independently for each image.
* optional band-limited texture T (random Fourier modes, wavelength 3..8
  voxels) added as T(x) to F and T(x + d(x)) to M, std = ``texture_std``.
* each image is min-max normalised to [0, 1].
* multimodal: M <- r(M), r a random cubic whose derivative changes sign on
  (0, 1), then min-max normalised again.

Displacement channel order: d[0] moves x (W axis), d[1] moves y (H), d[2]
moves z (D), matching the displacement-field layout of the library.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

BASE_SEED = 2025


@dataclasses.dataclass(frozen=True)
class PairSpec:
    shape: Tuple[int, int, int]            # (D, H, W)
    sigma_range: Tuple[float, float]       # blob sigma range in voxels
    max_disp: float                        # max ||d||_2 in voxels
    n_blobs: int = 20
    noise_std: float = 0.01
    disp_sigma: float = 6.0
    disp_modes: int = 24
    multimodal: bool = False
    texture_std: float = 0.0               # 0 disables texture
    texture_modes: int = 48


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    names = ("blobs", "noise", "disp", "remap", "texture")
    return {n: np.random.Generator(np.random.PCG64(s)) for n, s in zip(names, ss.spawn(len(names)))}


def _coords(shape, device, dtype):
    D, H, W = shape
    z = torch.arange(D, device=device, dtype=dtype).view(D, 1, 1)
    y = torch.arange(H, device=device, dtype=dtype).view(1, H, 1)
    x = torch.arange(W, device=device, dtype=dtype).view(1, 1, W)
    return z, y, x


def _blob_params(rng, spec: PairSpec):
    D, H, W = spec.shape
    n = spec.n_blobs
    cz = rng.uniform(0, D - 1, n)
    cy = rng.uniform(0, H - 1, n)
    cx = rng.uniform(0, W - 1, n)
    sig = rng.uniform(spec.sigma_range[0], spec.sigma_range[1], n)
    amp = rng.uniform(0.0, 1.0, n)
    return cz, cy, cx, sig, amp


def _eval_blobs(params, pz, py, px, out):
    """Accumulate the continuous blob model G at the points (pz, py, px)."""
    cz, cy, cx, sig, amp = params
    for j in range(len(amp)):
        r2 = (pz - cz[j]) ** 2 + (py - cy[j]) ** 2 + (px - cx[j]) ** 2
        out.add_(torch.exp(r2 * (-0.5 / (sig[j] ** 2))), alpha=float(amp[j]))
    return out


def _eval_modes(modes, pz, py, px, shape, device, dtype):
    """Sum of cosine modes a*cos(k.p + phi) at broadcastable points."""
    out = torch.zeros(shape, device=device, dtype=dtype)
    for (kz, ky, kx, ph, a) in modes:
        out.add_(torch.cos(pz * kz + py * ky + px * kx + ph), alpha=a)
    return out


def _disp_modes(rng, spec: PairSpec):
    # Gaussian smoothing with std s of white noise leaves the power spectrum
    # exp(-s^2 |k|^2): wave-vector components ~ N(0, 1/(2 s^2)).
    sd = 1.0 / (math.sqrt(2.0) * spec.disp_sigma)
    comps = []
    for _ in range(3):
        k = rng.normal(0.0, sd, (spec.disp_modes, 3))
        ph = rng.uniform(0, 2 * math.pi, spec.disp_modes)
        a = rng.normal(0.0, 1.0, spec.disp_modes)
        comps.append([(float(k[i, 0]), float(k[i, 1]), float(k[i, 2]), float(ph[i]), float(a[i]))
                      for i in range(spec.disp_modes)])
    return comps


def _texture_modes(rng, spec: PairSpec):
    n = spec.texture_modes
    lam = rng.uniform(3.0, 8.0, n)                    # wavelength in voxels
    dirs = rng.normal(0.0, 1.0, (n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    k = dirs * (2 * math.pi / lam)[:, None]
    ph = rng.uniform(0, 2 * math.pi, n)
    a = rng.normal(0.0, 1.0, n) / math.sqrt(n / 2.0)  # unit-variance sum
    return [(float(k[i, 0]), float(k[i, 1]), float(k[i, 2]), float(ph[i]), float(a[i])) for i in range(n)]


def _noise(rng, shape, std, device, on_device=False):
    seed = int(rng.integers(0, 2**62))
    if on_device and torch.device(device).type != "cpu":
        # fast path for bulk training data: the device's own generator (not
        # bitwise identical to the host stream, but seeded and repeatable)
        g = torch.Generator(device=device).manual_seed(seed)
        return torch.randn(shape, generator=g, dtype=torch.float32, device=device) * std
    g = torch.Generator(device="cpu").manual_seed(seed)
    return (torch.randn(shape, generator=g, dtype=torch.float32) * std).to(device)


def _minmax_(t):
    lo, hi = t.min(), t.max()
    t.sub_(lo).div_(hi - lo)
    return t


def _remap_coeffs(rng):
    while True:
        c = rng.normal(0.0, 1.0, 4)
        # r'(t) = c1 + 2 c2 t + 3 c3 t^2 changes sign on (0, 1)?
        ts = np.linspace(0.0, 1.0, 1001)
        dr = c[1] + 2 * c[2] * ts + 3 * c[3] * ts ** 2
        if dr.min() < 0.0 < dr.max():
            return c


def make_pair(spec: PairSpec, seed: int = BASE_SEED, device="cpu",
              with_disp: bool = True, z_range: Optional[Tuple[int, int]] = None, noise_on_device: bool = False,
              grid: Optional[Tuple[int, int, int]] = None):
    """Return dict(F, M, d) as float32 tensors on ``device``.

    ``z_range`` restricts evaluation to slices [z0, z1) of the full volume (the
    random parameters and the normalisation constants are those of the full
    volume only when the whole volume is generated; slab generation is for
    memory-bounded timing samples and uses the slab's own min/max).

    ``grid`` (Dc, Hc, Wc) evaluates the same continuous pair on a coarser
    corner-aligned grid (point i of an axis sits at i (n - 1)/(nc - 1) voxels
    of the full volume): the pair a downsampling of the full volume would
    see, without generating it.  d is then in the coarse grid's voxels, and
    the displacement scale, noise and normalisation come from the grid's own
    points."""
    st = _streams(seed)
    D, H, W = spec.shape
    dt = torch.float64
    if grid is not None:
        if z_range is not None:
            raise ValueError("grid and z_range are exclusive")
        shape = tuple(int(g) for g in grid)
        z, y, x = _coords(shape, device, dt)
        fs = [(n - 1) / (c - 1) if c > 1 else 0.0 for n, c in zip(spec.shape, shape)]  # full voxels per grid step
        z, y, x = z * fs[0], y * fs[1], x * fs[2]
    else:
        z0, z1 = (0, D) if z_range is None else z_range
        shape = (z1 - z0, H, W)
        z, y, x = _coords(spec.shape, device, dt)
        z = z[z0:z1]
    blobs = _blob_params(st["blobs"], spec)
    dmodes = _disp_modes(st["disp"], spec)
    tmodes = _texture_modes(st["texture"], spec) if spec.texture_std > 0 else None

    # known displacement, scaled to max norm; the scale is set on the full volume
    d = torch.stack([_eval_modes(dmodes[c], z, y, x, shape, device, dt) for c in range(3)])
    if z_range is None:  # the whole volume, or the coarse grid's points
        peak = torch.sqrt((d * d).sum(0)).max()
    else:  # scale from the full volume, computed slab-wise to bound memory
        peak = torch.zeros((), device=device, dtype=dt)
        zz, yy, xx = _coords(spec.shape, device, dt)
        step = max(1, (1 << 24) // (H * W))
        for a in range(0, D, step):
            b = min(D, a + step)
            dd = torch.stack([_eval_modes(dmodes[c], zz[a:b], yy, xx, (b - a, H, W), device, dt)
                              for c in range(3)])
            peak = torch.maximum(peak, torch.sqrt((dd * dd).sum(0)).max())
    d.mul_(spec.max_disp / peak)

    Fv = _eval_blobs(blobs, z, y, x, torch.zeros(shape, device=device, dtype=dt))
    # sample points x + d(x): channel 0 is x, 1 is y, 2 is z
    pz, py, px = z + d[2], y + d[1], x + d[0]
    Mv = _eval_blobs(blobs, pz, py, px, torch.zeros(shape, device=device, dtype=dt))
    if tmodes is not None:
        Fv.add_(_eval_modes(tmodes, z, y, x, shape, device, dt), alpha=spec.texture_std)
        Mv.add_(_eval_modes(tmodes, pz, py, px, shape, device, dt), alpha=spec.texture_std)
    del pz, py, px
    Fv.add_(_noise(st["noise"], shape, spec.noise_std, device, noise_on_device))
    Mv.add_(_noise(st["noise"], shape, spec.noise_std, device, noise_on_device))
    _minmax_(Fv)
    _minmax_(Mv)
    if spec.multimodal:
        c = _remap_coeffs(st["remap"])
        Mv = c[0] + Mv * (c[1] + Mv * (c[2] + Mv * c[3]))
        _minmax_(Mv)
    out = {"F": Fv.to(torch.float32).contiguous(), "M": Mv.to(torch.float32).contiguous()}
    if with_disp:
        if grid is not None:  # full-volume voxels -> grid voxels (channel 0 is x)
            for c, f in enumerate((fs[2], fs[1], fs[0])):
                d[c].mul_(1.0 / f if f > 0 else 0.0)
        out["d"] = d.to(torch.float32).contiguous()
    return out



def make_affine_pair(spec: PairSpec, B, c, seed: int = BASE_SEED, device="cpu"):
    """Pair related by a known affine map: F(X) = G(X), M(X) = G(B X + c)
    (X = (x, y, z) voxel coordinates, B 3x3 row-major, c 3-vector; blobs,
    texture and independent noise as in make_pair).  Returns dict(F, M, A, t)
    with A = B^-1, t = -B^-1 c, the transform for which M(A X + t) = G(X)."""
    st = _streams(seed)
    D, H, W = spec.shape
    dt = torch.float64
    z, y, x = _coords(spec.shape, device, dt)
    B = np.asarray(B, dtype=np.float64).reshape(3, 3)
    c = np.asarray(c, dtype=np.float64).reshape(3)
    blobs = _blob_params(st["blobs"], spec)
    _disp_modes(st["disp"], spec)  # keeps the stream layout of make_pair
    tmodes = _texture_modes(st["texture"], spec) if spec.texture_std > 0 else None
    px = B[0, 0] * x + B[0, 1] * y + B[0, 2] * z + c[0]
    py = B[1, 0] * x + B[1, 1] * y + B[1, 2] * z + c[1]
    pz = B[2, 0] * x + B[2, 1] * y + B[2, 2] * z + c[2]
    shape = (D, H, W)
    Fv = _eval_blobs(blobs, z, y, x, torch.zeros(shape, device=device, dtype=dt))
    Mv = _eval_blobs(blobs, pz, py, px, torch.zeros(shape, device=device, dtype=dt))
    if tmodes is not None:
        Fv.add_(_eval_modes(tmodes, z, y, x, shape, device, dt), alpha=spec.texture_std)
        Mv.add_(_eval_modes(tmodes, pz, py, px, shape, device, dt), alpha=spec.texture_std)
    Fv.add_(_noise(st["noise"], shape, spec.noise_std, device))
    Mv.add_(_noise(st["noise"], shape, spec.noise_std, device))
    _minmax_(Fv)
    _minmax_(Mv)
    Bi = np.linalg.inv(B)
    return {"F": Fv.to(torch.float32).contiguous(), "M": Mv.to(torch.float32).contiguous(),
            "A": Bi, "t": -Bi @ c}

def random_volume(shape: Sequence[int], seed: int, device="cpu", lo=0.0, hi=1.0):
    """i.i.d. uniform volume (edge-case and tiny-shape tests)."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    return (torch.rand(tuple(shape), generator=g, dtype=torch.float32) * (hi - lo) + lo).to(device)


def random_disp(shape: Sequence[int], seed: int, scale: float, device="cpu", avoid_kinks: bool = False):
    """i.i.d. displacement field [3, D, H, W]; with ``avoid_kinks`` the
    fractional part of every component lies in [0.1, 0.9] so that finite
    differences never straddle an integer sample coordinate."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    u = (torch.rand((3,) + tuple(shape), generator=g, dtype=torch.float64) * 2 - 1) * scale
    if avoid_kinks:
        f = torch.floor(u)
        frac = u - f
        u = f + 0.1 + 0.8 * frac
    return u.to(torch.float32).to(device)
