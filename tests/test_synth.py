"""The seeded input generator: determinism, ranges and the known displacement."""
import numpy as np
import torch

from paper_2509_25044_amd import synth
from paper_2509_25044_amd.configs import C1, C2


def test_deterministic_and_normalised():
    a = synth.make_pair(C1.pair, seed=2025)
    b = synth.make_pair(C1.pair, seed=2025)
    for k in ("F", "M", "d"):
        assert torch.equal(a[k], b[k])
    for k in ("F", "M"):
        assert float(a[k].min()) == 0.0 and float(a[k].max()) == 1.0
    nrm = torch.sqrt((a["d"].double() ** 2).sum(0))
    assert abs(float(nrm.max()) - C1.pair.max_disp) < 1e-5
    c = synth.make_pair(C1.pair, seed=2026)
    assert not torch.equal(a["F"], c["F"])


def test_multimodal_remap_is_not_monotone():
    spec = synth.PairSpec((24, 28, 32), (4.0, 12.0), 3.0, multimodal=True)
    p = synth.make_pair(spec, seed=2025)
    assert float(p["M"].min()) == 0.0 and float(p["M"].max()) == 1.0
    st = synth._streams(2025)
    c = synth._remap_coeffs(st["remap"])
    t = np.linspace(0, 1, 101)
    dr = c[1] + 2 * c[2] * t + 3 * c[3] * t ** 2
    assert dr.min() < 0 < dr.max()


def test_moving_image_follows_the_known_displacement():
    """Without noise, M(x) equals the continuous blob model at x + d(x)."""
    spec = synth.PairSpec((16, 16, 16), (3.0, 5.0), 2.0, noise_std=0.0)
    p = synth.make_pair(spec, seed=7)
    assert p["d"].shape == (3, 16, 16, 16)
    assert not torch.equal(p["F"], p["M"])
    spec0 = synth.PairSpec((16, 16, 16), (3.0, 5.0), 1e-30, noise_std=0.0)
    q = synth.make_pair(spec0, seed=7)
    assert torch.allclose(q["F"], q["M"], atol=1e-6)


def test_clinical_shape():
    assert C2.shape == (160, 192, 224)


def test_coarse_grid_is_the_subsampled_continuous_pair():
    """make_pair(grid=...) evaluates the same continuous pair at the corner-
    aligned coarse points: with noise off, F equals the full volume's every
    4th voxel once both are min-max normalised over those points, d is the
    full displacement in coarse voxels up to the max-norm scale (taken over
    the coarse points), and M differs only through that scale."""
    spec = synth.PairSpec((33, 41, 49), (2.0, 5.0), 3.0, noise_std=0.0, texture_std=0.05)
    full = synth.make_pair(spec, seed=11)
    co = synth.make_pair(spec, seed=11, grid=(9, 11, 13))
    assert co["F"].shape == (9, 11, 13) and co["d"].shape == (3, 9, 11, 13)

    def renorm(t):
        t = t.double()
        return (t - t.min()) / (t.max() - t.min())

    assert torch.allclose(renorm(full["F"][::4, ::4, ::4]), co["F"].double(), atol=2e-6)
    assert torch.allclose(renorm(full["M"][::4, ::4, ::4]), co["M"].double(), atol=2e-2)
    ratio = co["d"].double() / (full["d"][:, ::4, ::4, ::4].double() / 4.0)
    big = full["d"][:, ::4, ::4, ::4].abs() > 0.05
    r = ratio[big]
    assert float(r.max() - r.min()) < 1e-5 and abs(float(r.mean()) - 1.0) < 0.05
