"""Host-side logic of the registration driver (no GPU)."""
from paper_2509_25044_amd.register import RegConfig, axis_scales, level_shapes


def test_level_shapes():
    assert level_shapes((160, 192, 224), (0.25, 0.5, 1.0)) == [(40, 48, 56), (80, 96, 112), (160, 192, 224)]
    assert level_shapes((5, 3, 1), (0.5,)) == [(2, 2, 1)]


def test_axis_scales_corner_aligned():
    sx, sy, sz = axis_scales((80, 96, 112), (160, 192, 224))
    assert abs(sx - 223 / 111) < 1e-15 and abs(sy - 191 / 95) < 1e-15 and abs(sz - 159 / 79) < 1e-15
    assert axis_scales((1, 1, 1), (4, 4, 4)) == (1.0, 1.0, 1.0)


def test_config_defaults():
    c = RegConfig()
    assert c.loss == "lncc" and c.betas == (0.9, 0.999) and c.lr == 0.1
