"""Pins of the oracle's Adam update (O5): torch.optim.Adam in float64 and the
closed-form first step.  The paper's registration loop keeps first and second
moment states per voxel of the displacement (Sec. "Grid Parallel")."""
import numpy as np
import torch


def test_matches_torch_adam_over_several_steps(orc):
    rng = np.random.default_rng(50)
    n = 257
    x = rng.normal(size=n)
    xt = torch.tensor(x.copy(), requires_grad=True)
    opt = torch.optim.Adam([xt], lr=0.1, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(n)
    v = np.zeros(n)
    for step in range(1, 8):
        g = rng.normal(size=n) * (10.0 ** rng.integers(-3, 2))
        orc.adam(x, g.copy(), m, v, lr=0.1, step=step)
        xt.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(x, xt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_first_step_closed_form_and_zero_gradient():
    import oracle
    g = np.array([3.0, -0.5, 0.0, 1e-9])
    x = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    oracle.adam(x, g, m, v, lr=0.1, step=1)
    ref = -0.1 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(x, ref, rtol=1e-14, atol=0)
    assert x[2] == 0.0
