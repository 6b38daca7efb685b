"""Oracle pins for the Gaussian field smoothing (the sigma_grad / sigma_warp
regulariser of the paper's registration runs): agreement with an independent
library filter, the impulse response, and invariants a wrong tap, radius,
normalisation or boundary rule would break."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle


def _taps(sigma):
    R = int(np.ceil(3 * sigma))
    t = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-t * t / (2 * sigma * sigma))
    return g / g.sum(), R


@pytest.mark.parametrize("sigma", [0.5, 1.0, 0.7, 1.6])
def test_matches_scipy_gaussian_filter(sigma):
    """scipy's separable filter with edge replication ('nearest') and the same
    truncation radius ceil(3 sigma)."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 9, 11, 13)).astype(np.float32)
    got = oracle.gaussian_smooth(x, sigma)
    R = int(np.ceil(3 * sigma))
    for c in range(2):
        ref = ndi.gaussian_filter(x[c].astype(np.float64), sigma, mode="nearest", radius=R)
        np.testing.assert_allclose(got[c], ref, rtol=0, atol=1e-13)


def test_impulse_response_is_product_of_taps():
    g, R = _taps(1.0)
    x = np.zeros((15, 15, 15), np.float32)
    x[7, 7, 7] = 1.0
    y = oracle.gaussian_smooth(x, 1.0)
    ref = np.zeros((15, 15, 15))
    ref[7 - R:8 + R, 7 - R:8 + R, 7 - R:8 + R] = g[:, None, None] * g[None, :, None] * g[None, None, :]
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-16)
    assert abs(y.sum() - 1.0) < 1e-14


def test_constant_field_is_fixed_everywhere():
    """Normalised taps and edge replication keep a constant field constant,
    including at the array faces (zero padding would not)."""
    x = np.full((3, 6, 7, 8), 2.5, np.float32)
    y = oracle.gaussian_smooth(x, 1.0)
    np.testing.assert_allclose(y, 2.5, rtol=0, atol=1e-14)


def test_linear_field_is_fixed_in_the_interior():
    """A symmetric kernel reproduces affine functions away from the faces;
    at the faces replication bends them toward the edge value."""
    R = 3
    z, y, x = np.meshgrid(np.arange(12), np.arange(13), np.arange(14), indexing="ij")
    f = (0.5 * x - 0.25 * y + 0.125 * z).astype(np.float32)
    s = oracle.gaussian_smooth(f, 1.0)
    inner = (slice(R, -R),) * 3
    np.testing.assert_allclose(s[inner], f[inner], rtol=0, atol=1e-13)
    assert s[0, 0, 0] > f[0, 0, 0]  # low corner rises: replication, not extrapolation


def test_brute_force_tiny():
    """Pure-Python sum over the clamped neighbourhood on a 3 x 4 x 5 array."""
    sigma = 0.5
    g, R = _taps(sigma)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 4, 5)).astype(np.float32)
    y = oracle.gaussian_smooth(x, sigma)
    D, H, W = x.shape
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                acc = 0.0
                for a in range(-R, R + 1):
                    for b in range(-R, R + 1):
                        for c in range(-R, R + 1):
                            acc += (g[a + R] * g[b + R] * g[c + R] *
                                    float(x[min(max(z + a, 0), D - 1), min(max(yy + b, 0), H - 1),
                                            min(max(xx + c, 0), W - 1)]))
                assert abs(y[z, yy, xx] - acc) < 1e-13


def test_rejects_nonpositive_sigma():
    with pytest.raises(ValueError):
        oracle.gaussian_smooth(np.zeros((2, 2, 2), np.float32), 0.0)
