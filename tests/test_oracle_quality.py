"""Pins of the oracle's mean SSIM (Sec. 4, SSIM of Wang et al. 2004)."""
import numpy as np
import pytest

import oracle as O


def test_window_is_normalised_symmetric_gaussian():
    w = O.gaussian_window()
    assert w.shape == (11, 11)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    # ratio of neighbouring weights along an axis through the centre: exp(-(2k+1)/(2 sigma^2))
    r = w[5, 6] / w[5, 5]
    assert r == pytest.approx(np.exp(-1.0 / (2 * 1.5 ** 2)), rel=1e-12)
    assert w[5, 5] == w.max()


def test_identical_images_have_ssim_one():
    rng = np.random.default_rng(0)
    x = rng.integers(0, 256, (40, 52)).astype(np.float64)
    assert O.ssim(x, x, border=0) == pytest.approx(1.0, abs=1e-12)


def test_constant_images_closed_form():
    """Flat windows: variances vanish, SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 100.0, 140.0
    x = np.full((20, 20), a)
    y = np.full((20, 20), b)
    C1 = (0.01 * 255) ** 2
    assert O.ssim(x, y, border=0) == pytest.approx((2 * a * b + C1) / (a * a + b * b + C1), rel=1e-12)


def test_vectorised_form_equals_window_loops():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, (19, 23)).astype(np.float64)
    y = np.clip(x + rng.normal(0, 20, x.shape), -10, 270)   # clipping of the test image included
    assert O.ssim(x, y, border=0) == pytest.approx(O.ssim_bruteforce(x, y, border=0), abs=1e-12)
    assert O.ssim(x, y, border=2) == pytest.approx(O.ssim_bruteforce(x, y, border=2), abs=1e-12)


def test_symmetry_bounds_and_monotone_in_noise():
    rng = np.random.default_rng(2)
    x = 128 + 40 * rng.standard_normal((48, 48))
    x = np.clip(x, 0, 255)
    vals = []
    for s in (2.0, 8.0, 32.0):
        y = np.clip(x + s * rng.standard_normal(x.shape), 0, 255)
        v = O.ssim(x, y, border=0)
        assert v == pytest.approx(O.ssim(y, x, border=0), abs=1e-12)
        assert -1.0 <= v < 1.0
        vals.append(v)
    assert vals[0] > vals[1] > vals[2]


def test_border_is_removed():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (100, 100)).astype(np.float64)
    y = x.copy()
    y[:40, :] = 0      # damage only inside the 40-pixel border
    assert O.ssim(x, y, border=40) == pytest.approx(1.0, abs=1e-12)
    assert O.ssim(x, y, border=0) < 0.9
