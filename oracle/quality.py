"""Oracle (test infrastructure only): frame quality measures of Sec. 4.

PSNR lives in `frame.py`.  This module adds the mean structural similarity
the paper reports beside PSNR (Sec. 4, with reference to Wang, Bovik,
Sheikh, Simoncelli, "Image quality assessment: from error visibility to
structural similarity", IEEE TIP 2004).

Definition used (the SSIM paper's standard setting): for every 11x11 window
of the two images, weighted by a circular-symmetric Gaussian of standard
deviation 1.5 samples normalised to unit sum,
    SSIM = ((2 mu_x mu_y + C1) (2 s_xy + C2)) / ((mu_x^2 + mu_y^2 + C1) (s_x^2 + s_y^2 + C2))
with weighted means mu, weighted (co)variances s, C1 = (0.01 L)^2,
C2 = (0.03 L)^2, L = 255; the mean SSIM is the average over all window
positions that lie inside the image (no padding).

Readings: the paper evaluates SSIM "in the same manner" as PSNR, so the
40-pixel border is removed first and the reconstruction is clipped to
[0, 255] without rounding, as for PSNR.
"""
from __future__ import annotations

import numpy as np

K1, K2, L = 0.01, 0.03, 255.0


def gaussian_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """(size, size) Gaussian weights, unit sum (outer product of the 1-D
    normalised Gaussian, which is the same as normalising the 2-D one)."""
    g = _gauss1d(size, sigma)
    return np.outer(g, g)


def _prepare(ref, test, border):
    ref = np.asarray(ref, np.float64)
    test = np.clip(np.asarray(test, np.float64), 0.0, 255.0)
    H, W = ref.shape
    sl = (slice(border, H - border), slice(border, W - border))
    return ref[sl], test[sl]


def _gauss1d(size: int, sigma: float) -> np.ndarray:
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x ** 2 / (2.0 * sigma ** 2))
    return g / g.sum()


def _filter_valid(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Weighted sums sum_{u,v} g[u] g[v] img[y+u, x+v] over every window that
    fits in the image.  The window is the outer product g g^T, so the double
    sum is a 1-D weighted sum along the rows followed by one along the
    columns (sliding windows + tensordot as the library primitive)."""
    rows = np.tensordot(np.lib.stride_tricks.sliding_window_view(img, g.size, axis=1), g, axes=([2], [0]))
    return np.tensordot(np.lib.stride_tricks.sliding_window_view(rows, g.size, axis=0), g, axes=([2], [0]))


def ssim_map(ref, test, border: int = 40, size: int = 11, sigma: float = 1.5) -> np.ndarray:
    x, y = _prepare(ref, test, border)
    w = _gauss1d(size, sigma)
    C1, C2 = (K1 * L) ** 2, (K2 * L) ** 2
    mx, my = _filter_valid(x, w), _filter_valid(y, w)
    sxx = _filter_valid(x * x, w) - mx * mx
    syy = _filter_valid(y * y, w) - my * my
    sxy = _filter_valid(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(ref, test, border: int = 40, size: int = 11, sigma: float = 1.5) -> float:
    """Mean SSIM of `test` against `ref` (both H x W), border removed."""
    return float(np.mean(ssim_map(ref, test, border, size, sigma)))


def ssim_bruteforce(ref, test, border: int = 0, size: int = 11, sigma: float = 1.5) -> float:
    """The same quantity written as loops over windows with centred
    (co)variances (small images only)."""
    x, y = _prepare(ref, test, border)
    w = gaussian_window(size, sigma)
    C1, C2 = (K1 * L) ** 2, (K2 * L) ** 2
    H, W = x.shape
    vals = []
    for i in range(H - size + 1):
        for j in range(W - size + 1):
            px, py = x[i:i + size, j:j + size], y[i:i + size, j:j + size]
            mx, my = (w * px).sum(), (w * py).sum()
            sx = (w * (px - mx) ** 2).sum()
            sy = (w * (py - my) ** 2).sum()
            sxy = (w * (px - mx) * (py - my)).sum()
            vals.append(((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2)))
    return float(np.mean(vals))
