"""Oracle (test infrastructure only): projection of measured past pixels,
Sec. 2.2.

For a missing pixel of the current frame, an accepted motion vector that
points to a *measured* pixel of a past frame projects that measurement into
the current frame; if several past frames supply one, they are averaged.
Only measurements are projected, never reconstructed values.

Output classes: 0 unknown, 1 measured, 2 projected.
"""
from __future__ import annotations

import numpy as np


def project(cur, cur_mask, refs):
    """refs: sequence of dicts with keys alpha, beta, accept (bool), meas
    (uint8 measured frame t-k) and mask (uint8 mask of frame t-k).

    Returns (values float64 (H,W), cls uint8 (H,W)).  values holds the
    measurement at class 1, the projected mean at class 2, 0 elsewhere.
    """
    H, W = cur.shape
    y, x = np.mgrid[0:H, 0:W]
    missing = cur_mask == 0
    total = np.zeros((H, W), np.int64)
    count = np.zeros((H, W), np.int64)
    for r in refs:
        qy, qx = y + r["alpha"], x + r["beta"]
        assert ((qy >= 0) & (qy < H) & (qx >= 0) & (qx < W)).all()
        ok = missing & r["accept"] & (r["mask"][qy, qx] == 1)
        total += np.where(ok, r["meas"][qy, qx], 0).astype(np.int64)
        count += ok
    values = np.zeros((H, W), np.float64)
    cls = np.zeros((H, W), np.uint8)
    meas = cur_mask == 1
    values[meas] = cur[meas]
    cls[meas] = 1
    proj = missing & (count > 0)
    values[proj] = total[proj] / count[proj]
    cls[proj] = 2
    return values, cls
