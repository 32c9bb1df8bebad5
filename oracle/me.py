"""Oracle (test infrastructure only): motion estimation by pixel-wise
template matching, Sec. 2.2 (recursive FSR).

For each pixel p of the current frame t the motion vector into a past frame
t-k is found by matching a small template of the *measured* pixels of frame t
around p against the *already reconstructed* frame t-k (Sec. 2.2, Fig. 2a).
The paper gives no template size, boundary rule or tie rule; the readings used
here (all integer, so there is exactly one correct answer):

  * Template offsets D = {lo .. lo+T-1}^2 with lo = -floor((T-1)/2); for T=4
    that is {-1, 0, 1, 2}^2.
  * Cost S(p, v) = sum_{d in D} [p+d in frame] * b_t(p+d) * |f_t(p+d) - Rhat(clamp(p+d+v))|,
    where b_t is the current mask, f_t the measured frame and Rhat the
    reconstruction of frame t-k read with clamp-to-edge.
  * n(p) = sum_{d in D} [p+d in frame] * b_t(p+d), the number of template
    pixels that carry a measurement.
  * A candidate v is evaluated only if p+v lies inside the frame.
  * v in [-R, R]^2.  The minimiser uses the total order
    (S, |v|_1, raster index of v with the row offset outer, column inner).

Motion vectors are (alpha, beta) = (row offset, column offset).
"""
from __future__ import annotations

import numpy as np


def template_offsets(T: int) -> np.ndarray:
    """1-D template offsets {lo .. lo+T-1}, lo = -floor((T-1)/2)."""
    lo = -((T - 1) // 2)
    return np.arange(lo, lo + T, dtype=np.int64)


def _inside(y, x, H, W):
    return (y >= 0) & (y < H) & (x >= 0) & (x < W)


def cost_at(cur, mask, ref, py, px, vy, vx, T=4):
    """S(p, v) and n(p) for broadcastable integer arrays of p and v.

    Written out as the definition: one term per template offset d.
    Unmeasured positions of `cur` are never used (their term is multiplied
    by an integer 0 mask, and they are read only where the mask is 1).
    """
    H, W = cur.shape
    py, px, vy, vx = (np.asarray(a, np.int64) for a in (py, px, vy, vx))
    shape = np.broadcast_shapes(py.shape, px.shape, vy.shape, vx.shape)
    S = np.zeros(shape, np.int64)
    n = np.zeros(shape, np.int64)
    for dy in template_offsets(T):
        for dx in template_offsets(T):
            qy, qx = py + dy, px + dx
            ins = _inside(qy, qx, H, W)
            qyc, qxc = np.clip(qy, 0, H - 1), np.clip(qx, 0, W - 1)
            b = np.where(ins, mask[qyc, qxc], 0).astype(np.int64)
            f = np.where(b == 1, cur[qyc, qxc], 0).astype(np.int64)
            r = ref[np.clip(qy + vy, 0, H - 1), np.clip(qx + vx, 0, W - 1)].astype(np.int64)
            S = S + b * np.abs(f - r)
            n = n + b
    return S, n


def reverse_cost_at(cur, mask, ref, qy, qx, uy, ux, T=4):
    """Cost of the *reverse* match used by reverse motion estimation:
    the template is cut from the reconstruction Rhat around q (clamp-to-edge)
    and compared with the measured pixels of the current frame around q+u.

      S_rev(q, u) = sum_d [q+u+d in frame] b_t(q+u+d) |f_t(q+u+d) - Rhat(clamp(q+d))|
      n_rev(q, u) = sum_d [q+u+d in frame] b_t(q+u+d)

    (Written independently of `cost_at`; S_rev(q,u) = S(q+u, -u) is a test.)
    """
    H, W = cur.shape
    qy, qx, uy, ux = (np.asarray(a, np.int64) for a in (qy, qx, uy, ux))
    shape = np.broadcast_shapes(qy.shape, qx.shape, uy.shape, ux.shape)
    S = np.zeros(shape, np.int64)
    n = np.zeros(shape, np.int64)
    for dy in template_offsets(T):
        for dx in template_offsets(T):
            tmpl = ref[np.clip(qy + dy, 0, H - 1), np.clip(qx + dx, 0, W - 1)].astype(np.int64)
            sy, sx = qy + uy + dy, qx + ux + dx
            ins = _inside(sy, sx, H, W)
            syc, sxc = np.clip(sy, 0, H - 1), np.clip(sx, 0, W - 1)
            b = np.where(ins, mask[syc, sxc], 0).astype(np.int64)
            f = np.where(b == 1, cur[syc, sxc], 0).astype(np.int64)
            S = S + b * np.abs(f - tmpl)
            n = n + b
    return S, n


def n_map(mask, T=4):
    """n(p) for every pixel of the frame."""
    H, W = mask.shape
    y, x = np.mgrid[0:H, 0:W]
    n = np.zeros((H, W), np.int64)
    for dy in template_offsets(T):
        for dx in template_offsets(T):
            qy, qx = y + dy, x + dx
            ins = _inside(qy, qx, H, W)
            n += np.where(ins, mask[np.clip(qy, 0, H - 1), np.clip(qx, 0, W - 1)], 0)
    return n


def _candidates(R: int):
    """Candidates in raster order (row offset outer, column offset inner)."""
    for vy in range(-R, R + 1):
        for vx in range(-R, R + 1):
            yield vy, vx


def forward_me(cur, mask, ref, R, T=4):
    """Full-search forward motion estimation for every pixel.

    Returns (alpha, beta, S, n): int arrays (H, W); (alpha, beta) is the
    minimiser of (S, |v|_1, raster(v)) over valid candidates, S its cost,
    n the number of measured template pixels.
    """
    H, W = cur.shape
    y, x = np.mgrid[0:H, 0:W]
    best_S = np.full((H, W), np.iinfo(np.int64).max, np.int64)
    best_l1 = np.full((H, W), np.iinfo(np.int64).max, np.int64)
    alpha = np.zeros((H, W), np.int64)
    beta = np.zeros((H, W), np.int64)
    n = None
    for vy, vx in _candidates(R):
        S, n = cost_at(cur, mask, ref, y, x, vy, vx, T)
        valid = _inside(y + vy, x + vx, H, W)
        l1 = abs(vy) + abs(vx)
        better = valid & ((S < best_S) | ((S == best_S) & (l1 < best_l1)))
        best_S = np.where(better, S, best_S)
        best_l1 = np.where(better, l1, best_l1)
        alpha = np.where(better, vy, alpha)
        beta = np.where(better, vx, beta)
    return alpha, beta, best_S, n


def forward_me_at(cur, mask, ref, ys, xs, R, T=4):
    """Forward motion estimation at selected pixels only (same result as
    `forward_me` at those pixels); vectorised over the candidates."""
    H, W = cur.shape
    ys = np.asarray(ys, np.int64)
    xs = np.asarray(xs, np.int64)
    cand = np.array(list(_candidates(R)), np.int64)
    vy, vx = cand[:, 0], cand[:, 1]
    out = []
    for py, px in zip(ys, xs):
        S, n = cost_at(cur, mask, ref, py, px, vy, vx, T)
        valid = _inside(py + vy, px + vx, H, W)
        l1 = np.abs(vy) + np.abs(vx)
        raster = np.arange(cand.shape[0])
        # lexicographic (S, l1, raster) over valid candidates
        order = np.lexsort((raster, l1, np.where(valid, S, np.iinfo(np.int64).max)))
        k = order[0]
        out.append((vy[k], vx[k], S[k], n[k]))
    a = np.array(out, np.int64).reshape(-1, 4)
    return a[:, 0], a[:, 1], a[:, 2], a[:, 3]
