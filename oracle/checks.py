"""Oracle (test infrastructure only): consistency checks of the motion field.

RME (Sec. 2.2): the literature check.  A full reverse motion estimation is
run from the reference frame back into the current frame, and a forward
vector is accepted only if the two vectors coincide.

RMC (Sec. 3.1.1, Fig. 2b): the same number of reverse candidates as RME,
placed symmetrically around the vector that points back to the original
pixel.  FRMC (Sec. 3.1.1, Fig. 2c): only offsets {-7,-3,-1,0,1,3,7} per axis
(49 candidates instead of 361).  The motion is accepted if the back-pointing
("green") candidate has the lowest cost; if any other ("red") candidate has
the lowest cost it is rejected.

NNC (Sec. 3.1.2, Eq. (1), Fig. 2d): component-wise 3x3 median of the field;
accepted only if, for each of the four nearest neighbours, the sum of the
absolute component differences of the *filtered* vectors is at most one.
Used in cascade with FRMC: FRMC is evaluated only where NNC accepted.

Readings (the paper is silent or garbled):
  * Reverse cost of candidate u at q = p+v is S(q+u, -u) normalised by
    n(q+u) (template from the reconstruction, search over the measured
    pixels of the current frame; different candidates have different n).
    Normalised costs are compared exactly by cross-multiplication.
  * RME: reverse minimiser with total order (S/n, |u|_1, raster(u)); the
    vectors "coincide" iff u* = -v exactly.
  * RMC/FRMC: red candidate d != 0 is the reverse vector from q back to p+d,
    with cost S(p+d, v-d)/n(p+d); reds with p+d outside the frame are
    skipped; green must be *strictly* lowest (a tie means a red arrow has the
    lowest cost).  RMC uses offsets [-R, R]^2.  The Fig. 2 caption prints the
    small RMC range as {-2,-1,0,-1,2}; it is read as {-2,-1,0,1,2}.
  * NNC: borders of the median replicate the edge; neighbours outside the
    frame are not compared.  The filtered vector at p is compared with the
    filtered vectors at the neighbours; the raw vector is the one projected.

Options beside these readings (defaults give the readings above):
  * cost_norm=False compares raw S instead of S/n in RME, RMC and FRMC (an
    ablation of the normalisation reading);
  * nnc_center="raw" compares the raw vector at p with the filtered vectors
    of its neighbours (the other reading of Sec. 3.1.2);
  * frmc: any per-axis offset set for FRMC (containing 0), e.g. the small
    range {-2,-1,0,1,2} of the Fig. 2 caption.
"""
from __future__ import annotations

import numpy as np

from .me import cost_at, reverse_cost_at, _inside

CHECKS = ("none", "rme", "rmc", "frmc", "nnc", "nnc_frmc")


def frmc_offsets():
    """Per-axis FRMC offsets (Sec. 3.1.1)."""
    return np.array([-7, -3, -1, 0, 1, 3, 7], np.int64)


def rmc_offsets(R):
    """Per-axis RMC offsets: all of [-R, R] (Sec. 3.1.1)."""
    return np.arange(-R, R + 1, dtype=np.int64)


def reverse_me(cur, mask, ref, R, T=4, cost_norm=True):
    """Reverse motion field: for every q, the minimiser u* of
    (S_rev(q,u)/n_rev(q,u), |u|_1, raster(u)) over u in [-R,R]^2 with q+u in
    the frame (raw S_rev in place of S_rev/n_rev when not cost_norm).
    Returns (ualpha, ubeta, evaluations)."""
    H, W = cur.shape
    y, x = np.mgrid[0:H, 0:W]
    has = np.zeros((H, W), bool)
    bS = np.zeros((H, W), np.int64)
    bn = np.ones((H, W), np.int64)
    bl1 = np.zeros((H, W), np.int64)
    ua = np.zeros((H, W), np.int64)
    ub = np.zeros((H, W), np.int64)
    evals = 0
    for uy in range(-R, R + 1):
        for ux in range(-R, R + 1):
            S, n = reverse_cost_at(cur, mask, ref, y, x, uy, ux, T)
            if not cost_norm:
                n = np.ones_like(n)
            valid = _inside(y + uy, x + ux, H, W)
            evals += int(valid.sum())
            l1 = abs(uy) + abs(ux)
            lhs, rhs = S * bn, bS * n          # S/n  vs  bS/bn
            better = valid & (~has | (lhs < rhs) | ((lhs == rhs) & (l1 < bl1)))
            bS = np.where(better, S, bS)
            bn = np.where(better, n, bn)
            bl1 = np.where(better, l1, bl1)
            ua = np.where(better, uy, ua)
            ub = np.where(better, ux, ub)
            has |= better
    return ua, ub, evals


def rme_accept(alpha, beta, ualpha, ubeta):
    """Accept p iff the reverse vector at q = p+v equals -v."""
    H, W = alpha.shape
    y, x = np.mgrid[0:H, 0:W]
    qy, qx = y + alpha, x + beta
    assert _inside(qy, qx, H, W).all()
    return (ualpha[qy, qx] == -alpha) & (ubeta[qy, qx] == -beta)


def rmc_accept(cur, mask, ref, alpha, beta, offsets, T=4, where=None, cost_norm=True):
    """Reverse motion check with per-axis `offsets` (RMC or FRMC).

    Accept p iff for every d in offsets^2 \\ {0} with p+d in the frame:
        S(p,v)/n(p) < S(p+d, v-d)/n(p+d)
    (S(p,v) < S(p+d, v-d) when not cost_norm).
    `where` (bool array) restricts evaluation; elsewhere the result is False.
    Returns (accept, evaluations) where evaluations counts the red
    candidates inside the frame at evaluated pixels (no early exit).
    """
    H, W = cur.shape
    y, x = np.mgrid[0:H, 0:W]
    if where is None:
        where = np.ones((H, W), bool)
    Sg, ng = cost_at(cur, mask, ref, y, x, alpha, beta, T)
    if not cost_norm:
        ng = np.ones_like(ng)
    acc = where.copy()
    evals = 0
    for dy in offsets:
        for dx in offsets:
            if dy == 0 and dx == 0:
                continue
            sy, sx = y + dy, x + dx
            ins = _inside(sy, sx, H, W) & where
            Sr, nr = cost_at(cur, mask, ref, np.clip(sy, 0, H - 1), np.clip(sx, 0, W - 1),
                             alpha - dy, beta - dx, T)
            if not cost_norm:
                nr = np.ones_like(nr)
            red_wins = ins & (Sr * ng <= Sg * nr)
            acc &= ~red_wins
            evals += int(ins.sum())
    return acc, evals


def rmc_accept_at(cur, mask, ref, ys, xs, alpha, beta, offsets, T=4, cost_norm=True):
    """`rmc_accept` at selected pixels only: alpha, beta are the vectors at
    (ys, xs).  Returns bool array of the same shape as ys."""
    H, W = cur.shape
    ys, xs = np.asarray(ys, np.int64), np.asarray(xs, np.int64)
    alpha, beta = np.asarray(alpha, np.int64), np.asarray(beta, np.int64)
    Sg, ng = cost_at(cur, mask, ref, ys, xs, alpha, beta, T)
    if not cost_norm:
        ng = np.ones_like(ng)
    acc = np.ones(ys.shape, bool)
    for dy in offsets:
        for dx in offsets:
            if dy == 0 and dx == 0:
                continue
            sy, sx = ys + dy, xs + dx
            ins = _inside(sy, sx, H, W)
            Sr, nr = cost_at(cur, mask, ref, np.clip(sy, 0, H - 1), np.clip(sx, 0, W - 1),
                             alpha - dy, beta - dx, T)
            if not cost_norm:
                nr = np.ones_like(nr)
            acc &= ~(ins & (Sr * ng <= Sg * nr))
    return acc


def median3x3(a):
    """Component-wise 3x3 median, edge-replicated borders (Eq. (1))."""
    a = np.asarray(a)
    H, W = a.shape
    p = np.pad(a, 1, mode="edge")
    stack = np.stack([p[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)])
    return np.median(stack, axis=0).astype(np.int64)


def nnc_accept(alpha, beta, center="filtered"):
    """Nearest-neighbour check (Sec. 3.1.2).  center="raw" compares the
    unfiltered vector at p with the filtered neighbours."""
    H, W = alpha.shape
    am, bm = median3x3(alpha), median3x3(beta)
    if center == "filtered":
        ca, cb = am, bm
    elif center == "raw":
        ca, cb = np.asarray(alpha, np.int64), np.asarray(beta, np.int64)
    else:
        raise ValueError(center)
    y, x = np.mgrid[0:H, 0:W]
    acc = np.ones((H, W), bool)
    for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ey, ex = y + dy, x + dx
        ins = _inside(ey, ex, H, W)
        eyc, exc = np.clip(ey, 0, H - 1), np.clip(ex, 0, W - 1)
        diff = np.abs(ca - am[eyc, exc]) + np.abs(cb - bm[eyc, exc])
        acc &= ~ins | (diff <= 1)
    return acc


def motion_check(check, cur, mask, ref, alpha, beta, R, T=4, rmc_radius=None, frmc=None,
                 cost_norm=True, nnc_center="filtered"):
    """Accept map of one consistency check on a forward field.

    frmc: per-axis FRMC offsets (None: the paper's set); cost_norm and
    nnc_center as in the module docstring.
    Returns (accept bool (H,W), evaluations): evaluations counts reverse
    cost-function evaluations without early exit (the work measure of
    Sec. 4, Table 3 discussion).
    """
    H, W = cur.shape
    fo = frmc_offsets() if frmc is None else np.asarray(frmc, np.int64)
    if check == "none":
        return np.ones((H, W), bool), 0
    if check == "rme":
        ua, ub, ev = reverse_me(cur, mask, ref, R, T, cost_norm)
        return rme_accept(alpha, beta, ua, ub), ev
    if check == "rmc":
        return rmc_accept(cur, mask, ref, alpha, beta,
                          rmc_offsets(R if rmc_radius is None else rmc_radius), T, cost_norm=cost_norm)
    if check == "frmc":
        return rmc_accept(cur, mask, ref, alpha, beta, fo, T, cost_norm=cost_norm)
    if check == "nnc":
        return nnc_accept(alpha, beta, nnc_center), 0
    if check == "nnc_frmc":
        nn = nnc_accept(alpha, beta, nnc_center)
        acc, ev = rmc_accept(cur, mask, ref, alpha, beta, fo, T, where=nn, cost_norm=cost_norm)
        return acc, ev
    raise ValueError(check)
