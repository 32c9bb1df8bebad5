"""Pins of the oracle's motion estimation (Sec. 2.2) against things other
than itself: a brute-force loop over every pixel/candidate/template position
on tiny frames, the physics of a translated textured scene with the true
previous frame as reference, and quarter-mask counting facts."""
import numpy as np
import pytest

import oracle as O
import synth


def brute_me(cur, mask, ref, R, T):
    """Explicit loops: template offsets, clamp, exclusion, total order."""
    H, W = cur.shape
    lo = -((T - 1) // 2)
    offs = range(lo, lo + T)
    A = np.zeros((H, W), int)
    B = np.zeros((H, W), int)
    SS = np.zeros((H, W), int)
    NN = np.zeros((H, W), int)
    for y in range(H):
        for x in range(W):
            best = None
            n = 0
            for dy in offs:
                for dx in offs:
                    if 0 <= y + dy < H and 0 <= x + dx < W and mask[y + dy, x + dx]:
                        n += 1
            for vy in range(-R, R + 1):
                for vx in range(-R, R + 1):
                    if not (0 <= y + vy < H and 0 <= x + vx < W):
                        continue
                    s = 0
                    for dy in offs:
                        for dx in offs:
                            qy, qx = y + dy, x + dx
                            if 0 <= qy < H and 0 <= qx < W and mask[qy, qx]:
                                ry = min(max(qy + vy, 0), H - 1)
                                rx = min(max(qx + vx, 0), W - 1)
                                s += abs(int(cur[qy, qx]) - int(ref[ry, rx]))
                    key = (s, abs(vy) + abs(vx))
                    if best is None or key < best[0]:   # raster order wins ties
                        best = (key, vy, vx)
            (s, _), vy, vx = best
            A[y, x], B[y, x], SS[y, x], NN[y, x] = vy, vx, s, n
    return A, B, SS, NN


@pytest.mark.parametrize("H,W,R,T,seed", [(10, 12, 2, 4, 0), (12, 10, 3, 4, 1),
                                          (9, 11, 2, 3, 2), (8, 8, 1, 2, 3)])
def test_forward_me_matches_brute_force(H, W, R, T, seed):
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 256, (H, W)).astype(np.uint8)
    # few grey levels so that cost ties (and the tie order) actually occur
    cur = (rng.integers(0, 4, (H, W)) * 60).astype(np.uint8)
    Hm, Wm = H + H % 2, W + W % 2
    mask = synth.fixed_mask(Hm, Wm, rng)[:H, :W]
    ref2 = (rng.integers(0, 4, (H, W)) * 60).astype(np.uint8)
    for r in (ref, ref2):
        a, b, S, n = O.forward_me(cur, mask, r, R, T)
        A, B, SS, NN = brute_me(cur, mask, r, R, T)
        assert (a == A).all() and (b == B).all() and (S == SS).all() and (n == NN).all()
        ys, xs = np.nonzero(np.ones((H, W)))
        pa, pb, pS, pn = O.forward_me_at(cur, mask, r, ys, xs, R, T)
        assert (pa == A.ravel()).all() and (pb == B.ravel()).all()
        assert (pS == SS.ravel()).all() and (pn == NN.ravel()).all()


def test_true_motion_recovered_with_true_reference():
    """Textured scene under global integer translation; with the *true*
    previous frame as the reference every interior pixel finds the true
    vector with zero cost."""
    rng = np.random.default_rng(7)
    frames, offs = synth.video_translate_edges(2, 64, 64, rng, max_step=3)
    d = offs[1] - offs[0]
    mask = synth.fixed_mask(64, 64, rng)
    cur = synth.measured(frames[1], mask)
    a, b, S, n = O.forward_me(cur, mask, frames[0], 4)
    sl = (slice(8, -8), slice(8, -8))
    assert (S[sl] == 0).all()
    assert ((a[sl] == d[0]) & (b[sl] == d[1])).mean() > 0.99


def test_template_counts_under_quarter_masks():
    """Under a quarter mask a 4x4 template with offsets {-1..2} covers a full
    2x2 cell (n >= 1), at most 3x3 cells (n <= 9), and exactly 2x2 cells when
    both coordinates are odd (n == 4 away from the border)."""
    rng = np.random.default_rng(3)
    for kind in ("fixed", "dynamic"):
        m = synth.mask_sequence(kind, 1, 40, 36, rng)[0]
        n = O.n_map(m, 4)
        assert n.min() >= 1 and n.max() <= 9
        assert (n[1:-2:2, 1:-2:2] == 4).all()


def test_unmeasured_values_never_used():
    rng = np.random.default_rng(4)
    frames, _ = synth.video_translate_edges(2, 32, 32, rng)
    mask = synth.fixed_mask(32, 32, rng)
    cur = synth.measured(frames[1], mask)
    garbage = cur.copy()
    garbage[mask == 0] = rng.integers(0, 256, int((mask == 0).sum()))
    r1 = O.forward_me(cur, mask, frames[0], 3)
    r2 = O.forward_me(garbage, mask, frames[0], 3)
    for u, v in zip(r1, r2):
        assert (u == v).all()
