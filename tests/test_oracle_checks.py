"""Pins of the oracle's consistency checks: candidate sets printed in
Sec. 3.1.1, hand-worked NNC examples (Eq. (1), Sec. 3.1.2), brute-force
reverse search on tiny frames, the physics of a translated scene (true
vectors pass, planted wrong vectors fail), and exact relations between the
checks (reverse-cost identity, RMC-accept implies FRMC-accept)."""
import numpy as np
import pytest

import oracle as O
import synth
from _golden import read_grids, read_lines, read_pairs


def test_candidate_sets_match_paper():
    offs = [int(t) for t in read_lines("frmc_offsets.txt")[0].split()]
    assert list(O.frmc_offsets()) == offs
    counts = read_pairs("candidate_counts.txt")
    assert len(O.frmc_offsets()) ** 2 == counts["frmc"]
    assert len(O.rmc_offsets(9)) ** 2 == counts["rmc_radius9"]
    # FRMC's set is a subset of RMC's for R >= 7
    assert set(O.frmc_offsets()) <= set(O.rmc_offsets(7))


@pytest.mark.parametrize("name", ["nnc_outlier.txt", "nnc_l1_sum.txt"])
def test_nnc_hand_worked(name):
    g = read_grids(name)
    assert (O.median3x3(g["alpha"]) == g["median_alpha"]).all()
    acc = O.nnc_accept(g["alpha"], g["beta"])
    assert (acc.astype(int) == g["accept"]).all()


def test_median_is_fifth_of_nine():
    rng = np.random.default_rng(0)
    a = rng.integers(-9, 10, (7, 9))
    m = O.median3x3(a)
    p = np.pad(a, 1, mode="edge")
    for y in range(7):
        for x in range(9):
            assert m[y, x] == sorted(p[y:y + 3, x:x + 3].ravel())[4]


def test_nnc_uniform_and_step():
    a = np.full((6, 7), 3)
    assert O.nnc_accept(a, -a).all()
    step = np.zeros((6, 7), int)
    step[:, 4:] = 2
    acc = O.nnc_accept(step, np.zeros_like(step))
    assert (~acc[:, 3:5]).all() and acc[:, :3].all() and acc[:, 5:].all()


def test_reverse_cost_identity():
    """Reverse matching (template from the reconstruction at q, search over the
    current frame) equals forward cost at (q+u, -u), borders included."""
    rng = np.random.default_rng(1)
    H, W = 14, 18
    cur = rng.integers(0, 256, (H, W)).astype(np.uint8)
    ref = rng.integers(0, 256, (H, W)).astype(np.uint8)
    mask = synth.fixed_mask(H, W, rng)
    qy, qx = np.mgrid[0:H, 0:W]
    for uy in range(-3, 4):
        for ux in range(-3, 4):
            S1, n1 = O.reverse_cost_at(cur, mask, ref, qy, qx, uy, ux)
            S2, n2 = O.cost_at(cur, mask, ref, qy + uy, qx + ux, -uy, -ux)
            ins = (qy + uy >= 0) & (qy + uy < H) & (qx + ux >= 0) & (qx + ux < W)
            assert (S1[ins] == S2[ins]).all() and (n1[ins] == n2[ins]).all()


def brute_reverse(cur, mask, ref, R, norm=True):
    """Explicit loops, exact rational comparison via fractions (raw S
    without `norm`)."""
    from fractions import Fraction
    H, W = cur.shape
    UA = np.zeros((H, W), int)
    UB = np.zeros((H, W), int)
    for y in range(H):
        for x in range(W):
            best = None
            for uy in range(-R, R + 1):
                for ux in range(-R, R + 1):
                    sy, sx = y + uy, x + ux
                    if not (0 <= sy < H and 0 <= sx < W):
                        continue
                    s = n = 0
                    for dy in range(-1, 3):
                        for dx in range(-1, 3):
                            cy, cx = sy + dy, sx + dx
                            if 0 <= cy < H and 0 <= cx < W and mask[cy, cx]:
                                t = ref[min(max(y + dy, 0), H - 1), min(max(x + dx, 0), W - 1)]
                                s += abs(int(cur[cy, cx]) - int(t))
                                n += 1
                    key = (Fraction(s, n) if norm else Fraction(s), abs(uy) + abs(ux))
                    if best is None or key < best[0]:
                        best = (key, uy, ux)
            UA[y, x], UB[y, x] = best[1], best[2]
    return UA, UB


def test_reverse_me_matches_brute_force():
    rng = np.random.default_rng(2)
    H, W = 10, 12
    cur = (rng.integers(0, 4, (H, W)) * 50).astype(np.uint8)
    ref = (rng.integers(0, 4, (H, W)) * 50).astype(np.uint8)
    mask = synth.fixed_mask(H, W, rng)
    ua, ub, _ = O.reverse_me(cur, mask, ref, 2)
    UA, UB = brute_reverse(cur, mask, ref, 2)
    assert (ua == UA).all() and (ub == UB).all()


def brute_rmc(cur, mask, ref, a, b, offsets, norm=True):
    from fractions import Fraction
    H, W = cur.shape

    def S(y, x, vy, vx):
        s = n = 0
        for dy in range(-1, 3):
            for dx in range(-1, 3):
                qy, qx = y + dy, x + dx
                if 0 <= qy < H and 0 <= qx < W and mask[qy, qx]:
                    r = ref[min(max(qy + vy, 0), H - 1), min(max(qx + vx, 0), W - 1)]
                    s += abs(int(cur[qy, qx]) - int(r))
                    n += 1
        return Fraction(s, n) if norm else Fraction(s)

    acc = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            g = S(y, x, a[y, x], b[y, x])
            ok = True
            for dy in offsets:
                for dx in offsets:
                    if (dy, dx) == (0, 0) or not (0 <= y + dy < H and 0 <= x + dx < W):
                        continue
                    if S(y + dy, x + dx, a[y, x] - dy, b[y, x] - dx) <= g:
                        ok = False
            acc[y, x] = ok
    return acc


def test_rmc_frmc_match_brute_force():
    rng = np.random.default_rng(5)
    H, W = 12, 12
    frames, _ = synth.video_translate_edges(2, H, W, rng, max_step=1)
    mask = synth.fixed_mask(H, W, rng)
    cur = synth.measured(frames[1], mask)
    a, b, _, _ = O.forward_me(cur, mask, frames[0], 2)
    a = a.copy()
    a[4, 5] += 1    # a wrong vector somewhere
    for offs in (O.rmc_offsets(2), np.array([-1, 0, 1]), O.frmc_offsets()):
        acc, _ = O.rmc_accept(cur, mask, frames[0], a, b, offs)
        assert (acc == brute_rmc(cur, mask, frames[0], a, b, offs)).all()


@pytest.fixture(scope="module")
def translated():
    rng = np.random.default_rng(11)
    # no edges: an unclipped textured scene, so no flat (ambiguous) areas
    frames, offs = synth.video_translate_edges(2, 48, 48, rng, max_step=3, n_edges=0)
    mask = synth.fixed_mask(48, 48, rng)
    cur = synth.measured(frames[1], mask)
    a, b, S, n = O.forward_me(cur, mask, frames[0], 9)
    return cur, mask, frames[0], a, b, offs[1] - offs[0]


@pytest.mark.parametrize("check", ["rme", "rmc", "frmc", "nnc", "nnc_frmc"])
def test_true_motion_accepted(translated, check):
    cur, mask, ref, a, b, d = translated
    acc, _ = O.motion_check(check, cur, mask, ref, a, b, 9)
    sl = (slice(12, -12), slice(12, -12))
    true = (a == d[0]) & (b == d[1])
    assert true[sl].mean() > 0.95
    assert acc[sl][true[sl]].mean() > 0.98


@pytest.mark.parametrize("check", ["rme", "rmc", "frmc"])
def test_planted_wrong_vector_rejected(translated, check):
    cur, mask, ref, a, b, d = translated
    a2, b2 = a.copy(), b.copy()
    pts = [(20, 20), (23, 27), (27, 22)]
    for y, x in pts:
        a2[y, x] += 3
        b2[y, x] -= 3      # offset (3,-3) lies in the FRMC set
    acc, _ = O.motion_check(check, cur, mask, ref, a2, b2, 9)
    for y, x in pts:
        assert not acc[y, x]


def test_rmc_accept_implies_frmc_accept():
    rng = np.random.default_rng(12)
    frames = synth.video_regions(2, 48, 48, rng, grid=3, vmax=5)
    mask = synth.mask_sequence("dynamic", 2, 48, 48, rng)[1]
    cur = synth.measured(frames[1], mask)
    noisy = np.clip(frames[0].astype(int) + rng.integers(-6, 7, (48, 48)), 0, 255).astype(np.uint8)
    a, b, _, _ = O.forward_me(cur, mask, noisy, 7)
    rmc, _ = O.rmc_accept(cur, mask, noisy, a, b, O.rmc_offsets(7))
    frmc, _ = O.rmc_accept(cur, mask, noisy, a, b, O.frmc_offsets())
    assert not (rmc & ~frmc).any()
    assert rmc.sum() < frmc.sum()     # and the fast check is strictly weaker here


def test_cascade_is_conjunction():
    rng = np.random.default_rng(13)
    frames = synth.video_regions(2, 40, 40, rng, grid=3, vmax=5)
    mask = synth.mask_sequence("dynamic", 2, 40, 40, rng)[1]
    cur = synth.measured(frames[1], mask)
    a, b, _, _ = O.forward_me(cur, mask, frames[0], 6)
    nn, _ = O.motion_check("nnc", cur, mask, frames[0], a, b, 6)
    fr, ev_full = O.motion_check("frmc", cur, mask, frames[0], a, b, 6)
    cas, ev_cas = O.motion_check("nnc_frmc", cur, mask, frames[0], a, b, 6)
    assert (cas == (nn & fr)).all()
    assert ev_cas <= ev_full


def test_rmc_accept_at_equals_full_frame():
    import synth
    rng = np.random.default_rng(12)
    H, W = 24, 28
    frames, _ = synth.video_translate_edges(2, H, W, rng, max_step=2, n_edges=3)
    m = synth.fixed_mask(H, W, rng)
    cur = frames[1] * m
    a, b, S, n = O.forward_me(cur, m, frames[0], 4)
    for offs in (O.frmc_offsets(), O.rmc_offsets(3)):
        full, _ = O.rmc_accept(cur, m, frames[0], a, b, offs)
        ys, xs = np.mgrid[0:H, 0:W]
        at = O.rmc_accept_at(cur, m, frames[0], ys.ravel(), xs.ravel(), a.ravel(), b.ravel(), offs)
        assert np.array_equal(at.reshape(H, W), full)


# ---- options beside the readings: raw costs, raw NNC centre, FRMC offset sets

def test_raw_cost_checks_match_brute_force():
    """cost_norm=False compares raw S: RME and RMC/FRMC against explicit loops
    with exact integer comparison, and the raw reading differs from the
    normalised one on this quarter-sampled frame (n varies from 1 to 9)."""
    rng = np.random.default_rng(6)
    H, W = 12, 12
    frames, _ = synth.video_translate_edges(2, H, W, rng, max_step=1)
    mask = synth.fixed_mask(H, W, rng)
    cur = synth.measured(frames[1], mask)
    ref = np.clip(frames[0].astype(int) + rng.integers(-20, 21, (H, W)), 0, 255).astype(np.uint8)
    ua, ub, _ = O.reverse_me(cur, mask, ref, 2, cost_norm=False)
    UA, UB = brute_reverse(cur, mask, ref, 2, norm=False)
    assert (ua == UA).all() and (ub == UB).all()
    a, b, _, _ = O.forward_me(cur, mask, ref, 2)
    differ = 0
    for offs in (O.rmc_offsets(2), O.frmc_offsets(), np.array([-3, 0, 2])):
        raw, _ = O.rmc_accept(cur, mask, ref, a, b, offs, cost_norm=False)
        assert (raw == brute_rmc(cur, mask, ref, a, b, offs, norm=False)).all()
        nrm, _ = O.rmc_accept(cur, mask, ref, a, b, offs)
        differ += int((raw != nrm).sum())
    assert differ > 0


def test_raw_and_normalised_costs_agree_when_n_is_constant():
    """With every pixel measured, n = 16 at every template inside the frame,
    so comparing S or S/n decides alike for pixels whose candidates all lie
    at least 2 pixels inside the frame."""
    rng = np.random.default_rng(7)
    H, W = 20, 20
    cur = rng.integers(0, 256, (H, W)).astype(np.uint8)
    ref = np.clip(np.roll(cur, 1, axis=1).astype(int) + rng.integers(-30, 31, (H, W)), 0, 255).astype(np.uint8)
    full = np.ones((H, W), np.uint8)
    a, b, _, _ = O.forward_me(cur, full, ref, 2)
    offs = O.rmc_offsets(2)
    raw, _ = O.rmc_accept(cur, full, ref, a, b, offs, cost_norm=False)
    nrm, _ = O.rmc_accept(cur, full, ref, a, b, offs)
    inner = (slice(6, -6), slice(6, -6))
    assert np.array_equal(raw[inner], nrm[inner])


def test_nnc_raw_center_hand_worked():
    g = read_grids("nnc_outlier.txt")
    acc = O.nnc_accept(g["alpha"], g["beta"], center="raw")
    assert (acc.astype(int) == g["accept_raw_center"]).all()
    # the two readings differ exactly at the isolated outlier
    lit = O.nnc_accept(g["alpha"], g["beta"])
    assert list(zip(*np.nonzero(acc != lit))) == [(1, 2)]


def test_nnc_raw_center_uniform_field():
    a = np.full((5, 6), -2)
    assert O.nnc_accept(a, a, center="raw").all()


def test_frmc_offset_set_as_data():
    """An FRMC offset set is data: the set [-r, r] is RMC of radius r (the
    small range of the Fig. 2 caption, read as {-2,-1,0,1,2}), and any set
    follows the brute-force loops; through motion_check the default set is
    the paper's."""
    rng = np.random.default_rng(8)
    H, W = 14, 16
    frames, _ = synth.video_translate_edges(2, H, W, rng, max_step=2)
    mask = synth.fixed_mask(H, W, rng)
    cur = synth.measured(frames[1], mask)
    a, b, _, _ = O.forward_me(cur, mask, frames[0], 3)
    b = b.copy()
    b[6, 7] -= 2
    small, _ = O.motion_check("frmc", cur, mask, frames[0], a, b, 3, frmc=(-2, -1, 0, 1, 2))
    rmc2, _ = O.motion_check("rmc", cur, mask, frames[0], a, b, 3, rmc_radius=2)
    assert np.array_equal(small, rmc2)
    odd = (-5, -2, 0, 4)
    acc, _ = O.motion_check("frmc", cur, mask, frames[0], a, b, 3, frmc=odd)
    assert (acc == brute_rmc(cur, mask, frames[0], a, b, np.array(odd))).all()
    dflt, _ = O.motion_check("frmc", cur, mask, frames[0], a, b, 3)
    paper, _ = O.motion_check("frmc", cur, mask, frames[0], a, b, 3, frmc=(-7, -3, -1, 0, 1, 3, 7))
    assert np.array_equal(dflt, paper)


def test_support_crop_check_matches_whole_frame():
    """The GPU tests' crop-based recomputation of a block support's motion
    inputs (tests/_gpu.check_support_fields) reproduces the whole-frame
    oracle, frame corners included, and catches a single changed decision."""
    from _gpu import check_support_fields
    rng = np.random.default_rng(21)
    H, W, R = 96, 88, 9
    frames = synth.video_regions(2, H, W, rng, grid=3, vmax=6)
    mask = synth.mask_sequence("dynamic", 2, H, W, rng)[1]
    cur = synth.measured(frames[1], mask)
    recon = np.clip(frames[0].astype(int) + rng.integers(-5, 6, (H, W)), 0, 255).astype(np.uint8)
    a, b, S, _ = O.forward_me(cur, mask, recon, R)
    acc, _ = O.motion_check("nnc_frmc", cur, mask, recon, a, b, R)
    blocks = [(0, 0), (H // 4 - 1, W // 4 - 1), (11, 10), (5, 0)]
    assert check_support_fields(cur, mask, recon, a, b, acc, S, blocks, R) > 0
    bad = acc.copy()
    bad[44, 40] = ~bad[44, 40]
    with pytest.raises(AssertionError):
        check_support_fields(cur, mask, recon, a, b, bad, S, [(11, 10)], R)
