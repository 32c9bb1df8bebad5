"""GPU parity of rfsr_motion_check (forward ME, Sec. 2.2; RME, Sec. 2.2;
RMC/FRMC, Sec. 3.1.1; NNC and the NNC->FRMC cascade, Sec. 3.1.2): motion
vectors, costs and check decisions bit-exact against the integer oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import dev, host, need_gpu

pytestmark = pytest.mark.gpu


def c1_pair(seed=None):
    frames, masks = synth.workload_c1(seed=seed)
    meas = synth.measured(frames, masks)
    return meas[1], masks[1], frames[0]


def gpu_me(R, cur, mask, ref, search, check="none", rmc_radius=0):
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    mv, acc, cost = R.motion_check(dev(cur), dev(mask), dev(ref),
                                   R.MEParams(search=search, check=check, rmc_radius=rmc_radius),
                                   counters=cnt)
    return host(mv).astype(np.int64), host(acc).astype(bool), host(cost).astype(np.int64) & 0xFFFF, host(cnt)


@pytest.mark.parametrize("search", [8, 9, 3, 0, 15])
def test_forward_me_bit_exact(search):
    R = need_gpu()
    cur, mask, ref = c1_pair()
    mv, _, cost, cnt = gpu_me(R, cur, mask, ref, search)
    a, b, S, n = O.forward_me(cur, mask, ref, search)
    assert (mv[0] == a).all() and (mv[1] == b).all() and (cost == S).all()
    H, W = cur.shape
    y, x = np.mgrid[0:H, 0:W]
    ny = np.minimum(search, y) + np.minimum(search, H - 1 - y) + 1
    nx = np.minimum(search, x) + np.minimum(search, W - 1 - x) + 1
    assert cnt[0] == (ny * nx).sum()


def test_forward_me_ragged_and_zero_values():
    """Ragged frame (not a multiple of the 16x16 tile), many measured zeros
    (exercises the masked-SAD correction) and saturated 255s."""
    R = need_gpu()
    rng = np.random.default_rng(3)
    H, W = 52, 76
    f = rng.integers(0, 256, (3, H, W))
    f[:, :20, :30] = 0
    f[:, 30:, 50:] = 255
    f = f.astype(np.uint8)
    m = synth.mask_sequence("dynamic", 2, H, W, rng)
    cur = synth.measured(f[1], m[1])
    for search in (9, 4):
        mv, _, cost, _ = gpu_me(R, cur, m[1], f[0], search)
        a, b, S, n = O.forward_me(cur, m[1], f[0], search)
        assert (mv[0] == a).all() and (mv[1] == b).all() and (cost == S).all()


@pytest.mark.parametrize("check", ["rme", "rmc", "frmc", "nnc", "nnc_frmc"])
def test_checks_bit_exact(check):
    R = need_gpu()
    cur, mask, ref = c1_pair()
    noisy = np.clip(ref.astype(int) + np.random.default_rng(0).integers(-8, 9, ref.shape), 0, 255).astype(np.uint8)
    for r in (ref, noisy):
        mv, acc, _, cnt = gpu_me(R, cur, mask, r, 8, check)
        a, b, S, n = O.forward_me(cur, mask, r, 8)
        oacc, oev = O.motion_check(check, cur, mask, r, a, b, 8)
        print(f"{check}: accept {acc.mean():.3f}, gpu check costs {cnt[1]}, oracle (no early exit) {oev}")
        assert (acc == oacc).all()
        assert cnt[3] == oacc.sum()
        if check == "rme":
            assert cnt[1] == oev
        else:
            assert cnt[1] <= oev


def test_rmc_radius_and_fig2_small_ranges():
    R = need_gpu()
    cur, mask, ref = c1_pair()
    for rr in (2, 5):
        mv, acc, _, _ = gpu_me(R, cur, mask, ref, 8, "rmc", rmc_radius=rr)
        a, b, S, n = O.forward_me(cur, mask, ref, 8)
        oacc, _ = O.rmc_accept(cur, mask, ref, a, b, O.rmc_offsets(rr))
        assert (acc == oacc).all()


def test_full_hd_sampled_pixels():
    R = need_gpu()
    H, W = 1080, 1920
    f, m = synth.workload_c2(n=2, h=H, w=W)
    cur = synth.measured(f[1], m[1])
    mv, acc, cost, _ = gpu_me(R, cur, m[1], f[0], 9, "nnc_frmc")
    rng = np.random.default_rng(1)
    ys = np.concatenate([[0, H - 1, 0, H - 1], rng.integers(0, H, 300)])
    xs = np.concatenate([[0, W - 1, W - 1, 0], rng.integers(0, W, 300)])
    a, b, S, n = O.forward_me_at(cur, m[1], f[0], ys, xs, 9)
    assert (mv[0][ys, xs] == a).all() and (mv[1][ys, xs] == b).all() and (cost[ys, xs] == S).all()
    # FRMC decisions at sampled pixels, given the GPU's (verified) field
    Sg, ng = O.cost_at(cur, m[1], f[0], ys, xs, a, b)
    acc_o = np.ones(len(ys), bool)
    for dy in O.frmc_offsets():
        for dx in O.frmc_offsets():
            if dy == 0 and dx == 0:
                continue
            sy, sx = ys + dy, xs + dx
            ins = (sy >= 0) & (sy < H) & (sx >= 0) & (sx < W)
            Sr, nr = O.cost_at(cur, m[1], f[0], np.clip(sy, 0, H - 1), np.clip(sx, 0, W - 1), a - dy, b - dx)
            acc_o &= ~(ins & (Sr * ng <= Sg * nr))
    nnc_o = O.nnc_accept(mv[0], mv[1])[ys, xs]
    assert (acc[ys, xs] == (acc_o & nnc_o)).all()
