"""Edge cases on the GPU: the maximum supported frame dimension (16384) as
thin strips, the smallest frames, frames whose height or width is a single
FSR block row/column, and an all-unknown frame."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import FLOAT64_FORMS, FSR_TOL, TAU_FP64, dev, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W", [(16, 16384), (16384, 12), (4, 4), (4, 64), (64, 4)])
@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_fsr_extreme_shapes_sampled(H, W, precision):
    R = need_gpu()
    rng = np.random.default_rng(H + W)
    f = np.clip(128 + 40 * synth.bandlimited_noise(H, W, 2.0, rng), 0, 255).astype(np.uint8)
    m = synth.fixed_mask(H, W, rng)
    vals = (f * m).astype(np.float64)
    out, _ = R.fsr_blocks(dev(vals, torch.float32), dev(m), R.FSRParams(iters=40, precision=precision))
    out = host(out)
    nbh, nbw = H // 4, W // 4
    idx = rng.choice(nbh * nbw, size=min(64, nbh * nbw), replace=False)
    blocks = np.stack([idx // nbw, idx % nbw], axis=1)
    blocks[0] = [0, 0]
    blocks[-1] = [nbh - 1, nbw - 1]
    ora, gaps = O.fsr.fsr_blocks_out(vals, m, blocks, K=40)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    assert np.isfinite(out).all()
    if (~amb).any():      # a frame of one block may hold only a near tie
        print(f"{H}x{W} {precision}: max {d[~amb].max():.2e} over {(~amb).sum()} blocks")
        assert d[~amb].max() <= FSR_TOL


@pytest.mark.parametrize("H,W", [(16, 16384), (16384, 16)])
def test_motion_extreme_shapes_sampled(H, W):
    """Forward ME and the FRMC decision at sampled pixels of a maximum-length
    strip, bit-exact against the oracle."""
    R = need_gpu()
    rng = np.random.default_rng(7 + H)
    frames, _ = synth.video_translate_edges(2, H, W, rng, max_step=2, n_edges=4)
    m = synth.fixed_mask(H, W, rng)
    cur = synth.measured(frames[1:], m[None])[0]
    ref = frames[0]
    mv, acc, cost = R.motion_check(dev(cur), dev(m), dev(ref), R.MEParams(search=5, check="none"))
    mv, cost = host(mv), host(cost).astype(np.int64) & 0xFFFF
    ys = np.concatenate([[0, H - 1], rng.integers(0, H, 100)])
    xs = np.concatenate([[0, W - 1], rng.integers(0, W, 100)])
    a, b, S, n = O.forward_me_at(cur, m, ref, ys, xs, 5)
    assert (mv[0][ys, xs] == a).all() and (mv[1][ys, xs] == b).all() and (cost[ys, xs] == S).all()


def test_all_unknown_frame_reconstructs_zero():
    R = need_gpu()
    H, W = 32, 48
    vals = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    cls = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    out, u8 = R.fsr_blocks(vals, cls, R.FSRParams(iters=20))
    assert (host(out) == 0).all() and (host(u8) == 0).all()


def test_rejects_unsupported_shapes():
    R = need_gpu()
    x = torch.zeros((6, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RfsrError):
        R.fsr_blocks(x.float(), x)
    y = torch.zeros((8, 16388), dtype=torch.uint8, device="cuda")
    with pytest.raises(R.RfsrError):
        R.fsr_blocks(y.float(), y)
