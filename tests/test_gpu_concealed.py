"""GPU FSR with non-zero concealed weighting (wavefront over raster order)
against the oracle's sequential form.  Teacher-forced: the oracle takes the
GPU's reconstructions of earlier blocks as the concealed values, so every
block is checked on the same inputs; free-running: frame PSNR."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import FSR_TOL, PSNR_TOL, TAU_FP64, dev, host, need_gpu

pytestmark = pytest.mark.gpu


def case(H, W, seed, proj_frac=0.2):
    rng = np.random.default_rng(seed)
    f, _ = synth.video_translate_edges(1, H, W, rng, n_edges=3)
    m = synth.fixed_mask(H, W, rng)
    cls = m.astype(np.uint8)
    cls[(m == 0) & (rng.random((H, W)) < proj_frac)] = 2
    vals = np.where(cls > 0, f[0].astype(np.float64) + (cls == 2) * rng.normal(0, 2, (H, W)), 0.0)
    return f[0], vals.astype(np.float32).astype(np.float64), cls


@pytest.mark.parametrize("H,W,delta,K,overwrite", [(64, 80, 0.5, 40, "dfsr"), (48, 36, 1.0, 30, "rfsr"),
                                                   (32, 128, 0.25, 60, "dfsr")])
def test_concealed_fsr_teacher_forced(H, W, delta, K, overwrite):
    R = need_gpu()
    f, vals, cls = case(H, W, H + W)
    prm = R.FSRParams(iters=K, concealed_weight=delta, overwrite=overwrite)
    out, u8 = R.fsr_blocks(dev(vals, torch.float32), dev(cls), prm)
    out = host(out)
    ora, gaps = O.fsr_frame_concealed(vals, cls, delta, K=K, overwrite=overwrite, given=out)
    d = np.abs(out - ora).reshape(H // 4, 4, W // 4, 4).max(axis=(1, 3))
    amb = gaps < TAU_FP64
    print(f"{H}x{W} delta={delta} K={K}: max {d[~amb].max():.2e}, ambiguous {amb.sum()}/{amb.size}")
    assert d[~amb].max() <= FSR_TOL
    assert (host(u8) == O.quantize(out)).all()
    # free-running: the oracle's own sequential recursion
    ora_free, _ = O.fsr_frame_concealed(vals, cls, delta, K=K, overwrite=overwrite)
    assert abs(O.psnr(f, out, 4) - O.psnr(f, ora_free, 4)) <= PSNR_TOL


def test_concealed_changes_the_result_and_first_block_does_not():
    R = need_gpu()
    f, vals, cls = case(32, 32, 3)
    v_d, c_d = dev(vals, torch.float32), dev(cls)
    a = host(R.fsr_blocks(v_d, c_d, R.FSRParams(iters=30))[0])
    b = host(R.fsr_blocks(v_d, c_d, R.FSRParams(iters=30, concealed_weight=0.5))[0])
    assert np.array_equal(a[:4, :4], b[:4, :4])
    assert not np.array_equal(a, b)


def test_concealed_recursive_frame_against_oracle():
    R = need_gpu()
    rng = np.random.default_rng(9)
    H, W = 48, 64
    frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=2, n_edges=3)
    masks = synth.mask_sequence("dynamic", 4, H, W, rng)
    meas = synth.measured(frames, masks)
    refs = [(frames[3 - k], meas[3 - k], masks[3 - k]) for k in (1, 2, 3)]
    me = O.MEParams(search=6, check="nnc_frmc")
    fsr = O.FSRParams(iters=40, concealed_weight=0.5)
    ora = O.reconstruct_frame(meas[3], masks[3], refs, me, fsr)
    out, _ = R.reconstruct_frame(dev(meas[3]), dev(masks[3]), [(dev(a), dev(b), dev(c)) for a, b, c in refs],
                                 R.MEParams(search=6, check="nnc_frmc"),
                                 R.FSRParams(iters=40, concealed_weight=0.5))
    out = host(out)
    dp = O.psnr(frames[3], out, 4) - O.psnr(frames[3], ora["out"], 4)
    print(f"recursive frame delta=0.5: PSNR delta {dp:+.5f} dB")
    assert abs(dp) <= PSNR_TOL


def test_batch_concealed_equals_single_frames():
    """The batch runs every frame's wavefront in shared steps: each frame's
    result equals the single-frame wavefront, bit for bit."""
    R = need_gpu()
    me, fsr = R.MEParams(search=5, check="nnc_frmc"), R.FSRParams(iters=30, concealed_weight=0.5)
    sizes = [(64, 64, 3), (32, 96, 1), (96, 32, 0), (16, 24, 2), (48, 48, 3)]
    streams = []
    for i, (H, W, nref) in enumerate(sizes):
        rng = np.random.default_rng(700 + i)
        frames, _ = synth.video_translate_edges(nref + 1, H, W, rng, max_step=2, n_edges=2)
        masks = synth.mask_sequence("dynamic", nref + 1, H, W, rng)
        meas = synth.measured(frames, masks)
        refs = [(dev(frames[nref - 1 - k]), dev(meas[nref - 1 - k]), dev(masks[nref - 1 - k])) for k in range(nref)]
        streams.append((dev(meas[nref]), dev(masks[nref]), refs))
    singles = [tuple(host(t).copy() for t in R.reconstruct_frame(c, m, r, me, fsr)) for c, m, r in streams]
    frames = [R.BatchFrame(c, m, tuple(r), out_u8=torch.empty_like(c)) for c, m, r in streams]
    outs = R.Batch(frames, me, fsr).run()
    for i, ((o, u), (so, su)) in enumerate(zip(outs, singles)):
        assert np.array_equal(host(o), so), i
        assert np.array_equal(host(u), su), i
