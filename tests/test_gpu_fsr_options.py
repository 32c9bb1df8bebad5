"""GPU parity of the FSR-literature options (frequency-weighting prior,
residual-energy early stop), each alone and together, against the oracle's
forms of the same loop: whole frames (blockwise under the near-tie rule,
which for the stop also covers decisions within rounding of the threshold),
the recursive frame path, and sampled blocks of a 1920x1080 frame.  A stop
ratio that is never reached reproduces the default kernel bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import FSR_TOL, PSNR_TOL, AMB_MAX, TAU_FP64, compare_fsr, dev, host, need_gpu

pytestmark = pytest.mark.gpu

OPTIONS = [(0.85, 0.0), (0.0, 1e-3), (0.85, 1e-3), (0.6, 1e-2)]


def frame(seed, H, W):
    f, m = synth.workload_c2(n=1, h=H, w=W, seed=seed)
    return f[0], m[0], synth.measured(f, m)[0]


@pytest.mark.parametrize("sigma,ratio", OPTIONS)
def test_fsr_options_frame_parity(sigma, ratio):
    R = need_gpu()
    f, m, meas = frame(31, 132, 100)
    vals = meas.astype(np.float64)
    ora, gaps = O.fsr_frame(vals, m, K=100, prior_sigma=sigma, stop_ratio=ratio)
    out, u8 = R.fsr_blocks(dev(vals, torch.float32), dev(m),
                           R.FSRParams(iters=100, prior_sigma=sigma, stop_ratio=ratio))
    out = host(out)
    worst, namb, nb = compare_fsr(out, ora, gaps)
    print(f"sigma={sigma} ratio={ratio}: max {worst:.2e}, ambiguous {namb}/{nb}, "
          f"PSNR {O.psnr(f, out, 8):.3f} (oracle {O.psnr(f, ora, 8):.3f})")
    assert worst <= FSR_TOL
    assert namb <= AMB_MAX * nb
    assert abs(O.psnr(f, out, 8) - O.psnr(f, ora, 8)) <= PSNR_TOL
    assert (host(u8) == O.quantize(out)).all()


def test_fsr_options_change_the_result_and_unreached_stop_is_default():
    R = need_gpu()
    f, m, meas = frame(32, 64, 80)
    v, c = dev(meas, torch.float32), dev(m)
    base = host(R.fsr_blocks(v, c, R.FSRParams(iters=60))[0])
    never = host(R.fsr_blocks(v, c, R.FSRParams(iters=60, stop_ratio=1e-300))[0])
    assert np.array_equal(base, never)
    prior = host(R.fsr_blocks(v, c, R.FSRParams(iters=60, prior_sigma=0.8))[0])
    stop = host(R.fsr_blocks(v, c, R.FSRParams(iters=60, stop_ratio=0.05))[0])
    assert not np.array_equal(base, prior) and not np.array_equal(base, stop)


def test_fsr_options_in_the_frame_path():
    """rfsr_reconstruct_frame with both options against the oracle's frame
    (same uint8 references on both sides; three references)."""
    R = need_gpu()
    rng = np.random.default_rng(33)
    H, W = 64, 80
    frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=3, n_edges=3)
    masks = synth.mask_sequence("dynamic", 4, H, W, rng)
    meas = synth.measured(frames, masks)
    refs = [(frames[2 - k], meas[2 - k], masks[2 - k]) for k in range(3)]
    ora = O.reconstruct_frame(meas[3], masks[3], refs, O.MEParams(search=8),
                              O.FSRParams(iters=80, prior_sigma=0.85, stop_ratio=1e-3))
    out, _ = R.reconstruct_frame(dev(meas[3]), dev(masks[3]), [tuple(dev(x) for x in r) for r in refs],
                                 R.MEParams(search=8), R.FSRParams(iters=80, prior_sigma=0.85, stop_ratio=1e-3))
    worst, namb, nb = compare_fsr(host(out), ora["out"], ora["gaps"])
    print(f"frame path with prior + stop: max {worst:.2e}, ambiguous {namb}/{nb}")
    assert worst <= FSR_TOL and namb <= AMB_MAX * nb


def test_fsr_options_1080p_sampled_blocks():
    R = need_gpu()
    f, m, meas = frame(34, 1080, 1920)
    vals = meas.astype(np.float64)
    rng = np.random.default_rng(1081)
    blocks = np.stack([rng.integers(0, 270, 128), rng.integers(0, 480, 128)], axis=1)
    ora, gaps = O.fsr.fsr_blocks_out(vals, m, blocks, K=100, prior_sigma=0.85, stop_ratio=1e-3)
    out, _ = R.fsr_blocks(dev(vals, torch.float32), dev(m), R.FSRParams(iters=100, prior_sigma=0.85,
                                                                          stop_ratio=1e-3))
    out = host(out)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    print(f"1080p prior + stop: max {d[~amb].max():.2e} over {(~amb).sum()} blocks")
    assert d[~amb].max() <= FSR_TOL


def test_fsr_options_in_a_batch_equal_single_frames():
    """A batch of frames of different sizes with both options gives the
    single-frame results bit for bit."""
    R = need_gpu()
    me, fsr = R.MEParams(search=6), R.FSRParams(iters=60, prior_sigma=0.9, stop_ratio=1e-4)
    frames = []
    for i, (H, W, nref) in enumerate([(64, 80, 3), (48, 64, 1), (32, 96, 0)]):
        rng = np.random.default_rng(700 + i)
        f, _ = synth.video_translate_edges(nref + 1, H, W, rng, max_step=2, n_edges=2)
        m = synth.mask_sequence("dynamic", nref + 1, H, W, rng)
        meas = synth.measured(f, m)
        refs = tuple((dev(f[nref - 1 - k]), dev(meas[nref - 1 - k]), dev(m[nref - 1 - k])) for k in range(nref))
        frames.append((dev(meas[nref]), dev(m[nref]), refs))
    single = [tuple(host(x) for x in R.reconstruct_frame(c, mk, refs, me, fsr)) for c, mk, refs in frames]
    b = R.Batch([R.BatchFrame(c, mk, refs, out_u8=torch.empty_like(c)) for c, mk, refs in frames], me, fsr)
    got = [(host(o), host(u)) for o, u in b.run()]
    for (o1, u1), (o2, u2) in zip(single, got):
        assert np.array_equal(o1, o2) and np.array_equal(u1, u2)
