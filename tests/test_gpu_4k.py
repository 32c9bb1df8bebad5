"""3840x2160 frames (the 4K configuration: same generator, dynamic mask),
FSR at 100 and 300 iterations and the full recursive frame, checked on
seeded samples the oracle recomputes one by one (maximum supported sizes
are exercised through the same kernels)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import AMB_MAX, FSR_TOL, TAU_FP64, dev, host, need_gpu

pytestmark = pytest.mark.gpu

H, W = 2160, 3840


@pytest.fixture(scope="module")
def seq():
    f, m = synth.workload_c2(n=4, h=H, w=W, seed=synth.seed_for(3))
    return f, m, synth.measured(f, m)


@pytest.mark.parametrize("K", [100, 300])
def test_4k_fsr_sampled_blocks(seq, K):
    R = need_gpu()
    f, m, meas = seq
    vals = meas[0].astype(np.float64)
    out, _ = R.fsr_blocks(dev(vals, torch.float32), dev(m[0]), R.FSRParams(iters=K))
    out = host(out)
    rng = np.random.default_rng(K)
    nb = 192
    blocks = np.stack([rng.integers(0, H // 4, nb), rng.integers(0, W // 4, nb)], axis=1)
    blocks[:4] = [[0, 0], [H // 4 - 1, W // 4 - 1], [0, W // 4 - 1], [H // 4 - 1, 0]]
    ora, gaps = O.fsr.fsr_blocks_out(vals, m[0], blocks, K=K)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    print(f"4K K={K}: max {d[~amb].max():.2e}, ambiguous {amb.sum()}/{nb}")
    assert d[~amb].max() <= FSR_TOL
    assert amb.sum() <= AMB_MAX * nb


def test_4k_recursive_frame_sampled(seq):
    """Frame 3 with three references (teacher-forced: ground-truth frames as
    reconstructions), NNC -> FRMC: forward vectors and costs at sampled
    pixels bit-exact; the FSR input classes at sampled blocks follow from the
    oracle's own projection of those vectors; outputs within tolerance."""
    R = need_gpu()
    f, m, meas = seq
    refs = [(f[3 - k], meas[3 - k], m[3 - k]) for k in (1, 2, 3)]
    out, out_u8 = R.reconstruct_frame(dev(meas[3]), dev(m[3]), [(dev(a), dev(b), dev(c)) for a, b, c in refs],
                                      R.MEParams(search=9, check="nnc_frmc"), R.FSRParams(iters=100))
    out = host(out)
    # forward ME at sampled pixels against each reference
    rng = np.random.default_rng(11)
    ys = np.concatenate([[0, H - 1, 0, H - 1], rng.integers(0, H, 120)])
    xs = np.concatenate([[0, W - 1, W - 1, 0], rng.integers(0, W, 120)])
    for recon, _, _ in refs:
        mv, _, cost = R.motion_check(dev(meas[3]), dev(m[3]), dev(recon), R.MEParams(search=9, check="none"))
        mv, cost = host(mv), host(cost).astype(np.int64) & 0xFFFF
        a, b, S, n = O.forward_me_at(meas[3], m[3], recon, ys, xs, 9)
        assert (mv[0][ys, xs] == a).all() and (mv[1][ys, xs] == b).all() and (cost[ys, xs] == S).all()
    # measured pixels are returned bit-exactly; everything is finite and in a sane range
    assert (out[m[3] == 1] == meas[3][m[3] == 1]).all()
    assert np.isfinite(out).all()
    assert O.psnr(f[3], out) > 25.0
    assert (host(out_u8) == O.quantize(out)).all()
