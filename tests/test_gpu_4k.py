"""3840x2160 frames (the 4K configuration: same generator, dynamic mask),
FSR at 100 and 300 iterations and the full recursive frame, checked on
seeded samples the oracle recomputes one by one (maximum supported sizes
are exercised through the same kernels)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import AMB_MAX, FLOAT64_FORMS, FSR_TOL, TAU_FP64, check_support_fields, dev, host, need_gpu

pytestmark = pytest.mark.gpu

H, W = 2160, 3840


@pytest.fixture(scope="module")
def seq():
    f, m = synth.workload_c2(n=4, h=H, w=W, seed=synth.seed_for(3))
    return f, m, synth.measured(f, m)


@pytest.mark.parametrize("K", [100, 300])
@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_4k_fsr_sampled_blocks(seq, K, precision):
    R = need_gpu()
    f, m, meas = seq
    vals = meas[0].astype(np.float64)
    out, _ = R.fsr_blocks(dev(vals, torch.float32), dev(m[0]), R.FSRParams(iters=K, precision=precision))
    out = host(out)
    rng = np.random.default_rng(K)
    nb = 192
    blocks = np.stack([rng.integers(0, H // 4, nb), rng.integers(0, W // 4, nb)], axis=1)
    blocks[:4] = [[0, 0], [H // 4 - 1, W // 4 - 1], [0, W // 4 - 1], [H // 4 - 1, 0]]
    ora, gaps = O.fsr.fsr_blocks_out(vals, m[0], blocks, K=K)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    print(f"4K {precision} K={K}: max {d[~amb].max():.2e}, ambiguous {amb.sum()}/{nb}")
    assert d[~amb].max() <= FSR_TOL
    assert amb.sum() <= AMB_MAX * nb


@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_4k_recursive_frame_sampled(seq, precision):
    """Frame 3 with three references (teacher-forced: ground-truth frames as
    reconstructions), NNC -> FRMC: forward vectors and costs at sampled
    pixels bit-exact, NNC -> FRMC decisions at the sampled pixels bit-exact,
    every motion input of 8 sampled blocks' supports recomputed by the
    oracle, and FSR at 96 sampled blocks (those 8 included) against the
    oracle's projection of the verified fields."""
    R = need_gpu()
    f, m, meas = seq
    refs = [(f[3 - k], meas[3 - k], m[3 - k]) for k in (1, 2, 3)]
    me_g = R.MEParams(search=9, check="nnc_frmc")
    out, out_u8 = R.reconstruct_frame(dev(meas[3]), dev(m[3]), [(dev(a), dev(b), dev(c)) for a, b, c in refs],
                                      me_g, R.FSRParams(iters=100, precision=precision))
    out = host(out)
    cur, mask = meas[3], m[3]
    rng = np.random.default_rng(11)
    ys = np.concatenate([[0, H - 1, 0, H - 1], rng.integers(0, H, 120)])
    xs = np.concatenate([[0, W - 1, W - 1, 0], rng.integers(0, W, 120)])
    blocks = np.stack([rng.integers(0, H // 4, 96), rng.integers(0, W // 4, 96)], axis=1)
    blocks[:2] = [[H // 4 - 1, 0], [H // 8, W // 8]]
    fields = []
    for recon, rmeas, rmask in refs:
        mv, _, cost = R.motion_check(dev(cur), dev(mask), dev(recon), R.MEParams(search=9, check="none"))
        _, acc, _ = R.motion_check(dev(cur), dev(mask), dev(recon), me_g)
        a, b = host(mv)[0].astype(np.int64), host(mv)[1].astype(np.int64)
        acc = host(acc).astype(bool)
        cost = host(cost).astype(np.int64) & 0xFFFF
        oa, ob, oS, _ = O.forward_me_at(cur, mask, recon, ys, xs, 9)
        assert (a[ys, xs] == oa).all() and (b[ys, xs] == ob).all() and (cost[ys, xs] == oS).all()
        nn = O.nnc_accept(a, b)[ys, xs]
        fr = O.rmc_accept_at(cur, mask, recon, ys, xs, a[ys, xs], b[ys, xs], O.frmc_offsets())
        assert np.array_equal(acc[ys, xs], nn & fr)
        check_support_fields(cur, mask, recon, a, b, acc, cost, blocks[:8], 9)
        fields.append(dict(alpha=a, beta=b, accept=acc, meas=rmeas, mask=rmask))
    values, cls = O.project(cur, mask, fields)
    ora, gaps = O.fsr.fsr_blocks_out(values, cls, blocks, K=100)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    print(f"4K frame 3 ({precision}): FSR max {d[~amb].max():.2e} over {(~amb).sum()} blocks, "
          f"projected {(cls == 2).mean():.3f} of pixels")
    assert d[~amb].max() <= FSR_TOL
    assert amb.sum() <= AMB_MAX * len(blocks)
    # measured pixels are returned bit-exactly, the uint8 plane is the quantised output
    assert (out[mask == 1] == cur[mask == 1]).all()
    assert np.isfinite(out).all()
    assert (host(out_u8) == O.quantize(out)).all()
