"""Parity on the two workload configurations that the CPU and the GPU both
finish: the CPU-sized 128x128 recursion (fixed mask, R = 8, RME and RMC
each), end to end against the oracle, and the 1920x1080 recursive frame in
the configuration bench.py times (dynamic mask, R = 9, NNC -> FRMC, K = 100,
three references that are the GPU's own reconstructions, consecutive frames
pipelined), on sampled pixels and blocks the oracle recomputes one by one
from the same inputs."""
import numpy as np
import pytest

import oracle as O
import synth
from _gpu import (AMB_MAX, FLOAT64_FORMS, FSR_TOL, PSNR_TOL, TAU_FP64, check_support_fields, compare_fsr, dev, host,
                  need_gpu)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("check", ["rme", "rmc"])
@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_cpu_sized_recursion(check, precision):
    """128x128, 4 frames, fixed mask, R = 8: every frame's motion fields and
    decisions bit-exact (both sides fed the same uint8 reconstructions), FSR
    within tolerance, and the free-running PSNR of each frame within 0.01 dB."""
    R = need_gpu()
    frames, masks = synth.workload_c1()
    meas = synth.measured(frames, masks)
    me_o, fsr_o = O.MEParams(search=8, check=check), O.FSRParams(iters=100)
    me_g, fsr_g = R.MEParams(search=8, check=check), R.FSRParams(iters=100, precision=precision)
    ora = O.reconstruct_sequence(meas, masks, me_o, fsr_o, track_gaps=True)
    seq = R.Sequence(128, 128, me_g, fsr_g)
    for t in range(4):
        # the GPU's own references for frame t (lags 1..3), taken before the push
        refs = [(host(r[0]).copy(), meas[t - 1 - k], masks[t - 1 - k])
                for k, r in enumerate(reversed(seq.ring[-3:]))]
        out, u8 = seq.push(dev(meas[t]), dev(masks[t]))
        out = host(out)
        # teacher-forced step: the oracle from those references
        tf = O.reconstruct_frame(meas[t], masks[t], refs, me_o, fsr_o)
        for k, (recon, _, _) in enumerate(refs):
            mv, acc, cost = R.motion_check(dev(meas[t]), dev(masks[t]), dev(recon), me_g)
            f = tf["fields"][k]
            assert np.array_equal(host(mv)[0], f["alpha"]) and np.array_equal(host(mv)[1], f["beta"])
            assert np.array_equal(host(acc).astype(bool), f["accept"]), (t, k)
        worst, namb, nb = compare_fsr(out, tf["out"], tf["gaps"])
        print(f"{check} {precision} t={t}: max {worst:.2e}, ambiguous {namb}/{nb}, "
              f"PSNR gpu {O.psnr(frames[t], out):.4f} oracle {O.psnr(frames[t], ora[t]['out']):.4f}")
        assert worst <= FSR_TOL
        assert abs(O.psnr(frames[t], out) - O.psnr(frames[t], ora[t]["out"])) <= PSNR_TOL


@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_1080p_recursive_frame_sampled(precision):
    R = need_gpu()
    H, W = 1080, 1920
    frames, masks = synth.workload_c2(n=4, h=H, w=W)
    meas = synth.measured(frames, masks)
    me_g, fsr_g = R.MEParams(search=9, check="nnc_frmc"), R.FSRParams(iters=100, precision=precision)
    seq = R.Sequence(H, W, me_g, fsr_g, pipelined=True)   # as bench.py runs it
    for t in range(3):
        seq.push(dev(meas[t]), dev(masks[t]))
    refs = [(host(r[0]).copy(), meas[2 - k], masks[2 - k]) for k, r in enumerate(reversed(seq.ring[-3:]))]
    out, _ = seq.push(dev(meas[3]), dev(masks[3]))
    out = host(out)
    cur, mask = meas[3], masks[3]
    rng = np.random.default_rng(1080)
    ys = np.concatenate([[0, H - 1, 0, H - 1, 540], rng.integers(0, H, 150)])
    xs = np.concatenate([[0, W - 1, W - 1, 0, 960], rng.integers(0, W, 150)])
    fields = []
    for recon, rmeas, rmask in refs:
        mv, _, cost = R.motion_check(dev(cur), dev(mask), dev(recon), R.MEParams(search=9, check="none"))
        _, acc, _ = R.motion_check(dev(cur), dev(mask), dev(recon), me_g)
        a, b = host(mv)[0].astype(np.int64), host(mv)[1].astype(np.int64)
        acc = host(acc).astype(bool)
        cost = host(cost).astype(np.int64) & 0xFFFF
        # forward ME at sampled pixels: bit-exact
        oa, ob, oS, _ = O.forward_me_at(cur, mask, recon, ys, xs, 9)
        assert (a[ys, xs] == oa).all() and (b[ys, xs] == ob).all() and (cost[ys, xs] == oS).all()
        # NNC on the (verified) field, FRMC where it accepts: decisions bit-exact at the samples
        nn = O.nnc_accept(a, b)[ys, xs]
        fr = O.rmc_accept_at(cur, mask, recon, ys, xs, a[ys, xs], b[ys, xs], O.frmc_offsets())
        assert np.array_equal(acc[ys, xs], nn & fr)
        fields.append(dict(alpha=a, beta=b, accept=acc, meas=rmeas, mask=rmask))
    # projection from the verified fields and decisions, then FSR at sampled blocks
    values, cls = O.project(cur, mask, fields)
    blocks = np.stack([rng.integers(0, H // 4, 96), rng.integers(0, W // 4, 96)], axis=1)
    blocks[:2] = [[0, W // 4 - 1], [H // 8, W // 8]]
    # the first 8 blocks: every motion input of their supports recomputed by
    # the oracle (vectors and costs on the support grown by 2, NNC -> FRMC
    # decisions on the support, all three references), so their FSR input
    # is oracle-derived end to end
    for f, (recon, _, _) in zip(fields, refs):
        _, _, cost = R.motion_check(dev(cur), dev(mask), dev(recon), R.MEParams(search=9, check="none"))
        n = check_support_fields(cur, mask, recon, f["alpha"], f["beta"], f["accept"],
                                 host(cost).astype(np.int64) & 0xFFFF, blocks[:8], 9)
        assert n >= 8 * 32 * 24
    ora, gaps = O.fsr.fsr_blocks_out(values, cls, blocks, K=100)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    print(f"1080p frame 3 ({precision}): FSR max {d[~amb].max():.2e} over {(~amb).sum()} blocks "
          f"(8 end to end: max {d[:8].max():.2e}), projected {(cls == 2).mean():.3f} of pixels")
    assert d[~amb].max() <= FSR_TOL
    assert amb.sum() <= AMB_MAX * len(blocks)
