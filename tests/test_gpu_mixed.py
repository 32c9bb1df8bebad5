"""The mixed-precision FSR (RFSR_PREC_MIXED: the float32 form with a near-tie
test, float64 for the blocks that fail it) held to the float64 form's bar:
parity with the float64 oracle at the float64 near-tie threshold, every
block of full 1080p and 4K frames within 1e-3 of the float64 kernel (which
is within ~2e-5 of the oracle), the recursive frame path teacher-forced,
results of a batch and of pipelined steps identical to single frames, edge
cases; and the bound itself calibrated with the margin diagnostic of the
plain float32 form on the 1080p workload."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import AMB_MAX, FSR_TOL, PSNR_TOL, compare_fsr, dev, host, need_gpu
from test_gpu_frame import teacher_forced_case

pytestmark = pytest.mark.gpu


def run(R, vals, cls, K=100, precision="mixed", counter=None, margins=None, **kw):
    prm = R.FSRParams(iters=K, precision=precision, rerun_blocks=counter, block_margin=margins, **kw)
    out, u8 = R.fsr_blocks(dev(vals, torch.float32), dev(cls), prm)
    return host(out), host(u8)


def frame(seed, H, W, kind="dynamic"):
    if kind == "dynamic":
        f, m = synth.workload_c2(n=1, h=H, w=W, seed=seed)
    else:
        f, m = synth.workload_c1(seed=seed)
        f, m = f[:1, :H, :W], m[:1, :H, :W]
    return f[0], m[0], synth.measured(f, m)[0]


@pytest.mark.parametrize("H,W,kind,K", [(128, 128, "dynamic", 100), (128, 128, "fixed", 100),
                                        (132, 100, "dynamic", 100), (68, 36, "dynamic", 300)])
def test_mixed_parity(H, W, kind, K):
    R = need_gpu()
    f, m, meas = frame(3, H, W, kind)
    vals = meas.astype(np.float64)
    ora, gaps = O.fsr_frame(vals, m, K=K)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out, u8 = run(R, vals, m, K=K, counter=cnt)
    worst, namb, nb = compare_fsr(out, ora, gaps)
    print(f"mixed {H}x{W} {kind} K={K}: max {worst:.2e}, ambiguous {namb}/{nb}, recomputed in float64 "
          f"{int(host(cnt)[0])}/{nb}")
    assert worst <= FSR_TOL and namb <= AMB_MAX * nb
    sl = (slice(8, -8), slice(8, -8))
    assert abs(O.psnr(f[sl], out[sl], 0) - O.psnr(f[sl], ora[sl], 0)) <= PSNR_TOL
    assert (u8 == O.quantize(out)).all()
    assert (out[m == 1] == meas[m == 1]).all()


def blockwise(a, b, B=4):
    H, W = a.shape
    return np.abs(a.astype(np.float64) - b).reshape(H // B, B, W // B, B).max(axis=(1, 3))


@pytest.mark.parametrize("H,W,K,seed", [(1080, 1920, 100, None), (2160, 3840, 300, "4k")])
def test_mixed_every_block_follows_float64(H, W, K, seed):
    """Every block of a full frame within 1e-3 of the float64 kernel."""
    R = need_gpu()
    f, m = synth.workload_c2(n=1, h=H, w=W) if seed is None else synth.workload_c2(n=1, h=H, w=W,
                                                                                    seed=synth.seed_for(3))
    vals = synth.measured(f, m)[0].astype(np.float64)
    o64, _ = run(R, vals, m[0], K=K, precision="fp64")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    omx, _ = run(R, vals, m[0], K=K, counter=cnt)
    o32, _ = run(R, vals, m[0], K=K, precision="fp32")
    d, d32 = blockwise(omx, o64), blockwise(o32, o64)
    nb = d.size
    n = int(host(cnt)[0])
    print(f"{W}x{H} K={K}: mixed vs float64 max {d.max():.2e} (median {np.median(d):.2e}); recomputed {n}/{nb} "
          f"({100 * n / nb:.2f} %); plain float32: {(d32 > 1e-3).sum()} blocks beyond 1e-3, max {d32.max():.3g}")
    assert d.max() <= FSR_TOL
    if K == 100:
        # measured 10.1 % at the library's bound; at K = 300 the residual falls
        # much further below the float32 rounding scale and most blocks go to
        # float64 (measured 60 %)
        assert n < 0.2 * nb
    assert (d32 > 1e-3).sum() > 0     # the float32 form alone does depart: the test has teeth


def test_margin_diagnostic_calibrates_the_bound():
    """On the 1080p workload's frame, the plain float32 form's blocks that
    depart from the float64 kernel by more than 1e-3 all have margins far
    below the library's bound, and the mixed form recomputes the blocks whose
    margin is at most the bound (up to rounding of the threshold)."""
    R = need_gpu()
    H, W = 1080, 1920
    f, m = synth.workload_c2(n=1, h=H, w=W)
    vals = synth.measured(f, m)[0].astype(np.float64)
    nb = (H // 4) * (W // 4)
    margins = torch.full((nb,), float("nan"), dtype=torch.float32, device="cuda")
    o32, _ = run(R, vals, m[0], precision="fp32", margins=margins)
    o64, _ = run(R, vals, m[0], precision="fp64")
    mg = host(margins).reshape(H // 4, W // 4)
    assert not np.isnan(mg).any()      # every block wrote its margin
    bad = blockwise(o32, o64) > 1e-3
    need = float(mg[bad].max())
    a = R.MIXED_BOUND
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    run(R, vals, m[0], counter=cnt)
    n = int(host(cnt)[0])
    within = int((mg <= a).sum())
    print(f"1080p frame: float32 departs in {bad.sum()} blocks, largest margin among them {need:.3f} "
          f"(bound {a}: {a / need:.1f}x); margin <= bound: {within} blocks ({100 * within / nb:.2f} %), "
          f"recomputed by the mixed form {n}; margin quantiles 1/5/50 %: "
          f"{np.quantile(mg, 0.01):.3g} {np.quantile(mg, 0.05):.3g} {np.quantile(mg, 0.5):.3g}")
    assert bad.sum() > 0
    assert need <= a / 2
    assert abs(n - within) <= 0.001 * nb


def test_mixed_recursive_frame_teacher_forced():
    teacher_forced_case(64, 80, "nnc_frmc", "dynamic", 3, seed=31, K=100, precision="mixed")


def test_mixed_batch_and_pipeline_equal_single_frames():
    R = need_gpu()
    from test_gpu_batch import MIX, make_stream
    me, fsr = R.MEParams(search=6, check="nnc_frmc"), R.FSRParams(iters=60, precision="mixed")
    streams = [make_stream(H, W, nref, kind, 300 + i) for i, (H, W, nref, kind) in enumerate(MIX)]
    singles = [R.reconstruct_frame(cur, mask, refs, me, fsr) for cur, mask, refs in streams]
    frames = [R.BatchFrame(cur, mask, tuple(refs), out_u8=torch.empty_like(cur)) for cur, mask, refs in streams]
    for fr in frames:
        fr.out = torch.full(fr.cur.shape, float("nan"), device=fr.cur.device)
    outs = R.Batch(frames, me, fsr).run()
    for i, ((o1, u1), (o2, u2)) in enumerate(zip(singles, outs)):
        assert np.array_equal(host(o1), host(o2)), i
        assert np.array_equal(host(u1), host(u2)), i
    # a pipelined recursion equals the plain one
    H, W, T = 96, 128, 6
    rng = np.random.default_rng(9)
    fr_, _ = synth.video_translate_edges(T, H, W, rng, max_step=2, n_edges=2)
    mk = synth.mask_sequence("dynamic", T, H, W, rng)
    ms = synth.measured(fr_, mk)
    res = []
    for pipelined in (False, True):
        seq = R.Sequence(H, W, me, fsr, pipelined=pipelined)
        res.append([host(seq.push(dev(ms[t]), dev(mk[t]))[0]).copy() for t in range(T)])
    for t in range(T):
        assert np.array_equal(res[0][t], res[1][t]), t


def test_mixed_edge_cases():
    R = need_gpu()
    # a constant scene: every residual reaches the float32 rounding floor, the
    # blocks go to float64 and follow the closed form
    rng = np.random.default_rng(1)
    m = synth.fixed_mask(64, 64, rng)
    vals = np.where(m == 1, 100.0, 0.0)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out, _ = run(R, vals, m, K=40, counter=cnt)
    assert np.max(np.abs(out[m == 0] - 100.0 * (1 - 0.5 ** 40))) < 1e-3
    print(f"constant scene: recomputed {int(host(cnt)[0])}/256 blocks")
    # K = 0, no samples, one block
    f, m2, meas = frame(6, 32, 32)
    out0, _ = run(R, meas.astype(np.float32), m2, K=0)
    assert (out0[m2 == 0] == 0).all() and (out0[m2 == 1] == meas[m2 == 1]).all()
    z, _ = run(R, np.zeros((8, 8), np.float32), np.zeros((8, 8), np.uint8), K=5)
    assert (z == 0).all()
    mb = np.array([[1, 0, 1, 0], [0, 0, 0, 0], [0, 1, 0, 1], [0, 0, 0, 0]], np.uint8)
    vb = np.where(mb == 1, 50.0, 0.0)
    ora, _ = O.fsr_frame(vb, mb, K=10)
    ob, _ = run(R, vb, mb, K=10)
    assert np.max(np.abs(ob - ora)) < FSR_TOL
    # a 16384-pixel strip and K = 1024 against the oracle on its blocks
    f, m3 = synth.workload_c2(n=1, h=4, w=16384, seed=8)
    v3 = synth.measured(f, m3)[0].astype(np.float64)
    o3, _ = run(R, v3, m3[0], K=64)
    blocks = np.stack([np.zeros(64, int), np.random.default_rng(2).integers(0, 4096, 64)], axis=1)
    ora3, gaps3 = O.fsr.fsr_blocks_out(v3, m3[0], blocks, K=64)
    got3 = np.stack([o3[0:4, 4 * bj:4 * bj + 4] for _, bj in blocks])
    assert np.abs(got3 - ora3).max() <= FSR_TOL
    f, m4, meas4 = frame(7, 16, 16)
    ora4, gaps4 = O.fsr_frame(meas4.astype(np.float64), m4, K=1024)
    o4, _ = run(R, meas4.astype(np.float64), m4, K=1024)
    worst, namb, nb = compare_fsr(o4, ora4, gaps4)
    print(f"K=1024 16x16: max {worst:.2e}, ambiguous {namb}/{nb}")
    assert worst <= FSR_TOL
