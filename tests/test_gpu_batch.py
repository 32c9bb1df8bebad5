"""GPU tests of rfsr_reconstruct_batch: many streams of different sizes,
masks and reference counts in one launch chain give exactly (bit for bit)
what rfsr_reconstruct_frame gives on each frame alone; graph replays of the
chain equal eager runs; a job-table image built for other descriptors makes
the kernels skip all work."""
import numpy as np
import pytest
import torch

import synth
from _gpu import dev, host, need_gpu

pytestmark = pytest.mark.gpu

# (H, W, nref, mask kind): uneven sizes, ragged 4-multiples, frames without references
MIX = [(64, 64, 3, "dynamic"), (48, 96, 2, "fixed"), (96, 44, 1, "dynamic"), (32, 32, 0, "fixed"),
       (128, 160, 3, "dynamic"), (20, 36, 3, "fixed"), (4, 8, 1, "dynamic")]


def make_stream(H, W, nref, kind, seed):
    rng = np.random.default_rng(seed)
    frames, _ = synth.video_translate_edges(nref + 1, H, W, rng, max_step=2, n_edges=2)
    masks = synth.mask_sequence(kind, nref + 1, H, W, rng)
    meas = synth.measured(frames, masks)
    recon = [np.clip(frames[nref - 1 - k].astype(int) + rng.integers(-3, 4, (H, W)), 0, 255).astype(np.uint8)
             for k in range(nref)]
    refs = [(dev(recon[k]), dev(meas[nref - 1 - k]), dev(masks[nref - 1 - k])) for k in range(nref)]
    return dev(meas[nref]), dev(masks[nref]), refs


@pytest.mark.parametrize("check", ["nnc_frmc", "rme", "rmc", "frmc", "nnc", "none"])
def test_batch_equals_single_frames(check):
    R = need_gpu()
    me, fsr = R.MEParams(search=6, check=check), R.FSRParams(iters=30)
    streams = [make_stream(H, W, nref, kind, 100 + i) for i, (H, W, nref, kind) in enumerate(MIX)]
    singles = [R.reconstruct_frame(cur, mask, refs, me, fsr) for cur, mask, refs in streams]
    frames = [R.BatchFrame(cur, mask, tuple(refs), out_u8=torch.empty_like(cur)) for cur, mask, refs in streams]
    for f in frames:
        f.out = torch.full(f.cur.shape, float("nan"), device=f.cur.device)
    b = R.Batch(frames, me, fsr)
    outs = b.run()
    for i, ((o1, u1), (o2, u2)) in enumerate(zip(singles, outs)):
        a1, a2 = host(o1), host(o2)
        assert np.array_equal(a1, a2), f"frame {i} {MIX[i]}: max diff {np.nanmax(np.abs(a1 - a2))}"
        assert np.array_equal(host(u1), host(u2)), f"frame {i}"


def test_batch_of_one_1080p_frame_equals_single():
    R = need_gpu()
    f, m = synth.workload_c2(n=4, h=1080, w=1920)
    meas = synth.measured(f, m)
    refs = [(dev(f[3 - k]), dev(meas[3 - k]), dev(m[3 - k])) for k in (1, 2, 3)]
    me, fsr = R.MEParams(search=9, check="nnc_frmc"), R.FSRParams(iters=100)
    o1, u1 = R.reconstruct_frame(dev(meas[3]), dev(m[3]), refs, me, fsr)
    b = R.Batch([R.BatchFrame(dev(meas[3]), dev(m[3]), tuple(refs), out_u8=torch.empty_like(u1))], me, fsr)
    (o2, u2), = b.run()
    assert np.array_equal(host(o1), host(o2))
    assert np.array_equal(host(u1), host(u2))


def test_stream_set_with_graphs_equals_sequences():
    """Causal recursion of three streams of different sizes, eight time steps,
    as one batch per step (graphs captured from t = 3 and replayed, with
    eager input copies between replays) against each stream's own Sequence
    on the single-frame path: identical outputs at every step."""
    R = need_gpu()
    sizes = [(64, 64), (48, 80), (32, 96)]
    T = 8
    me, fsr = R.MEParams(search=5, check="nnc_frmc"), R.FSRParams(iters=30)
    data = []
    for i, (H, W) in enumerate(sizes):
        rng = np.random.default_rng(300 + i)
        frames, _ = synth.video_translate_edges(T, H, W, rng, max_step=2, n_edges=2)
        masks = synth.mask_sequence("dynamic", T, H, W, rng)
        data.append((synth.measured(frames, masks), masks))
    ss = R.StreamSet(sizes, me, fsr, graphs=True)
    seqs = [R.Sequence(H, W, me, fsr) for H, W in sizes]
    for t in range(T):
        meas_t = [dev(d[0][t]) for d in data]
        mask_t = [dev(d[1][t]) for d in data]
        got = ss.step(meas_t, mask_t)
        for s in range(len(sizes)):
            ref_out, ref_u8 = seqs[s].push(meas_t[s], mask_t[s])
            assert np.array_equal(host(got[s][0]), host(ref_out)), f"t={t} stream {s}"
            assert np.array_equal(host(got[s][1]), host(ref_u8)), f"t={t} stream {s}"
    assert len(ss._graphs) == 4   # one per ring phase, each replayed at least once


@pytest.mark.parametrize("check", ["nnc_frmc", "rme"])
def test_pipelined_stream_set_equals_plain(check):
    """Pipelined time steps (every stream's lag-2/3 motion path on a side
    stream beside the previous step's FSR; rfsr_reconstruct_batch_part)
    against the plain batched recursion: identical outputs at every step.
    Four streams of different sizes, nine steps, no synchronisation between
    steps (each step's outputs are cloned on the main stream)."""
    R = need_gpu()
    sizes = [(64, 64), (48, 80), (32, 96), (128, 160)]
    T = 9
    me, fsr = R.MEParams(search=6, check=check), R.FSRParams(iters=40)
    data = []
    for i, (H, W) in enumerate(sizes):
        rng = np.random.default_rng(500 + i)
        frames, _ = synth.video_translate_edges(T, H, W, rng, max_step=2, n_edges=2)
        masks = synth.mask_sequence("dynamic" if i % 2 else "fixed", T, H, W, rng)
        data.append(([dev(x) for x in synth.measured(frames, masks)], [dev(x) for x in masks]))
    torch.cuda.synchronize()
    res = []
    for pipelined in (False, True):
        ss = R.StreamSet(sizes, me, fsr, graphs=False, pipelined=pipelined)
        outs = []
        for t in range(T):
            got = ss.step([d[0][t] for d in data], [d[1][t] for d in data])
            outs.append([(o.clone(), u.clone()) for o, u in got])
        torch.cuda.synchronize()
        res.append([[(host(o), host(u)) for o, u in step] for step in outs])
    for t in range(T):
        for s in range(len(sizes)):
            assert np.array_equal(res[0][t][s][0], res[1][t][s][0]), (t, s)
            assert np.array_equal(res[0][t][s][1], res[1][t][s][1]), (t, s)


def test_graph_replays_equal_eager():
    R = need_gpu()
    me, fsr = R.MEParams(search=6, check="nnc_frmc"), R.FSRParams(iters=30)
    streams = [make_stream(H, W, nref, kind, 200 + i) for i, (H, W, nref, kind) in enumerate(MIX)]
    frames = [R.BatchFrame(cur, mask, tuple(refs), out_u8=torch.empty_like(cur)) for cur, mask, refs in streams]
    b = R.Batch(frames, me, fsr)
    eager = [(host(o).copy(), host(u).copy()) for o, u in b.run()]
    g = b.capture()
    for rep in range(3):
        for f in frames:           # eager work between replays
            f.out.fill_(-1.0)
            f.out_u8.zero_()
        torch.cuda.synchronize()
        g.replay()
        for i, f in enumerate(frames):
            assert np.array_equal(host(f.out), eager[i][0]), f"replay {rep} frame {i}"
            assert np.array_equal(host(f.out_u8), eager[i][1]), f"replay {rep} frame {i}"


def test_stale_job_tables_skip_all_work():
    R = need_gpu()
    me, fsr = R.MEParams(search=4, check="nnc_frmc"), R.FSRParams(iters=10)
    s1 = [make_stream(32, 32, 2, "dynamic", 400), make_stream(16, 24, 0, "fixed", 401)]
    fa = [R.BatchFrame(c, m, tuple(r)) for c, m, r in s1]
    fb = [R.BatchFrame(c, m, tuple(r)) for c, m, r in s1]
    a = R.Batch(fa, me, fsr)
    b = R.Batch(fb, me, fsr, workspace=a.workspace)
    for f in fa + fb:
        f.out.fill_(7.0)
    b.tables.copy_(a.tables)       # image of other descriptors (other outputs)
    b.run()
    torch.cuda.synchronize()
    for f in fa + fb:
        assert (host(f.out) == 7.0).all()
