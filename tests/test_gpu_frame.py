"""GPU parity of rfsr_reconstruct_frame (Fig. 1 order: ME, check,
projection, FSR, overwrite, quantisation) and of the causal recursion."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import AMB_MAX, FLOAT64_FORMS, FSR_TOL, PSNR_TOL, compare_fsr, dev, host, need_gpu

pytestmark = pytest.mark.gpu


def teacher_forced_case(H, W, check, kind, nref, seed, K=60, search=8, overwrite="dfsr", me_opts=None,
                        precision="fp64"):
    R = need_gpu()
    rng = np.random.default_rng(seed)
    frames, _ = synth.video_translate_edges(nref + 1, H, W, rng, max_step=3, n_edges=3)
    masks = synth.mask_sequence(kind, nref + 1, H, W, rng)
    meas = synth.measured(frames, masks)
    t = nref
    # both sides consume the same uint8 references (true frames, lightly perturbed)
    recon = [np.clip(frames[t - 1 - k].astype(int) + rng.integers(-3, 4, (H, W)), 0, 255).astype(np.uint8)
             for k in range(nref)]
    refs = [(recon[k], meas[t - 1 - k], masks[t - 1 - k]) for k in range(nref)]
    me_opts = me_opts or {}
    me = O.MEParams(search=search, check=check, **me_opts)
    fsr = O.FSRParams(iters=K, overwrite=overwrite)
    ora = O.reconstruct_frame(meas[t], masks[t], refs, me, fsr)
    out, out_u8 = R.reconstruct_frame(dev(meas[t]), dev(masks[t]),
                                      [(dev(r), dev(mm), dev(b)) for r, mm, b in refs],
                                      R.MEParams(search=search, check=check, **me_opts),
                                      R.FSRParams(iters=K, overwrite=overwrite, precision=precision))
    out, out_u8 = host(out), host(out_u8)
    worst, namb, nb = compare_fsr(out, ora["out"], ora["gaps"])
    print(f"frame {precision} {H}x{W} {check} {kind} nref={nref}: max {worst:.2e}, ambiguous {namb}/{nb}, "
          f"projected {(ora['cls'] == 2).mean():.3f}")
    assert worst <= FSR_TOL
    assert namb <= AMB_MAX * nb
    assert abs(O.psnr(frames[t], out, 8) - O.psnr(frames[t], ora["out"], 8)) <= PSNR_TOL
    assert (out_u8 == O.quantize(out)).all()
    return ora


@pytest.mark.parametrize("check,kind,nref", [("nnc_frmc", "dynamic", 3), ("rme", "fixed", 2),
                                             ("rmc", "dynamic", 1), ("none", "dynamic", 3),
                                             ("frmc", "fixed", 3), ("nnc", "dynamic", 2)])
@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_frame_teacher_forced(check, kind, nref, precision):
    teacher_forced_case(64, 80, check, kind, nref, seed=10 + nref, precision=precision)


@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_frame_rfsr_overwrite(precision):
    teacher_forced_case(64, 64, "nnc_frmc", "dynamic", 3, seed=3, overwrite="rfsr", precision=precision)


def test_frame_no_reference_is_single_frame_fsr():
    R = need_gpu()
    f, m = synth.workload_c2(n=1, h=64, w=64, seed=2)
    meas = synth.measured(f, m)[0]
    out, _ = R.reconstruct_frame(dev(meas), dev(m[0]), [], R.MEParams(), R.FSRParams(iters=40))
    out2, _ = R.fsr_blocks(dev(meas.astype(np.float32)), dev(m[0]), R.FSRParams(iters=40))
    assert np.array_equal(host(out), host(out2))


def test_sequence_free_running_psnr():
    """Free-running recursion (each side consumes its own reconstructions):
    per-frame PSNR within 0.01 dB of the oracle's recursion."""
    R = need_gpu()
    rng = np.random.default_rng(21)
    H = W = 64
    frames, _ = synth.video_translate_edges(5, H, W, rng, max_step=2, n_edges=2)
    masks = synth.mask_sequence("dynamic", 5, H, W, rng)
    meas = synth.measured(frames, masks)
    me, fsr = O.MEParams(search=5, check="nnc_frmc"), O.FSRParams(iters=40)
    ora = O.reconstruct_sequence(meas, masks, me, fsr)
    seq = R.Sequence(H, W, R.MEParams(search=5, check="nnc_frmc"), R.FSRParams(iters=40))
    for t in range(5):
        out, _ = seq.push(dev(meas[t]), dev(masks[t]))
        p_g = O.psnr(frames[t], host(out), 8)
        p_o = O.psnr(frames[t], ora[t]["out"], 8)
        print(f"t={t}: gpu {p_g:.4f} dB oracle {p_o:.4f} dB")
        assert abs(p_g - p_o) <= PSNR_TOL


def test_sequence_rejects_an_output_it_still_reads():
    """An out_u8 that is one of the ring's reference planes would be
    overwritten while the frame reads it: push() refuses it, in both modes;
    one unchanged mask tensor for every frame is accepted."""
    R = need_gpu()
    rng = np.random.default_rng(22)
    H = W = 32
    frames, _ = synth.video_translate_edges(3, H, W, rng, max_step=1, n_edges=1)
    mask = synth.fixed_mask(H, W, rng)
    meas = synth.measured(frames, np.stack([mask] * 3))
    m_d = dev(mask)
    for pipelined in (False, True):
        seq = R.Sequence(H, W, R.MEParams(search=3), R.FSRParams(iters=10), pipelined=pipelined)
        u8 = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        seq.push(dev(meas[0]), m_d, out_u8=u8)
        with pytest.raises(R.RfsrError):
            seq.push(dev(meas[1]), m_d, out_u8=u8)
        seq.push(dev(meas[1]), m_d)
        torch.cuda.synchronize()


@pytest.mark.parametrize("check", ["nnc_frmc", "rme", "rmc"])
def test_frame_ignores_unmeasured_values(check):
    """Values of the current and the reference measured frames at unmeasured
    positions never influence a result: random bytes there (instead of the
    zeros the quarter sampling leaves) give bit-identical motion fields,
    decisions and reconstructions.  Ragged 44x60 frame (not a multiple of the
    16x16 ME tile), three references."""
    R = need_gpu()
    rng = np.random.default_rng(44)
    H, W = 44, 60
    frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=3, n_edges=3)
    masks = synth.mask_sequence("dynamic", 4, H, W, rng)
    meas = synth.measured(frames, masks)
    dirty = [np.where(m == 1, f, rng.integers(0, 256, f.shape)).astype(np.uint8) for f, m in zip(meas, masks)]
    recon = [frames[2 - k] for k in range(3)]
    me, fsr = R.MEParams(search=6, check=check), R.FSRParams(iters=30)
    outs = []
    for src in (meas, dirty):
        refs = [(dev(recon[k]), dev(src[2 - k]), dev(masks[2 - k])) for k in range(3)]
        o, u = R.reconstruct_frame(dev(src[3]), dev(masks[3]), refs, me, fsr)
        mv, acc, cost = R.motion_check(dev(src[3]), dev(masks[3]), dev(recon[0]), me)
        outs.append([host(x) for x in (o, u, mv, acc, cost)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("check", ["nnc_frmc", "rmc", "rme"])
@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_frame_split_equals_whole(check, precision):
    """rfsr_frame_motion(first) + rfsr_frame_finish(first) on one workspace
    give bit-identical outputs to rfsr_reconstruct_frame for every split
    point first = 0..3 (ragged 44x60 frame, three references)."""
    R = need_gpu()
    rng = np.random.default_rng(45)
    H, W = 44, 60
    frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=3, n_edges=3)
    masks = synth.mask_sequence("dynamic", 4, H, W, rng)
    meas = synth.measured(frames, masks)
    refs = [(dev(frames[2 - k]), dev(meas[2 - k]), dev(masks[2 - k])) for k in range(3)]
    cur, mask = dev(meas[3]), dev(masks[3])
    me, fsr = R.MEParams(search=6, check=check), R.FSRParams(iters=30, precision=precision)
    o, u = R.reconstruct_frame(cur, mask, refs, me, fsr)
    whole = (host(o), host(u))
    nbytes = R.workspace_bytes(H, W, 3, me, fsr)
    for first in range(4):
        ws = R.Workspace()
        ws.get(nbytes).random_(0, 256)   # no state from an earlier call can help
        R.frame_motion(cur, mask, refs, me, first, workspace=ws)
        o2, u2 = R.reconstruct_frame(cur, mask, refs, me, fsr, workspace=ws, first=first)
        assert np.array_equal(host(o2), whole[0]) and np.array_equal(host(u2), whole[1]), first


@pytest.mark.parametrize("H,W,T,check,nref", [(64, 80, 7, "nnc_frmc", 3), (64, 80, 6, "rme", 3),
                                              (64, 80, 6, "rmc", 3), (64, 80, 6, "frmc", 3),
                                              (64, 80, 6, "none", 3), (64, 80, 6, "nnc_frmc", 2),
                                              (64, 80, 5, "nnc_frmc", 1), (1080, 1920, 5, "nnc_frmc", 3)])
@pytest.mark.parametrize("precision", FLOAT64_FORMS)
def test_pipelined_sequence_equals_plain(H, W, T, check, nref, precision):
    """The pipelined recursion (early motion path of the lag >= 2 references
    on a side stream, overlapping the previous frame's FSR) reproduces the
    plain recursion bit for bit, frame by frame."""
    R = need_gpu()
    frames, masks = synth.workload_c2(n=T, h=H, w=W, seed=synth.seed_for(7))
    meas = synth.measured(frames, masks)
    d_meas = [dev(x) for x in meas]
    d_mask = [dev(x) for x in masks]
    torch.cuda.synchronize()
    me, fsr = R.MEParams(search=9, check=check), R.FSRParams(iters=100, precision=precision)
    res = []
    for pipelined in (False, True):
        seq = R.Sequence(H, W, me, fsr, nref=nref, pipelined=pipelined)
        outs = [seq.push(d_meas[t], d_mask[t]) for t in range(T)]
        torch.cuda.synchronize()
        res.append([(host(o), host(u)) for o, u in outs])
    for t in range(T):
        assert np.array_equal(res[0][t][0], res[1][t][0]) and np.array_equal(res[0][t][1], res[1][t][1]), t
