"""Pins of the oracle's frame pipeline (Fig. 1 order) and PSNR (Sec. 4)."""
import numpy as np

import oracle as O
import synth


def test_psnr_known_mse():
    ref = np.zeros((100, 100))
    test = np.full((100, 100), 5.0)
    assert abs(O.psnr(ref, test) - 10 * np.log10(255 ** 2 / 25)) < 1e-12
    test[:40] = 1e6      # inside the omitted border rows: no effect, clipping otherwise
    assert abs(O.psnr(ref, test) - 10 * np.log10(255 ** 2 / 25)) < 1e-12
    assert O.psnr(ref, ref) == np.inf


def test_quantize_round_half_even_and_clip():
    x = np.array([-3.0, 0.5, 1.5, 2.5, 254.5, 255.49, 400.0])
    assert list(O.quantize(x)) == [0, 0, 2, 2, 254, 255, 255]


def test_no_reference_is_single_frame_fsr():
    f, m = synth.workload_c2(n=1, h=40, w=48, seed=5)
    meas = synth.measured(f, m)
    me, fsr = O.MEParams(search=4), O.FSRParams(iters=15)
    res = O.reconstruct_frame(meas[0], m[0], [], me, fsr)
    out, _ = O.fsr_frame(meas[0].astype(float), m[0], K=15)
    assert (res["out"] == out).all()


def test_recursion_helps_on_translating_scene():
    """The recursion (D-FSR + NNC + FRMC, dynamic mask) beats single-frame
    FSR once three references exist (Sec. 4, Table 2 trend)."""
    rng = np.random.default_rng(9)
    H = W = 64
    frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=2, n_edges=2)
    masks = synth.mask_sequence("dynamic", 4, H, W, rng)
    meas = synth.measured(frames, masks)
    me, fsr = O.MEParams(search=4, check="nnc_frmc"), O.FSRParams(iters=40)
    res = O.reconstruct_sequence(meas, masks, me, fsr)
    single, _ = O.fsr_frame(meas[3].astype(float), masks[3], K=40)
    p_rec = O.psnr(frames[3], res[3]["out"], border=8)
    p_single = O.psnr(frames[3], single, border=8)
    assert (res[3]["cls"] == 2).mean() > 0.1
    assert p_rec > p_single + 1.0
