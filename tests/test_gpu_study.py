"""Quality study on synthetic video (Tables 1-2 / Fig. 4 analogue), small
configuration: orderings that follow from the method rather than from the
paper's sequences."""
import numpy as np
import pytest
import torch

import synth
from _gpu import need_gpu

pytestmark = pytest.mark.gpu


def test_recursion_beats_single_frame_fsr():
    R = need_gpu()
    from paper_2203_09200_amd import study
    H = W = 128
    T, S = 12, 3
    seqs, masks = [], []
    for s in range(S):
        rng = np.random.default_rng(synth.seed_for(6, s))
        seqs.append(synth.video_regions(T, H, W, rng))
        masks.append(synth.mask_sequence("dynamic", T, H, W, rng))
    dev = torch.device("cuda")
    res = {}
    for m in study.METHODS:
        p, s = study.run(seqs, m, masks, R, torch, dev)
        assert np.isfinite(p).all() and ((s > 0) & (s <= 1)).all()
        res[m[0]] = p
    fsr = res["FSR"]
    for name, p in res.items():
        print(f"{name:15s} {p.mean():.3f} dB (frame 0 {p[:, 0].mean():.3f})")
        # frame 0 has no reference: every method is single-frame FSR there
        assert np.allclose(p[:, 0], fsr[:, 0])
    for name in ("D-FSR+RME", "D-FSR+RMC", "D-FSR+FRMC", "D-FSR+NNC+FRMC"):
        assert res[name][:, 1:].mean() > fsr[:, 1:].mean() + 0.3, name
    # writing projected samples over the model (R-FSR) is worse than keeping them as samples (D-FSR)
    assert res["D-FSR+RME"].mean() > res["R-FSR+RME"].mean()
