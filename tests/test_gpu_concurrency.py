"""Calls on different streams with different workspaces run concurrently
and give the same results as one after another (the C ABI keeps no state
between calls)."""
import numpy as np
import pytest
import torch

import synth
from _gpu import dev, host, need_gpu

pytestmark = pytest.mark.gpu


def test_two_streams_concurrent_equal_sequential():
    R = need_gpu()
    me, fsr = R.MEParams(search=6, check="nnc_frmc"), R.FSRParams(iters=40)
    cases = []
    for s, (H, W) in enumerate([(96, 128), (64, 64), (128, 96), (48, 80)]):
        rng = np.random.default_rng(600 + s)
        frames, _ = synth.video_translate_edges(4, H, W, rng, max_step=2, n_edges=2)
        masks = synth.mask_sequence("dynamic", 4, H, W, rng)
        meas = synth.measured(frames, masks)
        refs = [(dev(frames[3 - k]), dev(meas[3 - k]), dev(masks[3 - k])) for k in (1, 2, 3)]
        cases.append((dev(meas[3]), dev(masks[3]), refs))
    seq = [tuple(host(t).copy() for t in R.reconstruct_frame(c, m, r, me, fsr)) for c, m, r in cases]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [R.Workspace(), R.Workspace()]
    outs = []
    torch.cuda.synchronize()
    for rep in range(3):
        outs.clear()
        for i, (c, m, r) in enumerate(cases):
            k = i % 2
            with torch.cuda.stream(streams[k]):
                outs.append(R.reconstruct_frame(c, m, r, me, fsr, workspace=wss[k], stream=streams[k]))
        torch.cuda.synchronize()
        for i, (o, u) in enumerate(outs):
            assert np.array_equal(host(o), seq[i][0]), (rep, i)
            assert np.array_equal(host(u), seq[i][1]), (rep, i)
