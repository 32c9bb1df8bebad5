"""Serving on the GPU: requests of concurrent streams of different sizes go
through the continuous-batching server (batches overlapping on two device
streams); every result equals, bit for bit, the same stream reconstructed
alone on the single-frame path."""
import numpy as np
import pytest
import torch

import synth
from _gpu import dev, host, need_gpu

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (48, 96), (32, 32), (96, 64), (64, 128), (16, 24)]
FRAMES = 7


def stream_data():
    data = []
    for s, (H, W) in enumerate(SIZES):
        rng = np.random.default_rng(500 + s)
        f, _ = synth.video_translate_edges(FRAMES, H, W, rng, max_step=2, n_edges=2)
        m = synth.mask_sequence("fixed" if s % 2 == 0 else "dynamic", FRAMES, H, W, rng)
        data.append(([dev(x) for x in synth.measured(f, m)], [dev(x) for x in m]))
    return data


def alone(data, R, me, fsr):
    res = []
    for s, (H, W) in enumerate(SIZES):
        q = R.Sequence(H, W, me, fsr)
        outs = []
        for t in range(FRAMES):
            o, u = q.push(data[s][0][t], data[s][1][t])
            outs.append((host(o).copy(), host(u).copy()))
        res.append(outs)
    return res


@pytest.mark.parametrize("mode,arrivals,precision", [("batch", "burst", "fp64"), ("batch", "poisson", "fp64"),
                                                     ("frame", "poisson", "fp64"), ("batch", "burst", "mixed"),
                                                     ("batch", "poisson", "mixed")])
def test_served_results_equal_alone(mode, arrivals, precision):
    R = need_gpu()
    from paper_2203_09200_amd import serving as S
    me, fsr = R.MEParams(search=5, check="nnc_frmc"), R.FSRParams(iters=30, precision=precision)
    data = stream_data()
    ref = alone(data, R, me, fsr)

    def keep(reqs, hs):    # runs on the batch's device stream right after it
        for r in reqs:
            r.res = (r.out.clone(), r.out_u8.clone())

    ex = S.GpuExecutor(me, fsr, mode=mode, max_inflight=2, on_launch=keep)
    srv = S.Server(ex, 1 << 34, max_batch=4, max_inflight=2)
    sids = [srv.open_stream(H, W) for H, W in SIZES]
    if arrivals == "burst":
        trace = sorted((0.0, s, t) for t in range(FRAMES) for s in range(len(SIZES)))
    else:
        _, trace = S.poisson_trace(len(SIZES), FRAMES, 400.0, np.random.default_rng(7), sizes=SIZES)
    reqs = S.run_trace(srv, trace, lambda s, t: (data[s][0][t], data[s][1][t]), sids)
    torch.cuda.synchronize()
    assert len(reqs) == len(SIZES) * FRAMES
    for r in reqs:
        s = sids.index(r.stream)
        o, u = ref[s][r.index]
        assert np.array_equal(host(r.res[0]), o), f"stream {s} frame {r.index}"
        assert np.array_equal(host(r.res[1]), u), f"stream {s} frame {r.index}"
        assert r.done >= r.arrival - 1e-3   # device completion clock vs host arrival clock
    if mode == "batch":
        assert max(n for _, n in srv.batches) > 1      # frames of different streams were mixed
    assert srv.peak <= srv.budget
