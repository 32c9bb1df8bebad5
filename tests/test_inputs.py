"""Seeded input generators: quarter-mask invariants (introduction and
Sec. 2.1 sampling model; dynamic mask: each 2x2 position read exactly once
within four frames, pattern repeating every fourth frame)."""
import numpy as np

import synth


def cells(m):
    H, W = m.shape
    return m.reshape(H // 2, 2, W // 2, 2).transpose(0, 2, 1, 3).reshape(H // 2, W // 2, 4)


def test_fixed_mask_one_per_cell():
    rng = np.random.default_rng(1)
    m = synth.mask_sequence("fixed", 5, 64, 48, rng)
    assert m.dtype == np.uint8 and set(np.unique(m)) <= {0, 1}
    for t in range(5):
        assert (cells(m[t]).sum(-1) == 1).all()
        assert (m[t] == m[0]).all()
    # positions are spread over all four cell positions
    counts = cells(m[0]).sum(axis=(0, 1))
    assert (counts > 0).all()


def test_dynamic_mask_each_position_once_per_four_frames():
    rng = np.random.default_rng(2)
    m = synth.mask_sequence("dynamic", 11, 32, 40, rng)
    for t in range(11):
        assert (cells(m[t]).sum(-1) == 1).all()
    for t0 in range(11 - 3):
        window = sum(cells(m[t]).astype(int) for t in range(t0, t0 + 4))
        assert (window == 1).all()
    for t in range(11 - 4):
        assert (m[t + 4] == m[t]).all()


def test_measured_is_frame_times_mask():
    frames, masks = synth.workload_c1()
    meas = synth.measured(frames, masks)
    assert (meas[masks == 1] == frames[masks == 1]).all()
    assert (meas[masks == 0] == 0).all()


def test_generators_seeded_and_shaped():
    f1, m1 = synth.workload_c1()
    f2, m2 = synth.workload_c1()
    assert (f1 == f2).all() and (m1 == m2).all()
    assert f1.shape == (4, 128, 128) and f1.dtype == np.uint8
    f, m = synth.workload_c2(n=3, h=96, w=160)
    assert f.shape == (3, 96, 160) and m.shape == (3, 96, 160)
    assert f.std() > 5


def test_multistream_workload_sizes_and_masks():
    assert len(synth.C4_SIZES) == 48
    assert sum(h * w for h, w in synth.C4_SIZES) == 74_428_416
    small = [(32, 48), (16, 24), (24, 16)]
    ws = synth.workload_c4(n=4, sizes=small)
    for s, ((f, m), (h, w)) in enumerate(zip(ws, small)):
        assert f.shape == m.shape == (4, h, w)
        cells = m.reshape(4, h // 2, 2, w // 2, 2).sum(axis=(2, 4))
        assert (cells == 1).all()
        if s % 2 == 0:   # fixed
            assert (m == m[0]).all()
        else:            # dynamic: every position once in four frames
            assert (m.sum(axis=0) == 1).all()
