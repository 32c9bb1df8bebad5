"""Pins of the oracle's projection (Sec. 2.2): closed forms on static
scenes under dynamic and fixed quarter masks, and the averaging rule."""
import numpy as np

import oracle as O
import synth


def _zero_fields(H, W, meas, mask, accept=True):
    z = np.zeros((H, W), np.int64)
    return dict(alpha=z, beta=z, accept=np.full((H, W), accept), meas=meas, mask=mask)


def test_static_scene_dynamic_mask_fills_everything():
    """Static scene, dynamic mask, three references, every vector zero and
    accepted: each missing pixel of frame t>=3 was measured in exactly one of
    t-1..t-3, so projection recovers every pixel exactly."""
    rng = np.random.default_rng(0)
    H, W = 24, 30
    f = rng.integers(0, 256, (H, W)).astype(np.uint8)
    masks = synth.mask_sequence("dynamic", 4, H, W, rng)
    meas = synth.measured(np.stack([f] * 4), masks)
    refs = [_zero_fields(H, W, meas[3 - k], masks[3 - k]) for k in (1, 2, 3)]
    vals, cls = O.project(meas[3], masks[3], refs)
    assert set(np.unique(cls)) == {1, 2}
    assert (vals == f).all()
    assert ((cls == 1) == (masks[3] == 1)).all()


def test_fixed_mask_zero_motion_projects_nothing():
    rng = np.random.default_rng(1)
    H, W = 16, 16
    f = rng.integers(0, 256, (H, W)).astype(np.uint8)
    masks = synth.mask_sequence("fixed", 4, H, W, rng)
    meas = synth.measured(np.stack([f] * 4), masks)
    refs = [_zero_fields(H, W, meas[3 - k], masks[3 - k]) for k in (1, 2, 3)]
    _, cls = O.project(meas[3], masks[3], refs)
    assert not (cls == 2).any()


def test_rejected_vectors_do_not_project():
    rng = np.random.default_rng(2)
    H, W = 16, 16
    f = rng.integers(0, 256, (H, W)).astype(np.uint8)
    masks = synth.mask_sequence("dynamic", 2, H, W, rng)
    meas = synth.measured(np.stack([f] * 2), masks)
    _, cls = O.project(meas[1], masks[1], [_zero_fields(H, W, meas[0], masks[0], accept=False)])
    assert not (cls == 2).any()


def test_average_of_several_sources():
    H, W = 4, 4
    cur = np.zeros((H, W), np.uint8)
    cmask = np.zeros((H, W), np.uint8)
    cmask[0, 0] = 1
    cur[0, 0] = 9
    ones = np.ones((H, W), np.uint8)
    z = np.zeros((H, W), np.int64)
    r1 = dict(alpha=z, beta=z, accept=np.ones((H, W), bool), meas=np.full((H, W), 10, np.uint8), mask=ones)
    r2 = dict(alpha=z, beta=z, accept=np.ones((H, W), bool), meas=np.full((H, W), 13, np.uint8), mask=ones)
    r3 = dict(alpha=z, beta=z, accept=np.ones((H, W), bool), meas=np.full((H, W), 20, np.uint8), mask=ones)
    vals, cls = O.project(cur, cmask, [r1, r2, r3])
    assert vals[0, 0] == 9 and cls[0, 0] == 1
    assert (vals[cls == 2] == (10 + 13 + 20) / 3).all()
    # a vector pointing to an unmeasured pixel of a reference does not project
    r3["mask"] = np.zeros((H, W), np.uint8)
    vals, _ = O.project(cur, cmask, [r1, r2, r3])
    assert (vals[cls == 2] == 11.5).all()


def test_projection_follows_vectors():
    H, W = 6, 6
    cur = np.zeros((H, W), np.uint8)
    cmask = np.zeros((H, W), np.uint8)
    meas = np.arange(H * W, dtype=np.uint8).reshape(H, W)
    a = np.zeros((H, W), np.int64)
    b = np.zeros((H, W), np.int64)
    a[2, 3], b[2, 3] = 1, -2
    ref = dict(alpha=a, beta=b, accept=np.ones((H, W), bool), meas=meas, mask=np.ones((H, W), np.uint8))
    vals, _ = O.project(cur, cmask, [ref])
    assert vals[2, 3] == meas[3, 1]
