"""Pins of where the oracle's FSR reads and writes a block (Sec. 2.1: each
block is modelled on a support that surrounds it) and of which frames the
recursion pairs (Sec. 4: the three previous frames).

* A frame A (-1)^y is the Nyquist-row basis function (16, 0) on every
  support, so every block reconstructs it in closed form; a support or
  synthesis window shifted by one row flips the sign of the block.
* Mirroring the frame mirrors the output exactly when the support is centred
  on its block (the mirrored support is then the support of the mirrored
  block), so an off-centre support breaks the equivariance even where the
  gather and the synthesis windows are shifted together.
* The recursion hands frame t the reconstruction, the measured frame and the
  mask of the same earlier frame t-1-k as its reference of lag k+1."""
import numpy as np
import pytest

import oracle as O
import oracle.frame as OF
from oracle import fsr as F
import synth

B, M, GAMMA = 4, 32, 0.5


@pytest.mark.parametrize("axis", [0, 1])
def test_nyquist_frame_closed_form(axis):
    """Samples A (-1)^y (or A (-1)^x) under a quarter mask: the single
    self-conjugate bin (16, 0) (or (0, 16)) is chosen until the residual
    reaches rounding level, so unknown pixels equal A (1-(1-gamma)^K) (-1)^y,
    border blocks (supports partly outside the frame) included."""
    rng = np.random.default_rng(20 + axis)
    H, W, A, K = 48, 40, 50.0, 100
    mask = synth.fixed_mask(H, W, rng)
    y, x = np.mgrid[0:H, 0:W]
    truth = A * (-1.0) ** (y if axis == 0 else x)
    vals = np.where(mask == 1, truth, 0.0)
    out, _ = O.fsr_frame(vals, mask, K=K, gamma=GAMMA)
    expect = A * (1 - (1 - GAMMA) ** K) * (-1.0) ** (y if axis == 0 else x)
    unknown = mask == 0
    assert np.max(np.abs(out[unknown] - expect[unknown])) < 1e-9
    assert (out[mask == 1] == vals[mask == 1]).all()


def test_nyquist_block_sign_at_odd_block_rows():
    """The same closed form block by block through fsr_blocks_out, at blocks
    whose first row is a multiple of 4 plus an odd support offset: a window
    one row off gives -A instead of +A at every unknown pixel."""
    rng = np.random.default_rng(31)
    H, W, A, K = 64, 64, 80.0, 60
    mask = synth.fixed_mask(H, W, rng)
    y = np.mgrid[0:H, 0:W][0]
    vals = np.where(mask == 1, A * (-1.0) ** y, 0.0)
    blocks = np.array([[0, 0], [1, 3], [7, 2], [15, 15], [8, 9]])
    out, _ = F.fsr_blocks_out(vals, mask, blocks, K=K, gamma=GAMMA)
    scale = A * (1 - (1 - GAMMA) ** K)
    for (bi, bj), o in zip(blocks, out):
        rows = 4 * bi + np.arange(B)
        want = scale * (-1.0) ** rows[:, None] * np.ones((1, B))
        unk = mask[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] == 0
        assert np.max(np.abs(o[unk] - want[unk])) < 1e-9, (bi, bj)


@pytest.mark.parametrize("b", [(3, 5), (29, 2), (16, 7)])
def test_synthesize_reads_the_centre_of_the_support(b):
    """A model of one complex coefficient z at bin b is z phi_b; the block
    output is its real part at support rows and columns 14..17 ((M - B) / 2
    onwards), the block's place in the centre of its support."""
    z = 2.5 - 1.25j
    c = np.zeros((1, M, M), np.complex128)
    c[0, b[0], b[1]] = z
    out = F.synthesize(c, B)[0]
    o = (M - B) // 2
    assert o == 14
    m = np.arange(o, o + B)
    phi = np.exp(2j * np.pi * (b[0] * m[:, None] + b[1] * m[None, :]) / M)
    assert np.allclose(out, (z * phi).real, atol=1e-12, rtol=0)
    # the neighbouring windows give a different block: the pin has teeth
    for s in (-1, 1):
        ms = m + s
        phis = np.exp(2j * np.pi * (b[0] * ms[:, None] + b[1] * ms[None, :]) / M)
        assert np.max(np.abs(out - (z * phis).real)) > 1e-3


@pytest.mark.parametrize("flip", ["rows", "cols"])
def test_mirror_equivariance(flip):
    """Mirroring frame and mask mirrors the reconstruction (to rounding)
    outside blocks whose greedy loop meets a near tie (where the mirrored
    problem may take the other equally valid pick)."""
    f, m = synth.workload_c2(n=1, h=48, w=56, seed=4)
    meas = synth.measured(f, m)[0].astype(np.float64)
    mask = m[0]
    ax = 0 if flip == "rows" else 1
    out, gaps = O.fsr_frame(meas, mask, K=40)
    outf, gapsf = O.fsr_frame(np.flip(meas, ax).copy(), np.flip(mask, ax).copy(), K=40)
    back = np.flip(outf, ax)
    gb = np.flip(gapsf, ax)
    H, W = mask.shape
    d = np.abs(back - out).reshape(H // B, B, W // B, B).max(axis=(1, 3))
    ok = (gaps > 1e-9) & (gb > 1e-9)
    assert ok.mean() > 0.9
    assert d[ok].max() < 1e-8


def test_recursion_pairs_each_reference_with_its_own_frame(monkeypatch):
    """reconstruct_sequence gives frame t, as the reference of lag k+1, the
    uint8 reconstruction of frame t-1-k together with the measured frame and
    the mask of that same frame, k = 0 .. min(t, 3) - 1."""
    rng = np.random.default_rng(3)
    n, H, W = 6, 24, 24
    frames, _ = synth.video_translate_edges(n, H, W, rng, max_step=1, n_edges=2)
    masks = synth.mask_sequence("dynamic", n, H, W, rng)
    meas = synth.measured(frames, masks)
    seen = []
    real = OF.reconstruct_frame

    def spy(cur, cur_mask, refs, me, fsr, track_gaps=True):
        res = real(cur, cur_mask, refs, me, fsr, track_gaps)
        seen.append((cur, refs, res))
        return res

    monkeypatch.setattr(OF, "reconstruct_frame", spy)
    res = O.reconstruct_sequence(meas, masks, O.MEParams(search=2, check="nnc_frmc"), O.FSRParams(iters=8))
    assert len(seen) == n
    for t, (cur, refs, r) in enumerate(seen):
        assert cur is meas[t] or np.array_equal(cur, meas[t])
        assert r is res[t]
        assert len(refs) == min(t, 3)
        for k, (recon, rmeas, rmask) in enumerate(refs):
            assert recon is res[t - 1 - k]["out_u8"], (t, k)
            assert np.array_equal(rmeas, meas[t - 1 - k]), (t, k)
            assert np.array_equal(rmask, masks[t - 1 - k]), (t, k)
