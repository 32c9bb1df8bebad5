"""Precision study of the block DFT on the matrix cores: FSR with the DFT as
two 32x32 GEMM stages in bfloat16 / float16 split operands (hi*hi + hi*lo +
lo*hi, float32 accumulation) against the float64 FFT path and the float64
oracle, at 100 and 300 iterations, on the 3840x2160 workload (seeded sample
of blocks) and on a full 128x128 frame (PSNR).  The iterations are float64 in
every variant, so the differences measure the DFT alone.  The plain float32
form (every step float32) is measured beside them."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import FSR_TOL, TAU_FP32, TAU_FP64, dev, host, need_gpu

pytestmark = pytest.mark.gpu

PRECS = ("fp64", "bf16x3", "fp16x3", "fp32")


def block_errors(out, ora, blocks):
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    return np.abs(got.astype(np.float64) - ora).max(axis=(1, 2))


@pytest.fixture(scope="module")
def frame4k():
    f, m = synth.workload_c2(n=1, h=2160, w=3840, seed=synth.seed_for(3))
    return f[0], m[0], synth.measured(f, m)[0]


@pytest.mark.parametrize("K", [100, 300])
def test_mfma_dft_against_oracle_4k_sample(frame4k, K):
    R = need_gpu()
    f, m, meas = frame4k
    H, W = m.shape
    vals = meas.astype(np.float64)
    rng = np.random.default_rng(1000 + K)
    nb = 256
    blocks = np.stack([rng.integers(0, H // 4, nb), rng.integers(0, W // 4, nb)], axis=1)
    ora, gaps = O.fsr.fsr_blocks_out(vals, m, blocks, K=K)
    v_d, m_d = dev(vals, torch.float32), dev(m)
    res = {}
    for p in PRECS:
        # the float64 kernel is held to the float64 near-tie threshold, the
        # forms with float32 rounding (accumulation or residual) to the float32 one
        amb = gaps < (TAU_FP64 if p == "fp64" else TAU_FP32)
        out, _ = R.fsr_blocks(v_d, m_d, R.FSRParams(iters=K, precision=p))
        d = block_errors(host(out), ora, blocks)
        res[p] = (d, amb)
        print(f"4K K={K} {p:7s}: max {d[~amb].max():.2e}  median {np.median(d[~amb]):.2e}  "
              f"blocks > 1e-3: {(d[~amb] > 1e-3).mean() * 100:.1f} %  (ambiguous {amb.sum()}/{nb})")
    d, amb = res["fp64"]
    assert d[~amb].max() <= FSR_TOL and amb.sum() == 0
    # measured shares of unambiguous sampled blocks beyond 1e-3 (K = 100 / 300):
    # fp16x3 0 % / 1.6 %, bf16x3 5.9 % / 32.9 %, fp32 0 % / 0.4 %; the bounds
    # allow about twice that
    bound = {100: {"fp16x3": 0.0, "bf16x3": 0.12, "fp32": 0.01},
             300: {"fp16x3": 0.04, "bf16x3": 0.50, "fp32": 0.02}}[K]
    for p in PRECS[1:]:
        d, amb = res[p]
        assert np.isfinite(d).all()
        assert (d[~amb] > 1e-3).mean() <= bound[p], p
        assert np.median(d[~amb]) < 1e-3, p


@pytest.mark.parametrize("K", [100, 300])
def test_mfma_dft_full_frame_psnr(K):
    R = need_gpu()
    f, m = synth.workload_c2(n=1, h=128, w=128, seed=77)
    meas = synth.measured(f, m)[0]
    vals = meas.astype(np.float64)
    ora, _ = O.fsr_frame(vals, m[0], K=K)
    p_ora = O.psnr(f[0], ora, 8)
    v_d, m_d = dev(vals, torch.float32), dev(m[0])
    for p in PRECS:
        out, _ = R.fsr_blocks(v_d, m_d, R.FSRParams(iters=K, precision=p))
        out = host(out)
        d = np.abs(out - ora)
        dp = O.psnr(f[0], out, 8) - p_ora
        print(f"128x128 K={K} {p:7s}: max-abs {d.max():.3e}  PSNR {p_ora + dp:.4f} dB (delta {dp:+.4f})")
        # measured |delta| at most 0.016 dB (bf16x3, K = 300)
        assert abs(dp) <= (0.01 if p == "fp64" else 0.05), p


def test_mfma_dft_timing_1080p():
    """FSR kernel time per 1080p frame for each DFT precision (reported)."""
    R = need_gpu()
    f, m = synth.workload_c2(n=1)
    meas = synth.measured(f, m)[0]
    v_d, m_d = dev(meas, torch.float32), dev(m[0])
    for p in PRECS:
        prm = R.FSRParams(iters=100, precision=p)
        R.fsr_blocks(v_d, m_d, prm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            R.fsr_blocks(v_d, m_d, prm)
        e1.record()
        torch.cuda.synchronize()
        print(f"1080p K=100 {p:7s}: {e0.elapsed_time(e1) / 3:.3f} ms per frame")
