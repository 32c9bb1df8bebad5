"""Real-valued (conjugate-pair) FSR on the GPU against the oracle's pair
loop, and its quality and speed beside the complex single-bin loop."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _gpu import FSR_TOL, PSNR_TOL, AMB_MAX, TAU_FP64, dev, host, need_gpu

pytestmark = pytest.mark.gpu


def frame(H, W, seed, proj=0.15):
    rng = np.random.default_rng(seed)
    f, m = synth.workload_c2(n=1, h=H, w=W, seed=seed)
    cls = m[0].astype(np.uint8)
    cls[(cls == 0) & (rng.random((H, W)) < proj)] = 2
    vals = np.where(cls > 0, f[0].astype(np.float64) + (cls == 2) * rng.normal(0, 3, (H, W)), 0.0)
    return f[0], vals.astype(np.float32).astype(np.float64), cls


@pytest.mark.parametrize("K,overwrite", [(30, "dfsr"), (50, "rfsr")])
def test_pairs_full_frame_against_oracle(K, overwrite):
    R = need_gpu()
    H, W = 64, 80
    f, vals, cls = frame(H, W, 31 + K)
    out, u8 = R.fsr_blocks(dev(vals, torch.float32), dev(cls), R.FSRParams(iters=K, pairs=True, overwrite=overwrite))
    out = host(out)
    ora, gaps = O.fsr_pairs_blocks_out(vals, cls, O.fsr.all_blocks(H, W), K=K, overwrite=overwrite)
    ora = ora.reshape(H // 4, W // 4, 4, 4).transpose(0, 2, 1, 3).reshape(H, W)
    d = np.abs(out - ora).reshape(H // 4, 4, W // 4, 4).max(axis=(1, 3))
    amb = gaps.reshape(H // 4, W // 4) < TAU_FP64
    print(f"pairs {H}x{W} K={K}: max {d[~amb].max():.2e}, ambiguous {amb.sum()}/{amb.size}")
    assert d[~amb].max() <= FSR_TOL
    assert amb.sum() <= AMB_MAX * amb.size
    assert abs(O.psnr(f, out, 8) - O.psnr(f, ora, 8)) <= PSNR_TOL
    assert (host(u8) == O.quantize(out)).all()


def test_pairs_4k_sample_against_oracle():
    R = need_gpu()
    f, m = synth.workload_c2(n=1, h=2160, w=3840, seed=synth.seed_for(3))
    vals = synth.measured(f, m)[0].astype(np.float64)
    out, _ = R.fsr_blocks(dev(vals, torch.float32), dev(m[0]), R.FSRParams(iters=50, pairs=True))
    out = host(out)
    rng = np.random.default_rng(50)
    blocks = np.stack([rng.integers(0, 540, 256), rng.integers(0, 960, 256)], axis=1)
    ora, gaps = O.fsr_pairs_blocks_out(vals, m[0], blocks, K=50)
    got = np.stack([out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] for bi, bj in blocks])
    d = np.abs(got - ora).max(axis=(1, 2))
    amb = gaps < TAU_FP64
    print(f"pairs 4K K=50: max {d[~amb].max():.2e}, ambiguous {amb.sum()}/256")
    assert d[~amb].max() <= FSR_TOL


def test_pairs_quality_and_speed_beside_complex():
    """Reported: PSNR of K/2 pair iterations against K complex ones (same
    number of basis functions), and FSR time per 1080p frame."""
    R = need_gpu()
    f, m = synth.workload_c2(n=1)
    meas = synth.measured(f, m)[0]
    v_d, m_d = dev(meas, torch.float32), dev(m[0])
    res = {}
    for name, prm in (("complex K=100", R.FSRParams(iters=100)), ("pairs K=50", R.FSRParams(iters=50, pairs=True)),
                      ("pairs K=100", R.FSRParams(iters=100, pairs=True))):
        out, _ = R.fsr_blocks(v_d, m_d, prm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            R.fsr_blocks(v_d, m_d, prm)
        e1.record()
        torch.cuda.synchronize()
        p = O.psnr(f[0], host(out))
        res[name] = p
        print(f"1080p {name:14s}: {e0.elapsed_time(e1) / 3:.3f} ms, PSNR {p:.3f} dB")
    assert abs(res["pairs K=50"] - res["complex K=100"]) < 0.5
