"""GPU PSNR / mean SSIM (rfsr_quality) against the oracle's definitions."""
import numpy as np
import pytest
import torch

import oracle as O
from _gpu import need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W,border,pitch", [(128, 128, 40, 128), (97, 61, 0, 64), (240, 320, 40, 336),
                                              (11, 11, 0, 11), (1080, 1920, 40, 1920)])
def test_quality_matches_oracle(H, W, border, pitch):
    R = need_gpu()
    rng = np.random.default_rng(H * 7 + W)
    ref = rng.integers(0, 256, (H, W)).astype(np.uint8)
    test = (ref.astype(np.float64) + rng.normal(0, 9, (H, W))).astype(np.float32)
    test[rng.random((H, W)) < 0.01] = 300.0        # clipped by both sides
    test[rng.random((H, W)) < 0.01] = -20.0
    r_d = torch.zeros((H, pitch), dtype=torch.uint8, device="cuda")[:, :W]
    t_d = torch.zeros((H, pitch), dtype=torch.float32, device="cuda")[:, :W]
    r_d.copy_(torch.from_numpy(ref))
    t_d.copy_(torch.from_numpy(test))
    p, s = R.quality(r_d, t_d, border)
    p_o = O.psnr(ref, test, border)
    s_o = O.ssim(ref, test, border)
    print(f"{H}x{W} border {border}: psnr {p:.9f} / {p_o:.9f}, ssim {s:.12f} / {s_o:.12f}")
    assert p == pytest.approx(p_o, abs=1e-9)
    assert s == pytest.approx(s_o, abs=1e-10)


def test_quality_identical_is_infinite_psnr_and_unit_ssim():
    R = need_gpu()
    x = torch.randint(0, 256, (64, 64), dtype=torch.uint8, device="cuda")
    p, s = R.quality(x, x.float(), 0)
    assert p == float("inf")
    assert s == pytest.approx(1.0, abs=1e-12)
