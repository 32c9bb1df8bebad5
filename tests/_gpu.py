"""Helpers shared by the GPU parity tests (marked `gpu`)."""
import numpy as np
import pytest
import torch

TAU_FP32 = 1e-5      # relative energy gap below which an FSR block is tie-ambiguous in FP32
FSR_TOL = 1e-3       # max-abs tolerance of FSR outputs on the 0..255 scale
PSNR_TOL = 0.01      # dB


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_09200_amd as R
    R.lib()          # raises if librfsr.so is missing: no silent fallback
    return R


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def compare_fsr(gpu_out, ora_out, gaps, B=4, tol=FSR_TOL, tau=TAU_FP32):
    """Blockwise comparison under the near-tie rule: blocks whose oracle
    energy gap is below tau are excluded from the max-abs check (counted).
    Returns (max_abs over unambiguous blocks, n_ambiguous, n_blocks)."""
    H, W = ora_out.shape
    d = np.abs(gpu_out.astype(np.float64) - ora_out).reshape(H // B, B, W // B, B).max(axis=(1, 3))
    amb = gaps < tau
    worst = d[~amb].max() if (~amb).any() else 0.0
    return float(worst), int(amb.sum()), int(amb.size)
