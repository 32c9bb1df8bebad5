"""Helpers shared by the GPU parity tests (marked `gpu`)."""
import numpy as np
import pytest
import torch

# Relative energy gap below which an FSR block is tie-ambiguous (the greedy
# argmax then has several correct answers).  The float64 kernel and the
# float64 oracle differ by rounding of about 1e-13 relative (the packed row
# code resolves 2^-47), so for them a gap of 1e-10 already decides; the
# float32 forms and the 16-bit split DFTs carry float32 rounding.
TAU_FP64 = 1e-10
TAU_FP32 = 1e-5
AMB_MAX = 0.005      # share of blocks that may be tie-ambiguous under TAU_FP64
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


def compare_fsr(gpu_out, ora_out, gaps, B=4, tol=FSR_TOL, tau=TAU_FP64):
    """Blockwise comparison under the near-tie rule: blocks whose oracle
    energy gap is below tau are excluded from the max-abs check (counted).
    Returns (max_abs over unambiguous blocks, n_ambiguous, n_blocks)."""
    H, W = ora_out.shape
    d = np.abs(gpu_out.astype(np.float64) - ora_out).reshape(H // B, B, W // B, B).max(axis=(1, 3))
    amb = gaps < tau
    worst = d[~amb].max() if (~amb).any() else 0.0
    return float(worst), int(amb.sum()), int(amb.size)
