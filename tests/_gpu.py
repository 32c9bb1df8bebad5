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
# The FSR forms held to the float64 model (tolerance FSR_TOL under TAU_FP64):
# float64 throughout, and float32 with float64 for the blocks whose picks
# float32 cannot vouch for.
FLOAT64_FORMS = ("fp64", "mixed")
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


def check_support_fields(cur, mask, recon, alpha, beta, accept, cost, blocks, search, pad=16):
    """For each listed FSR block, recompute with the oracle on a crop around
    its 32x32 support (plus `pad` rows and columns, more than the reach of
    forward ME feeding the NNC medians and of FRMC, so the crop's own edges do
    not matter inside the support) the forward vectors and costs on the
    support grown by 2 pixels, and the NNC -> FRMC decisions on the support,
    and assert that the GPU's full-frame planes equal them there.  Returns the
    number of support pixels checked."""
    import oracle as O
    H, W = cur.shape
    checked = 0
    for bi, bj in blocks:
        sy0, sx0 = max(0, 4 * bi - 14), max(0, 4 * bj - 14)
        sy1, sx1 = min(H, 4 * bi + 18), min(W, 4 * bj + 18)
        cy0, cx0 = max(0, sy0 - 2 - pad), max(0, sx0 - 2 - pad)
        cy1, cx1 = min(H, sy1 + 2 + pad), min(W, sx1 + 2 + pad)
        crop = (slice(cy0, cy1), slice(cx0, cx1))
        a, b, S, _ = O.forward_me(cur[crop], mask[crop], recon[crop], search)
        g = (slice(max(0, sy0 - 2) - cy0, min(H, sy1 + 2) - cy0), slice(max(0, sx0 - 2) - cx0, min(W, sx1 + 2) - cx0))
        gf = (slice(max(0, sy0 - 2), min(H, sy1 + 2)), slice(max(0, sx0 - 2), min(W, sx1 + 2)))
        assert np.array_equal(a[g], alpha[gf]) and np.array_equal(b[g], beta[gf]), (bi, bj)
        assert np.array_equal(S[g], cost[gf]), (bi, bj)
        acc, _ = O.motion_check("nnc_frmc", cur[crop], mask[crop], recon[crop], a, b, search)
        sup = (slice(sy0 - cy0, sy1 - cy0), slice(sx0 - cx0, sx1 - cx0))
        assert np.array_equal(acc[sup], accept[sy0:sy1, sx0:sx1]), (bi, bj)
        checked += (sy1 - sy0) * (sx1 - sx0)
    return checked
