"""Oracle (test infrastructure only): one recursive frame in the order of
Fig. 1 (ME -> consistency check -> projection -> FSR), the causal recursion
over a sequence (three previous frames, Sec. 4), and PSNR (Sec. 4: per
frame, a 40-pixel border omitted).

Readings: the reconstruction handed to later frames as their reference is
rint(clip(out, 0, 255)) as uint8 (round half to even); PSNR clips the float
output to [0, 255] without rounding.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .me import forward_me
from .checks import motion_check
from .projection import project
from .fsr import fsr_frame, fsr_frame_concealed


@dataclass
class MEParams:
    tmpl: int = 4
    search: int = 9
    check: str = "nnc_frmc"
    rmc_radius: int | None = None
    frmc: tuple | None = None         # per-axis FRMC offsets (None: {-7,-3,-1,0,1,3,7})
    cost_norm: bool = True            # reverse costs compared as S/n (False: raw S)
    nnc_center: str = "filtered"      # NNC compares the filtered ("filtered") or raw ("raw") vector at p


@dataclass
class FSRParams:
    block: int = 4
    support: int = 32
    iters: int = 100
    rho: float = 0.7
    gamma: float = 0.5
    proj_weight: float = 1.0
    overwrite: str = "dfsr"
    concealed_weight: float = 0.0     # delta; > 0: blocks in raster order (fsr_frame_concealed)
    prior_sigma: float = 0.0          # frequency-weighting prior (0: off), fsr.prior_table
    stop_ratio: float = 0.0           # residual-energy early stop (0: off)


def quantize(out):
    return np.rint(np.clip(out, 0.0, 255.0)).astype(np.uint8)


def psnr(ref, test, border=40):
    ref = np.asarray(ref, np.float64)
    test = np.clip(np.asarray(test, np.float64), 0.0, 255.0)
    H, W = ref.shape
    sl = (slice(border, H - border), slice(border, W - border))
    mse = np.mean((ref[sl] - test[sl]) ** 2)
    return np.inf if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def motion_fields(cur, cur_mask, refs, me: MEParams):
    """Forward ME and the check for each reference (lag 1..len(refs))."""
    fields = []
    for recon, meas, mask in refs:
        a, b, S, n = forward_me(cur, cur_mask, recon, me.search, me.tmpl)
        acc, ev = motion_check(me.check, cur, cur_mask, recon, a, b, me.search, me.tmpl,
                               me.rmc_radius, me.frmc, me.cost_norm, me.nnc_center)
        fields.append(dict(alpha=a, beta=b, S=S, n=n, accept=acc, evals=ev,
                           meas=meas, mask=mask))
    return fields


def reconstruct_frame(cur, cur_mask, refs, me: MEParams, fsr: FSRParams, track_gaps=True):
    """refs: list of (recon uint8, meas uint8, mask uint8) for lags 1..nref."""
    fields = motion_fields(cur, cur_mask, refs, me)
    values, cls = project(cur, cur_mask, fields)
    if fsr.concealed_weight > 0:
        if fsr.prior_sigma > 0 or fsr.stop_ratio > 0:
            raise ValueError("the prior and the early stop are not combined with concealed weighting")
        out, gaps = fsr_frame_concealed(values, cls, fsr.concealed_weight, fsr.block, fsr.support,
                                        fsr.rho, fsr.gamma, fsr.iters, fsr.proj_weight, fsr.overwrite)
    else:
        out, gaps = fsr_frame(values, cls, fsr.block, fsr.support, fsr.rho, fsr.gamma,
                              fsr.iters, fsr.proj_weight, fsr.overwrite, track_gaps,
                              prior_sigma=fsr.prior_sigma, stop_ratio=fsr.stop_ratio)
    return dict(out=out, out_u8=quantize(out), values=values, cls=cls, fields=fields,
                gaps=gaps)


def reconstruct_sequence(meas, masks, me: MEParams, fsr: FSRParams, nref=3,
                         track_gaps=False):
    """Causal recursion: frame t uses the reconstructions of t-1..t-nref."""
    ring = []
    results = []
    for t in range(meas.shape[0]):
        refs = [(r["out_u8"], meas[t - 1 - k], masks[t - 1 - k]) for k, r in
                enumerate(reversed(ring[-nref:]))] if ring else []
        res = reconstruct_frame(meas[t], masks[t], refs, me, fsr, track_gaps)
        results.append(res)
        ring.append(res)
    return results
