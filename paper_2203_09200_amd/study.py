"""Quality study on synthetic video: the method grid of the paper's Tables 1
and 2 (single-frame FSR; D-FSR with RME, RMC, FRMC and the NNC -> FRMC
cascade; R-FSR with RME) for the fixed and the dynamic quarter mask, and the
frame-wise gain of the recursion over single-frame FSR (the analogue of
Fig. 4), with PSNR and mean SSIM as in Sec. 4 (40-pixel border omitted).

The paper's sequences are not available; `--sequences` synthetic sequences
of `--size` stand in for them (the 1080p generator: smooth texture, 8x8
translating regions, occluders).  All sequences of one (method, mask) run
advance together as one batch per time step (`StreamSet`), and PSNR / SSIM
are computed on the device (`rfsr_quality`).

    python -m paper_2203_09200_amd.study [--size 832x480] [--frames 50] [--sequences 8]

prints one JSON line (per method and mask: mean PSNR, mean SSIM, mean over
frames 3.. ("steady"), and the per-frame PSNR gain over FSR averaged over
the sequences).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METHODS = [
    # (name, check, overwrite, references)
    ("FSR", "none", "dfsr", 0),
    ("R-FSR+RME", "rme", "rfsr", 3),
    ("D-FSR+RME", "rme", "dfsr", 3),
    ("D-FSR+RMC", "rmc", "dfsr", 3),
    ("D-FSR+FRMC", "frmc", "dfsr", 3),
    ("D-FSR+NNC+FRMC", "nnc_frmc", "dfsr", 3),
]


def run(sequences, method, kind_masks, R, torch, dev, search=9, iters=100, precision="fp64", concealed=0.0,
        prior=0.0, stop=0.0):
    """Per-frame (psnr, ssim) arrays (n_seq, T) of one method on the given
    sequences (uint8 frames (T, H, W) each) with their masks."""
    import numpy as np
    name, check, overwrite, nref = method
    T = sequences[0].shape[0]
    sizes = [tuple(f.shape[1:]) for f in sequences]
    me = R.MEParams(search=search, check=check if nref else "none")
    fsr = R.FSRParams(iters=iters, overwrite=overwrite, precision=precision, concealed_weight=concealed,
                      prior_sigma=prior, stop_ratio=stop)
    ss = R.StreamSet(sizes, me, fsr, nref=nref, graphs=True, device=dev)
    gt = [[torch.from_numpy(f[t]).to(dev) for t in range(T)] for f in sequences]
    meas = [[torch.from_numpy(f[t] * m[t]).to(dev) for t in range(T)] for f, m in zip(sequences, kind_masks)]
    masks = [[torch.from_numpy(m[t]).to(dev) for t in range(T)] for m in kind_masks]
    res = torch.empty((len(sequences), T, 2), dtype=torch.float64, device=dev)
    for t in range(T):
        outs = ss.step([q[t] for q in meas], [q[t] for q in masks])
        for s, (o, _) in enumerate(outs):
            R.quality_async(gt[s][t], o, 40, result=res[s, t])
    r = res.cpu().numpy()
    return r[..., 0], r[..., 1]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--size", default="832x480", help="WxH")
    ap.add_argument("--frames", type=int, default=50)
    ap.add_argument("--sequences", type=int, default=8)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--search", type=int, default=9)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--concealed", type=float, default=0.0, help="concealed weighting delta")
    ap.add_argument("--prior", type=float, default=0.0, help="FSR frequency-weighting prior sigma (0: off)")
    ap.add_argument("--stop", type=float, default=0.0, help="FSR residual-energy early-stop ratio (0: off)")
    a = ap.parse_args(argv)

    import numpy as np
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    from . import _lib as R

    if not torch.cuda.is_available():
        print("study: no GPU visible", file=sys.stderr)
        return 1
    R.lib()
    dev = torch.device("cuda:0")
    W, H = (int(x) for x in a.size.lower().split("x"))
    log = lambda m: print(f"# {m}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    seqs, masks = [], {"fixed": [], "dynamic": []}
    for s in range(a.sequences):
        rng = np.random.default_rng(synth.seed_for(6, s))
        f = synth.video_regions(a.frames, H, W, rng)
        seqs.append(f)
        for kind in masks:
            masks[kind].append(synth.mask_sequence(kind, a.frames, H, W, rng))
    log(f"{a.sequences} sequences of {a.frames} frames {W}x{H} generated in {time.perf_counter() - t0:.1f} s")

    out = {"study": "quality grid on synthetic video (Tables 1-2 / Fig. 4 analogue)", "size": f"{W}x{H}",
           "frames": a.frames, "sequences": a.sequences, "iters": a.iters, "search": a.search,
           "precision": a.precision, "concealed": a.concealed, "prior": a.prior, "stop": a.stop, "results": {}}
    for kind in ("fixed", "dynamic"):
        base = None
        for method in METHODS:
            t1 = time.perf_counter()
            p, s = run(seqs, method, masks[kind], R, torch, dev, a.search, a.iters, a.precision, a.concealed,
                       a.prior, a.stop)
            if method[0] == "FSR":
                base = p
            gain = (p - base).mean(axis=0)
            out["results"].setdefault(kind, {})[method[0]] = {
                "psnr": round(float(p.mean()), 3), "ssim": round(float(s.mean()), 4),
                "psnr_steady": round(float(p[:, 3:].mean()), 3), "ssim_steady": round(float(s[:, 3:].mean()), 4),
                "gain_per_frame": [round(float(g), 3) for g in gain]}
            log(f"{kind:7s} {method[0]:15s}: PSNR {p.mean():.3f} dB  SSIM {s.mean():.4f}  "
                f"({time.perf_counter() - t1:.1f} s)")
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
