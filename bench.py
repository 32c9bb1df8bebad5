#!/usr/bin/env python3
"""Throughput of the recursive D-FSR hot path on one MI355X.

Workload (the metric's configuration): 1920x1080 uint8 synthetic video, 16
frames, dynamic quarter-sampling mask, D-FSR with the NNC -> FRMC cascade,
search radius 9, 4x4 templates, FSR with 4x4 blocks, 32x32 supports,
rho = 0.7, gamma = 0.5, 100 iterations, three reference frames.

One step = the causal recursion over the 16-frame sequence (every frame runs
ME + check against up to three references, projection, FSR, overwrite and
quantisation on the GPU).  Inputs are resident in HBM before timing.
Consecutive frames are pipelined (results unchanged): the motion path of a
frame's lag-2 and lag-3 references runs on a side stream during the previous
frame's FSR (--no-pipeline: one frame after the other).

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]

Prints one JSON line: HR megapixels per second, per-frame latency
percentiles, per-stage times, the FSR kernel's roofline position and the CPU
oracle's throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def fsr_flops_per_block(K: int, pairs: bool = False) -> int:
    """Algorithmic flops of one FSR block:
    complex bins: K iterations x 1024 bins x 11 (complex multiply-subtract 8,
    energy 3); conjugate pairs: K x 513 independent bins x 19 (two complex
    multiply-subtracts, energy); one 32x32 complex FFT (5 N log2 N,
    N = 1024); synthesis K x 16 x 4."""
    it = 19 * 513 * K if pairs else 11 * 1024 * K
    return it + 5 * 1024 * 10 + 64 * K


def psnr(ref, test, border=40):
    """PSNR of a reconstruction against the ground-truth frame on the 0..255
    scale, clamped, without a `border`-pixel frame (quality report only)."""
    import numpy as np
    ref = np.asarray(ref, np.float64)
    test = np.clip(np.asarray(test, np.float64), 0.0, 255.0)
    H, W = ref.shape
    sl = (slice(border, H - border), slice(border, W - border))
    mse = np.mean((ref[sl] - test[sl]) ** 2)
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


FORM_SUFFIX = {"fp64": "", "fp32": ", FSR all float32", "mixed": ", FSR float32 with float64 for near-tie blocks"}


def dtype_of(precision):
    """The arithmetic type the FSR path computes in, per precision option."""
    return {"fp64": "f64", "fp32": "f32", "mixed": "f32 (f64 for near-tie blocks)"}.get(
        precision, f"f64 (block DFT {precision}, float32 accumulate)")


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def counters_from_profile(precision="fp64"):
    """The committed PMC record of one 1080p FSR launch in the given form (HBM
    bytes and VALU wave-instructions; for mixed, the float32 pass and the
    float64 recomputation together), or {} when there is none or the kernels'
    sources changed since the counters were taken."""
    from paper_2203_09200_amd.profiling import FORMS, kernel_digest
    if precision not in FORMS:
        return {}
    path = os.path.join(ROOT, "profiles", FORMS[precision]["record"])
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha256") != kernel_digest(precision):
        return {}
    return rec


# ------------------------------------------------------------ CPU baseline --
# The oracle timed on the host cores: a band of rows of one frame of the
# workload.  The motion path (forward ME and the check, per reference) runs on
# column strips of the rows whose decisions the band's FSR supports read, the
# projection in this process, FSR on tiles of blocks; each strip or tile is a
# task of a process pool.  A strip is computed on a crop with `halo` pixels of
# margin wherever the crop edge is not the frame's: around a pixel the oracle
# reads within 2R + 2 (reverse ME), R + 4 (forward ME feeding the NNC medians),
# the largest check offset + 2 (RMC, FRMC) or 14 (an FSR support) pixels, so
# every kept pixel equals the whole-frame oracle's (tests/test_bench_host.py
# checks this).


def oracle_halo(me_o):
    """Margin of a motion crop that leaves its kept pixels as in the whole frame."""
    rr = me_o.rmc_radius or 0
    offs = max((abs(d) for d in me_o.frmc), default=0) if me_o.frmc is not None else 7
    return max(2 * me_o.search, rr, offs, 14) + 4


def _crop(n, a, b, halo):
    return max(0, a - halo), min(n, b + halo)


def _oracle_motion_task(args):
    """Forward ME + check of one reference on a crop; returns the kept pixels."""
    from oracle.frame import motion_fields
    cur, mask, recon, ky, kx, me = args
    f = motion_fields(cur, mask, [(recon, None, None)], me)[0]
    return f["alpha"][ky, kx], f["beta"][ky, kx], f["accept"][ky, kx]


def _oracle_fsr_task(args):
    """FSR of the block rows [bi0, bi1) x columns [bj0, bj1) of a crop whose
    origin is block (cb, cj)."""
    import numpy as np
    import oracle as O
    values, cls, cb, cj, bi0, bi1, bj0, bj1, fsr = args
    bi, bj = np.mgrid[bi0 - cb:bi1 - cb, bj0 - cj:bj1 - cj]
    blocks = np.stack([bi.ravel(), bj.ravel()], axis=1)
    out, _ = O.fsr.fsr_blocks_out(values, cls, blocks, fsr.block, fsr.support, fsr.rho, fsr.gamma,
                                  fsr.iters, fsr.proj_weight, fsr.overwrite, track_gaps=False)
    return out


def oracle_frame_rows(pool, cur, cur_mask, refs, me_o, fsr_o, y0, y1, strips=8, halo=None):
    """The oracle's reconstruction of rows [y0, y1) of one frame (multiples of
    4), computed as tasks on `pool`: per reference `strips` column strips of
    the motion path (crops with `halo` pixels of margin, default
    oracle_halo), then FSR on `strips` x (rows / 4) tiles of blocks.
    refs: [(recon, meas, mask)] for lags 1..nref (full frames).  Returns
    out[y0:y1] (float64)."""
    import numpy as np
    import oracle as O
    H, W = cur.shape
    halo = oracle_halo(me_o) if halo is None else halo
    m0, m1 = max(0, y0 - 16), min(H, y1 + 16)          # rows whose decisions feed the blocks' supports
    cy0, cy1 = _crop(H, m0, m1, halo)
    edges = [(W * i // strips) & ~3 for i in range(strips)] + [W]
    tasks, where = [], []
    for k, (recon, _, _) in enumerate(refs):
        for x0, x1 in zip(edges[:-1], edges[1:]):
            if x1 <= x0:
                continue
            cx0, cx1 = _crop(W, x0, x1, halo)
            crop = (slice(cy0, cy1), slice(cx0, cx1))
            keep = (slice(m0 - cy0, m1 - cy0), slice(x0 - cx0, x1 - cx0))
            tasks.append((cur[crop], cur_mask[crop], recon[crop], keep[0], keep[1], me_o))
            where.append((k, x0, x1))
    fields = [dict(alpha=np.zeros((H, W), np.int64), beta=np.zeros((H, W), np.int64),
                   accept=np.zeros((H, W), bool), meas=meas, mask=mask) for _, meas, mask in refs]
    for (k, x0, x1), (a, b, acc) in zip(where, pool.map(_oracle_motion_task, tasks)):
        f = fields[k]
        f["alpha"][m0:m1, x0:x1], f["beta"][m0:m1, x0:x1], f["accept"][m0:m1, x0:x1] = a, b, acc
    values, cls = O.project(cur, cur_mask, fields)
    tasks, where = [], []
    for r0 in range(y0, y1, 4):
        for x0, x1 in zip(edges[:-1], edges[1:]):
            if x1 <= x0:
                continue
            ry0, ry1 = _crop(H, r0, r0 + 4, 16)
            rx0, rx1 = _crop(W, x0, x1, 16)
            tasks.append((values[ry0:ry1, rx0:rx1], cls[ry0:ry1, rx0:rx1], ry0 // 4, rx0 // 4,
                          r0 // 4, r0 // 4 + 1, x0 // 4, x1 // 4, fsr_o))
            where.append((r0, x0, x1))
    out = np.zeros((y1 - y0, W))
    for (r0, x0, x1), ob in zip(where, pool.map(_oracle_fsr_task, tasks)):
        out[r0 - y0:r0 - y0 + 4, x0:x1] = ob.transpose(1, 0, 2).reshape(4, x1 - x0)
    return out


def cpu_cores():
    """Host cores for the oracle: this process's CPU affinity, at most 16
    (one GPU's share of the host)."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def cpu_baseline(pool, cores, frames, masks, recons, me_o, fsr_o, rows_per_core=8):
    """The oracle (float64 FSR, integer ME) on frame 3 of the workload with
    the GPU's reconstructions of frames 0..2 as its references, on a band of
    `rows_per_core` rows per process (full width) in the middle of the frame."""
    import synth
    H, W = frames.shape[1:]
    rows = min(H, rows_per_core * cores) & ~3
    y0 = ((H - rows) // 2) & ~3
    meas = synth.measured(frames[:4], masks[:4])
    refs = [(recons[3 - k], meas[3 - k], masks[3 - k]) for k in (1, 2, 3)]
    strips = max(1, cores // 2)
    t0 = time.perf_counter()
    oracle_frame_rows(pool, meas[3], masks[3], refs, me_o, fsr_o, y0, y0 + rows, strips=strips)
    dt = time.perf_counter() - t0
    return {"value": round(rows * W / dt / 1e6, 6), "unit": "HR Mpix/s", "cores": cores,
            "kind": "oracle",
            "sample": f"frame 3, rows {y0}..{y0 + rows - 1} ({W}x{rows}; three references = the GPU's "
                      f"uint8 reconstructions of frames 0-2), {cores} processes: motion path on {strips} column "
                      f"strips per reference, FSR on block tiles; {dt:.1f} s"}


def other_form(a, precision, pipelined, seq_args, d_meas, d_mask, frames, ref_out, stream, form):
    """The same recursion with FSR in another arithmetic form, reported beside
    the headline: one untimed and one timed step of the sequence.  Reports
    throughput, PSNR and the distance of its outputs from the headline's."""
    import numpy as np
    import torch
    import paper_2203_09200_amd as R
    H, W, me, dev = seq_args
    F = len(d_meas)
    prm = R.FSRParams(iters=a.iters, precision=precision)
    seq = R.Sequence(H, W, me, prm, device=dev, pipelined=pipelined)
    outs = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(F)]

    def step():
        seq.reset()
        for t in range(F):
            seq.push(d_meas[t], d_mask[t], stream=stream, out=outs[t])

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    got = [o.cpu().numpy() for o in outs]
    d = np.concatenate([np.abs(g.astype(np.float64) - r).ravel() for g, r in zip(got, ref_out)])
    # frame 0 has no references: both forms run FSR on the same input
    d0 = np.abs(got[0].astype(np.float64) - ref_out[0]).reshape(H // 4, 4, W // 4, 4).max(axis=(1, 3))
    return {"value": round(F * H * W / dt / 1e6, 3), "unit": "HR Mpix/s", "ms_per_step": round(dt * 1e3, 3),
            "psnr_db": round(float(np.mean([psnr(frames[t], got[t]) for t in range(F)])), 3),
            "max_abs_vs_headline": round(float(d.max()), 4),
            "frac_px_over_1e-3_vs_headline": round(float((d > 1e-3).mean()), 5),
            "frame0_blocks_within_1e-3_of_headline": round(float((d0 <= 1e-3).mean()), 5),
            "frame0_max_abs_vs_headline": float(f"{d0.max():.4g}"),
            "form": form + ("; pipelined as the headline" if pipelined else
                            "; single stream, one frame at a time") + "; one timed step"}


def run_multistream(a, dev):
    """48 streams of uneven size (16 x 352x288, 16 x 1280x720, 12 x 1920x1080,
    4 x 3840x2160; even streams fixed mask, odd dynamic), 8 frames each,
    cycled.  One step = one time step of every stream as ONE batch; by
    default consecutive steps are pipelined (the lag-2/3 motion path of every
    stream beside the previous step's FSR, rfsr_reconstruct_batch_part);
    --no-pipeline: whole steps (rfsr_reconstruct_batch), replayed from a
    captured graph once every stream has three references.  Inputs are
    resident in HBM; the per-step input copies into the streams' ring slots
    are inside the timed region."""
    import numpy as np
    import torch
    import synth
    import paper_2203_09200_amd as R

    T = 8
    t_gen = time.perf_counter()
    data = synth.workload_c4(n=T)
    t_gen = time.perf_counter() - t_gen
    print(f"# 48-stream workload generated in {t_gen:.1f} s", file=sys.stderr, flush=True)
    sizes = [f.shape[1:] for f, _ in data]
    meas = [[torch.from_numpy(synth.measured(f[t], m[t])).to(dev) for t in range(T)] for f, m in data]
    masks = [[torch.from_numpy(m[t]).to(dev) for t in range(T)] for _, m in data]
    me = R.MEParams(search=a.search, check=a.check)
    fsr = R.FSRParams(iters=a.iters, precision=a.precision, pairs=a.pairs, concealed_weight=a.concealed,
                      prior_sigma=a.prior, stop_ratio=a.stop)
    px_step = sum(h * w for h, w in sizes)

    pipelined = not a.no_pipeline
    ss = R.StreamSet(sizes, me, fsr, graphs=not a.no_graphs, device=dev, pipelined=pipelined)
    warm = max(a.warmup, 0) * T + 4      # every ring phase captured before timing
    for t in range(warm):
        ss.step([m[t % T] for m in meas], [m[t % T] for m in masks])
    torch.cuda.synchronize()
    print(f"# warmup: {warm} time steps", file=sys.stderr, flush=True)
    ev = [R.Event() for _ in range(a.steps + 1)]
    ev[0].record()
    t0 = time.perf_counter()
    for k in range(a.steps):
        t = ss.t
        ss.step([m[t % T] for m in meas], [m[t % T] for m in masks])
        ev[k + 1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = [ev[k].elapsed_ms(ev[k + 1]) for k in range(a.steps)]
    print(f"# timed {a.steps} time steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    t_last = (ss.t - 1) % T
    slot = (ss.t - 1) % ss.SLOTS
    psnr_mean = float(np.mean([psnr(data[s][0][t_last], ss.out[s][slot].cpu().numpy(), 8)
                               for s in range(len(sizes))]))

    plain = None
    if a.plain:
        seqs = [R.Sequence(h, w, me, fsr, device=dev) for h, w in sizes]
        for t in range(4):   # fill the rings
            for s, seq in enumerate(seqs):
                seq.push(meas[s][t % T], masks[s][t % T])
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for k in range(a.steps):
            for s, seq in enumerate(seqs):
                seq.push(meas[s][(4 + k) % T], masks[s][(4 + k) % T])
        torch.cuda.synchronize()
        pe = time.perf_counter() - p0
        plain = {"value": round(px_step * a.steps / pe / 1e6, 3), "unit": "HR Mpix/s",
                 "ms_per_step": round(pe / a.steps * 1e3, 3),
                 "form": "one frame at a time through rfsr_reconstruct_frame, no batching, no graphs"}

    res = {
        "metric": "HR Mpix/s reconstructed, 48 uneven streams per time step (batched)",
        "value": round(px_step * a.steps / elapsed / 1e6, 3),
        "unit": "HR Mpix/s",
        "n_gpus": 1, "steps": a.steps, "warmup": warm,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_of(a.precision),
        "data": "synthetic (seeded smooth texture, 8x8 translating regions, 5% occluders) per stream",
        "config": {"workload": f"48 streams (16x352x288, 16x1280x720, 12x1920x1080, 4x3840x2160), "
                               f"{T} frames cycled, even streams fixed mask / odd dynamic, D-FSR + "
                               f"{a.check.upper().replace('_', '+')}, R={a.search}, K={a.iters}, 3 references, "
                               f"one batch per time step" + (", pipelined time steps" if pipelined else
                                                             "" if a.no_graphs else ", graph replay")
                               + FORM_SUFFIX.get(a.precision, f", block DFT {a.precision}")
                               + (f", concealed weighting {a.concealed}" if a.concealed else ""),
                   "streams": len(sizes), "hr_px_per_step": px_step, "parallelism": "single GPU",
                   "pipelined": pipelined},
        "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3)},
        "psnr_db": round(psnr_mean, 3),
        "plain": plain,
    }
    print(json.dumps(res))
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--search", type=int, default=9)
    ap.add_argument("--check", default="nnc_frmc")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prior", type=float, default=0.0,
                    help="FSR frequency-weighting prior sigma (0: off; an FSR-literature option)")
    ap.add_argument("--stop", type=float, default=0.0,
                    help="FSR residual-energy early-stop ratio (0: off; an FSR-literature option)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="no overlap of consecutive frames / time steps (each frame's motion path after the "
                         "previous frame)")
    ap.add_argument("--workload", choices=["c2", "c4"], default="c2",
                    help="c2: the metric's 1080p recursion (default); c4: 48 streams of uneven "
                         "size advanced one time step per batch")
    ap.add_argument("--plain", action="store_true",
                    help="c4 only: also time the same steps one frame at a time (no batch, no graphs)")
    ap.add_argument("--no-graphs", action="store_true", help="c4 only: run batches eagerly")
    ap.add_argument("--concealed", type=float, default=0.0,
                    help="concealed weighting delta (> 0: raster-order blocks as a wavefront)")
    ap.add_argument("--pairs", action="store_true",
                    help="real-valued FSR (a conjugate pair per iteration; use about half the iterations)")
    ap.add_argument("--precision", choices=["fp64", "bf16x3", "fp16x3", "fp32", "mixed"], default="mixed",
                    help="FSR arithmetic: float32 with a near-tie test and float64 for the blocks that fail it "
                         "(mixed, default: the float64 model's result); float64 throughout (fp64); block DFT as "
                         "matrix-core GEMMs with split 16-bit operands and float64 iterations; or every step "
                         "float32 (fp32)")
    ap.add_argument("--no-other-forms", "--no-fp32-form", action="store_true",
                    help="skip the float32 (and, beside mixed, the float64) form reported beside the result")
    a = ap.parse_args(argv)

    if a.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {a.gpus} is not supported "
              "(independent streams would shard across GPUs without communication)", file=sys.stderr)
        return 2

    # the oracle's process pool starts before anything initialises the GPU
    pool, cores = None, 0
    if not a.no_cpu_baseline and a.workload == "c2":
        import multiprocessing as mp
        cores = cpu_cores()
        pool = mp.get_context("spawn").Pool(cores)
    try:
        return run(a, pool, cores)
    finally:
        if pool is not None:
            pool.terminate()


def run(a, pool, cores):
    import numpy as np
    import torch
    import synth
    import paper_2203_09200_amd as R

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    R.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.workload == "c4":
        return run_multistream(a, dev)

    F, H, W = a.frames, a.height, a.width
    t_gen = time.perf_counter()
    frames, masks = synth.workload_c2(n=F, h=H, w=W)
    meas = synth.measured(frames, masks)
    t_gen = time.perf_counter() - t_gen
    print(f"# workload generated in {t_gen:.1f} s", file=sys.stderr, flush=True)
    d_meas = [torch.from_numpy(meas[t]).to(dev) for t in range(F)]
    d_mask = [torch.from_numpy(masks[t]).to(dev) for t in range(F)]
    outs = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(F)]
    outs_u8 = [torch.empty((H, W), dtype=torch.uint8, device=dev) for _ in range(F)]
    me = R.MEParams(search=a.search, check=a.check)
    fsr = R.FSRParams(iters=a.iters, precision=a.precision, pairs=a.pairs, concealed_weight=a.concealed,
                      prior_sigma=a.prior, stop_ratio=a.stop)
    stream = torch.cuda.current_stream()
    seq = R.Sequence(H, W, me, fsr, device=dev, pipelined=not a.no_pipeline)
    torch.cuda.synchronize()   # inputs resident before any frame is enqueued

    def step(events=None):
        seq.reset()
        for t in range(F):
            seq.push(d_meas[t], d_mask[t], stage_events=None if events is None else events[t], stream=stream,
                     out=outs[t], out_u8=outs_u8[t])

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)
    reruns = None
    if a.precision == "mixed":   # count the blocks recomputed in float64 during the timed steps
        reruns = torch.zeros(1, dtype=torch.int64, device=dev)
        fsr.rerun_blocks = reruns

    ev = [[[R.Event() for _ in range(4)] for _ in range(F)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(ev[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"# timed {a.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # frame latency: completion of frame t after the completion of frame t-1
    # (its lag-1 reference); the first frame of a step from its own start
    lat, me_ms, proj_ms, fsr_ms = [], [], [], []
    lat_steady = []
    for k in range(a.steps):
        for t in range(F):
            e = ev[k][t]
            tot = (ev[k][t - 1][3] if t > 0 else e[0]).elapsed_ms(e[3])
            lat.append(tot)
            if t >= 3:
                lat_steady.append(tot)
            me_ms.append(e[0].elapsed_ms(e[1]))
            proj_ms.append(e[1].elapsed_ms(e[2]))
            fsr_ms.append(e[2].elapsed_ms(e[3]))

    host_out = [outs[t].cpu().numpy() for t in range(F)]
    q = float(np.mean([psnr(frames[t], host_out[t]) for t in range(F)]))

    npx = F * H * W
    value = npx * a.steps / elapsed / 1e6
    fsr_avg_s = float(np.mean(fsr_ms)) / 1e3
    nblk = (H // 4) * (W // 4)
    flops = fsr_flops_per_block(a.iters, a.pairs) * nblk
    achieved = flops / fsr_avg_s / 1e12
    rec = counters_from_profile(a.precision)
    default_fsr = not (a.pairs or a.concealed or a.prior or a.stop) and a.precision in ("fp64", "mixed") and \
        a.iters == 100 and (H, W) == (1080, 1920)
    # the counters were taken on this kernel and workload only
    traffic = rec.get("bytes_per_launch") if default_fsr else None
    f32 = a.precision in ("fp32", "mixed")
    peak = PEAK_FP32_VECTOR_TFLOPS if f32 else PEAK_FP64_VECTOR_TFLOPS
    roofline = {"kernel": "fsr_block_kernel_f32" if f32 else "fsr_block_kernel",
                "bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "flops_per_launch": flops, "avg_launch_ms": round(fsr_avg_s * 1e3, 4)}
    if f32:
        # the published FP32 vector rate counts packed FMAs (two per lane and
        # instruction); this library is built without packed FP32, whose FMA
        # rate is that of FP64
        roofline["frac_of_unpacked_fp32"] = round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4)
    if reruns is not None:
        n_re = int(reruns.item())
        # frame 0 has no references: its FSR input is the measured frame, so the
        # float64 form can run on the same input
        o64, _ = R.fsr_blocks(d_meas[0].float(), d_mask[0], R.FSRParams(iters=a.iters))
        d0 = np.abs(o64.cpu().numpy().astype(np.float64) - host_out[0]).reshape(H // 4, 4, W // 4, 4).max(axis=(1, 3))
        roofline["mixed"] = {"recomputed_in_f64": n_re, "blocks": nblk * F * a.steps,
                             "recomputed_frac": round(n_re / (nblk * F * a.steps), 5),
                             "frame0_max_abs_vs_f64": float(f"{d0.max():.3g}"),
                             "note": "avg_launch_ms covers the float32 pass and the float64 recomputation"}
    if default_fsr and rec.get("valu_insts_per_dispatch"):
        # the same launch against the vector-ALU issue rate: one wave64 instruction per 4 cycles per SIMD
        peak_issue = 256 * 4 * 2.4e9 / 4 / 1e9
        got = rec["valu_insts_per_dispatch"] / fsr_avg_s / 1e9
        roofline["issue"] = {"unit": "G wave-instr/s", "achieved": round(got, 2), "peak": peak_issue,
                             "frac": round(got / peak_issue, 4),
                             "valu_insts_per_launch": rec["valu_insts_per_dispatch"]}
    if a.stop:
        roofline["note"] = "flops counted for K iterations per block; the early stop runs fewer"
    if a.prior:
        roofline["note_prior"] = "the prior adds one multiply per bin and iteration, not counted"

    fp32_form = fp64_form = None
    if a.precision in ("fp64", "mixed") and not (a.pairs or a.concealed or a.prior or a.stop or a.no_other_forms):
        legs = dict(seq_args=(H, W, me, dev), d_meas=d_meas, d_mask=d_mask, frames=frames, ref_out=host_out,
                    stream=stream)
        fp32_form = other_form(a, "fp32", False, form="every FSR step in float32 (precision fp32)", **legs)
        if a.precision == "mixed":
            fp64_form = other_form(a, "fp64", not a.no_pipeline, form="FSR in float64 (precision fp64)", **legs)

    cpu = None
    if pool is not None:
        import oracle as O   # the CPU baseline leg
        print(f"# timing the CPU oracle sample on {cores} processes", file=sys.stderr, flush=True)
        recons = [outs_u8[t].cpu().numpy() for t in range(3)]
        cpu = cpu_baseline(pool, cores, frames, masks, recons, O.MEParams(search=a.search, check=a.check),
                           O.FSRParams(iters=a.iters))

    res = {
        "metric": "HR Mpix/s reconstructed (1080p, dynamic mask, D-FSR); p50/p99 frame latency",
        "value": round(value, 3),
        "unit": "HR Mpix/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_of(a.precision),
        "data": "synthetic (seeded smooth texture, 8x8 translating regions, 5% occluders)",
        "config": {"workload": f"{W}x{H} uint8, {F} frames, dynamic quarter mask, D-FSR + "
                               f"{a.check.upper().replace('_', '+')}, R={a.search}, T=4, "
                               f"4x4 blocks, 32x32 support, rho=0.7, gamma=0.5, K={a.iters}, 3 references"
                               + FORM_SUFFIX.get(a.precision, f", block DFT {a.precision}")
                               + (", conjugate-pair FSR" if a.pairs else "")
                               + (f", concealed weighting {a.concealed}" if a.concealed else "")
                               + (f", frequency prior sigma {a.prior}" if a.prior else "")
                               + (f", early stop ratio {a.stop}" if a.stop else ""),
                   "frames": F, "height": H, "width": W, "parallelism": "single GPU",
                   "pipelined": not a.no_pipeline},
        "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3),
                       "p50_steady": round(percentile(lat_steady, 50), 3) if lat_steady else None,
                       "p99_steady": round(percentile(lat_steady, 99), 3) if lat_steady else None,
                       "definition": "completion of frame t after the completion of frame t-1 (its lag-1 "
                                     "reference); steady: frames with three references"},
        "stage_ms_mean": {"me_and_check": round(float(np.mean(me_ms)), 4),
                          "projection": round(float(np.mean(proj_ms)), 4),
                          "fsr": round(float(np.mean(fsr_ms)), 4),
                          "note": ("me_and_check: the lag-1 reference (lags 2-3 run on a side stream during the "
                                   "previous frame's FSR)" if not a.no_pipeline else "all references")},
        "psnr_db": round(q, 3),
        "roofline": roofline,
        "fp64_form": fp64_form,
        "fp32_form": fp32_form,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
