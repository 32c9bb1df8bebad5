"""Small drivers to run under rocprofv3 (counter and trace collection).

    python -m paper_2203_09200_amd.profiling fsr  [--reps 3] [--delta D] [--precision P] [--iters K ...]
                                                   [--mixed-bound A]   # FSR kernel, 1080p workload frame
    python -m paper_2203_09200_amd.profiling copy [--mib 1024] # plain device copy of known size

`fsr` launches fsr_blocks on one frame of the 1920x1080 benchmark workload
(dynamic mask, K = 100 or the given iteration counts) `reps` times each.  `copy` copies a buffer of the given
size once with torch (reads and writes exactly `mib` MiB), so FETCH_SIZE and
WRITE_SIZE of the same run calibrate the counters' units.

`record [--precision fp64|mixed]` writes the form's record under profiles/
(FORMS) from the per-dispatch counter values read off the rocprofv3 CSVs,
keyed by the SHA-256 of the kernels' sources, so that bench.py reports
`traffic` only while the kernels are unchanged.  A mixed launch is two
dispatches (the float32 pass and the float64 recomputation of the listed
blocks); its record adds their per-dispatch averages.  With --sq-csv (a run that
collected SQ_INSTS_VALU) it also records the VALU wave-instructions per launch,
from which bench.py reports the position against the vector-ALU issue rate.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# per FSR form: the sources its kernels compile from, the kernel-name prefixes
# of its dispatches, and the record file under profiles/
FORMS = {
    "fp64": {"sources": ("fsr.hip", "fft.h", "common.h"), "kernels": ("fsr_block_kernel<",),
             "record": "fsr_block_kernel_1080p_traffic.json"},
    "mixed": {"sources": ("fsr32.hip", "fsr.hip", "fft.h", "common.h"),
              "kernels": ("fsr_block_kernel_f32<", "fsr_block_kernel<"),
              "record": "fsr_mixed_1080p_traffic.json"},
}
KERNEL_SOURCES = FORMS["fp64"]["sources"]


def kernel_digest(precision: str = "fp64") -> str:
    """SHA-256 over the sources of the form's FSR kernels, in a fixed order."""
    h = hashlib.sha256()
    for name in FORMS[precision]["sources"]:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def run_fsr(reps: int, delta: float = 0.0, precision: str = "fp64", iters=(100,), mixed_bound=None):
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import synth
    import paper_2203_09200_amd as R
    f, m = synth.workload_c2(n=1)
    meas = synth.measured(f, m)[0]
    v = torch.from_numpy(meas.astype(np.float32)).cuda()
    c = torch.from_numpy(m[0]).cuda()
    for K in iters:
        prm = R.FSRParams(iters=K, concealed_weight=delta, precision=precision)
        if mixed_bound is not None:
            prm.mixed_bound = mixed_bound
        cnt = None
        if precision == "mixed":
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        R.fsr_blocks(v, c, prm)
        torch.cuda.synchronize()
        prm.rerun_blocks = cnt
        e0, e1 = R.Event(), R.Event()
        e0.record()
        for _ in range(reps):
            R.fsr_blocks(v, c, prm)
        e1.record()
        extra = ""
        if cnt is not None:
            nb = (v.shape[0] // 4) * (v.shape[1] // 4)
            extra = f", bound {prm.mixed_bound}: {int(cnt.item()) / reps / nb:.2%} of the blocks recomputed in float64"
        print(f"fsr_blocks x{reps} done: {e0.elapsed_ms(e1) / reps:.3f} ms per 1080p frame "
              f"(K {K}, delta {delta}, precision {precision}{extra})", flush=True)


def run_copy(mib: int):
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB", flush=True)


def _counter_per_dispatch(csv_path: str, kernel_substr: str, counter: str):
    vals = []
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
            if kernel_substr in name and row.get("Counter_Name") == counter:
                vals.append(float(row["Counter_Value"]))
    return vals


def _per_launch(csv_path, kernels, counter):
    """Sum over the form's kernels of the counter's per-dispatch average."""
    total = 0.0
    for k in kernels:
        v = _counter_per_dispatch(csv_path, k, counter)
        if not v:
            raise SystemExit(f"no {counter} rows for {k} in {csv_path}")
        total += sum(v) / len(v)
    return total


def record(fsr_fetch_csv, fsr_write_csv, copy_fetch_csv, copy_write_csv, copy_mib, copy_kernel, sq_csv=None,
           precision="fp64"):
    form = FORMS[precision]
    ff = _per_launch(fsr_fetch_csv, form["kernels"], "FETCH_SIZE")
    fw = _per_launch(fsr_write_csv, form["kernels"], "WRITE_SIZE")
    cf = _counter_per_dispatch(copy_fetch_csv, copy_kernel, "FETCH_SIZE")
    cw = _counter_per_dispatch(copy_write_csv, copy_kernel, "WRITE_SIZE")
    nbytes = copy_mib << 20
    # counters read in KiB; the copy of known size fixes the scale of each
    s_fetch = nbytes / max(cf) if cf else None
    s_write = nbytes / max(cw) if cw else None
    rec = {"kernel": " + ".join(k.rstrip("<") for k in form["kernels"]), "precision": precision,
           "workload": "1920x1080 frame, dynamic mask, K=100",
           "kernel_sources": list(form["sources"]), "kernel_sha256": kernel_digest(precision),
           "fetch_kib_per_dispatch": ff, "write_kib_per_dispatch": fw, "copy_mib": copy_mib,
           "copy_fetch_kib": max(cf), "copy_write_kib": max(cw),
           "fetch_scale_bytes_per_unit": s_fetch, "write_scale_bytes_per_unit": s_write,
           "bytes_per_launch": ff * s_fetch + fw * s_write}
    if sq_csv:
        rec["valu_insts_per_dispatch"] = _per_launch(sq_csv, form["kernels"], "SQ_INSTS_VALU")
    out = os.path.join(ROOT, "profiles", form["record"])
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a1 = sub.add_parser("fsr")
    a1.add_argument("--reps", type=int, default=3)
    a1.add_argument("--delta", type=float, default=0.0, help="concealed weighting")
    a1.add_argument("--precision", default="fp64")
    a1.add_argument("--iters", type=int, nargs="+", default=[100],
                    help="iteration counts to time in turn (K = 0 times the setup alone)")
    a1.add_argument("--mixed-bound", type=float, default=None, help="near-tie bound a of the mixed form")
    a2 = sub.add_parser("copy")
    a2.add_argument("--mib", type=int, default=1024)
    a3 = sub.add_parser("record")
    a3.add_argument("fsr_fetch_csv")
    a3.add_argument("fsr_write_csv")
    a3.add_argument("copy_fetch_csv")
    a3.add_argument("copy_write_csv")
    a3.add_argument("--copy-mib", type=int, default=1024)
    a3.add_argument("--copy-kernel", default="copyBuffer")
    a3.add_argument("--sq-csv", default=None, help="counter CSV of a run with SQ_INSTS_VALU")
    a3.add_argument("--precision", choices=sorted(FORMS), default="fp64")
    a = ap.parse_args(argv)
    if a.cmd == "fsr":
        run_fsr(a.reps, a.delta, a.precision, a.iters, a.mixed_bound)
    elif a.cmd == "copy":
        run_copy(a.mib)
    else:
        record(a.fsr_fetch_csv, a.fsr_write_csv, a.copy_fetch_csv, a.copy_write_csv, a.copy_mib,
               a.copy_kernel, a.sq_csv, a.precision)
    return 0


if __name__ == "__main__":
    sys.exit(main())
