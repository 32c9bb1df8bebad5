"""Serving: per-frame reconstruction requests from concurrent streams.

Each stream is an independent causal recursion (Sec. 2.2): frame t of a
stream needs that stream's reconstructions of frames t-1..t-3, so the
server keeps every open stream's ring of reconstructions, measured frames
and masks resident in device memory, and a stream has at most one frame on
the GPU at a time.

Continuous batching: whenever fewer than `max_inflight` batches are on the
GPU, the scheduler forms a new batch from the oldest waiting head-of-line
requests of idle streams (FIFO by arrival), as many as fit the free memory
budget and `max_batch` frames, and launches it (rfsr_reconstruct_batch) on
one of `max_inflight` device streams.  Requests that arrive while batches
run are admitted as soon as a batch slot and memory free up; batches on
different device streams share no stream and therefore overlap on the GPU.

Memory admission: `open_stream` admits a stream only if (a) its ring fits
next to everything held now (the open rings and the batches in flight) and
(b) all rings together leave room for the largest one-frame batch of any
open stream, the new one included, so that every stream can always run
alone once the batches in flight retire (no stream is starved by rings
opened after it).  A batch takes memory (job tables and workspace) from the
budget until it retires, so the sum never exceeds the budget.

Executors: `GpuExecutor` runs batches through the C ABI (or, with
mode="frame", one frame at a time through rfsr_reconstruct_frame: the plain
loop the served form is compared with); `SimExecutor` models the device by a
throughput and a per-batch overhead, for tests of the scheduling rules and
what-if runs on a CPU.

    python -m paper_2203_09200_amd.serving [--streams 32] [--frames 300] [--fps 30] [--load 1.0]

prints one JSON line: offered load, sustained HR Mpix/s, p50/p99 latency
(arrival -> result ready on the device), for the batched server and for the
plain single-stream loops (float64 FSR, and every FSR step in float32) on the
same request trace.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time
from dataclasses import dataclass, field

SLOTS = 4   # ring slots per stream: frame t uses slot t mod 4, references t-1..t-3


class AdmissionError(RuntimeError):
    pass


@dataclass
class Request:
    """One frame of one stream.  meas / mask: the measured frame and its
    quarter-sampling mask (device uint8 planes for the GPU executor)."""
    stream: int
    index: int
    arrival: float
    meas: object = None
    mask: object = None
    launched: float | None = None
    done: float | None = None
    batch_size: int = 0
    out: object = None      # float32 result plane (ring slot view; valid for SLOTS - 1 more frames)
    out_u8: object = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


@dataclass
class _Stream:
    sid: int
    H: int
    W: int
    ring_bytes: int
    queue: collections.deque = field(default_factory=collections.deque)
    t: int = 0              # frames launched
    busy: bool = False
    expect: int = 0         # next frame index accepted by submit


@dataclass
class _Inflight:
    slot: int
    handle: object
    requests: list
    nbytes: int


class Server:
    """Continuous-batching scheduler over an executor (see module doc)."""

    def __init__(self, executor, mem_budget: int, max_batch: int = 64, max_inflight: int = 2,
                 nref: int = 3):
        if max_batch < 1 or max_inflight < 1 or not 0 <= nref <= 3:
            raise ValueError("max_batch >= 1, max_inflight >= 1, nref in 0..3")
        self.ex = executor
        self.budget = int(mem_budget)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.nref = nref
        self.streams: dict[int, _Stream] = {}
        self.inflight: list[_Inflight] = []
        self.used = 0           # bytes held by rings and in-flight batches
        self.peak = 0
        self.batches = []       # (launch time, frames) per launched batch
        self._next_sid = 0

    # ---------------------------------------------------------- streams --
    def _one_frame_bytes(self, H: int, W: int) -> int:
        return self.ex.batch_bytes([(H, W, self.nref)])

    def open_stream(self, H: int, W: int) -> int:
        ring = self.ex.ring_bytes(H, W)
        rings = sum(s.ring_bytes for s in self.streams.values())
        largest = max([self._one_frame_bytes(H, W)] +
                      [self._one_frame_bytes(s.H, s.W) for s in self.streams.values()])
        if rings + ring + largest > self.budget:
            raise AdmissionError(f"stream {H}x{W} does not fit the memory budget: rings "
                                 f"{rings + ring} + largest one-frame batch {largest} > {self.budget} bytes")
        if self.used + ring > self.budget:
            raise AdmissionError(f"stream {H}x{W} does not fit next to the memory held now "
                                 f"({self.used} + {ring} > {self.budget} bytes); retry after batches retire")
        sid = self._next_sid
        self._next_sid += 1
        self.ex.open(sid, H, W)
        self.streams[sid] = _Stream(sid, H, W, ring)
        self.used += ring
        self.peak = max(self.peak, self.used)
        return sid

    def close_stream(self, sid: int):
        s = self.streams[sid]
        if s.busy or s.queue:
            raise RuntimeError(f"stream {sid} still has work")
        self.ex.close(sid)
        self.used -= s.ring_bytes
        del self.streams[sid]

    def submit(self, req: Request):
        s = self.streams.get(req.stream)
        if s is None:
            raise KeyError(f"stream {req.stream} is not open")
        if req.index != s.expect:
            raise ValueError(f"stream {req.stream}: frame {req.index} submitted, {s.expect} expected")
        s.expect += 1
        s.queue.append(req)

    # -------------------------------------------------------- scheduling --
    def pending(self) -> int:
        return sum(len(s.queue) for s in self.streams.values()) + sum(len(b.requests) for b in self.inflight)

    def step(self, now: float) -> list:
        """Retire finished batches, then launch new ones while batch slots and
        memory allow.  Returns the requests that finished."""
        done = self._retire()
        while len(self.inflight) < self.max_inflight:
            if not self._launch(now):
                break
        return done

    def _retire(self) -> list:
        done = []
        keep = []
        for b in self.inflight:
            t = self.ex.poll(b.handle)
            if t is None:
                keep.append(b)
                continue
            for r in b.requests:
                r.done = t
                s = self.streams[r.stream]
                s.busy = False
                done.append(r)
            self.used -= b.nbytes
        self.inflight = keep
        return done

    def _launch(self, now: float) -> bool:
        cands = sorted((s for s in self.streams.values() if s.queue and not s.busy),
                       key=lambda s: (s.queue[0].arrival, s.sid))
        if not cands:
            return False
        free = self.budget - self.used
        items, shapes = [], []
        nbytes = 0
        for s in cands:
            if len(items) == self.max_batch:
                break
            shape = (s.H, s.W, min(s.t, self.nref))
            need = self.ex.batch_bytes(shapes + [shape])
            if need > free:
                break            # FIFO: a later, smaller frame does not overtake
            items.append(s)
            shapes.append(shape)
            nbytes = need
        if not items:
            return False         # wait for memory
        busy_slots = {b.slot for b in self.inflight}
        slot = next(k for k in range(self.max_inflight) if k not in busy_slots)
        reqs = []
        for s in items:
            r = s.queue.popleft()
            r.launched = now
            r.batch_size = len(items)
            reqs.append(r)
        handle = self.ex.launch([(self.streams[r.stream], r, min(self.streams[r.stream].t, self.nref))
                                 for r in reqs], slot)
        for s in items:
            s.busy = True
            s.t += 1
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        self.inflight.append(_Inflight(slot, handle, reqs, nbytes))
        self.batches.append((now, len(reqs)))
        return True

    def next_completion(self):
        ts = [self.ex.eta(b.handle) for b in self.inflight]
        ts = [t for t in ts if t is not None]
        return min(ts) if ts else None


# --------------------------------------------------------------- executors --
class SimExecutor:
    """Device model for CPU runs: a batch occupies the device for
    overhead + pixels / px_per_s; batches run one after another."""

    def __init__(self, px_per_s: float = 3.4e8, overhead: float = 2e-4, bytes_per_px: float = 48.0,
                 clock=None):
        self.px_per_s = px_per_s
        self.overhead = overhead
        self.bytes_per_px = bytes_per_px
        self.clock = clock          # callable returning the current time
        self.free_at = 0.0
        self.launched = []          # (slot, [(sid, index, nref)], start, end)

    def ring_bytes(self, H, W):
        return SLOTS * H * W * 7

    def batch_bytes(self, shapes):
        return int(sum(H * W for H, W, _ in shapes) * self.bytes_per_px) + 256 * (1 + len(shapes))

    def open(self, sid, H, W):
        pass

    def close(self, sid):
        pass

    def launch(self, items, slot):
        now = self.clock()
        start = max(now, self.free_at)
        end = start + self.overhead + sum(s.H * s.W for s, _, _ in items) / self.px_per_s
        self.free_at = end
        self.launched.append((slot, [(s.sid, r.index, nref) for s, r, nref in items], start, end))
        return end

    def poll(self, handle):
        return handle if self.clock() >= handle else None

    def eta(self, handle):
        return handle


class GpuExecutor:
    """Runs batches on the GPU through the C ABI.  mode="batch": one
    rfsr_reconstruct_batch per batch; mode="frame": rfsr_reconstruct_frame
    per request (the plain loop).  Each in-flight batch slot has its own
    device stream (default priority)."""

    def __init__(self, me=None, fsr=None, device=None, mode: str = "batch", max_inflight: int = 2,
                 on_launch=None):
        import torch
        from . import _lib as R
        self.torch, self.R = torch, R
        self.me = me or R.MEParams()
        self.fsr = fsr or R.FSRParams()
        self.device = device or torch.device("cuda")
        if mode not in ("batch", "frame"):
            raise ValueError(mode)
        self.mode = mode
        self.hs = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        self.rings = {}
        self.on_launch = on_launch        # callback(requests, device stream) after the launch
        self._frame_ws = [R.Workspace(self.device) for _ in range(max_inflight)]
        torch.cuda.synchronize(self.device)
        self.t0_host = time.perf_counter()
        self.t0_ev = torch.cuda.Event(enable_timing=True)
        self.t0_ev.record(torch.cuda.current_stream(self.device))
        torch.cuda.synchronize(self.device)
        self._bytes_cache = {}

    def reset_clock(self):
        self.torch.cuda.synchronize(self.device)
        self.t0_host = time.perf_counter()
        self.t0_ev.record(self.torch.cuda.current_stream(self.device))
        self.torch.cuda.synchronize(self.device)
        return self.t0_host

    def ring_bytes(self, H, W):
        return SLOTS * H * W * (1 + 1 + 4 + 1)

    def batch_bytes(self, shapes):
        """Sum of the one-frame batch sizes: an upper bound of the batch's
        bytes (each term carries its own FSR tables and table header)."""
        total = 0
        for shape in shapes:
            n = self._bytes_cache.get(shape)
            if n is None:
                n = self._bytes_cache[shape] = batch_bytes([shape], self.me, self.fsr)
            total += n
        return total

    def open(self, sid, H, W):
        torch = self.torch
        mk = lambda dt: [torch.empty((H, W), dtype=dt, device=self.device) for _ in range(SLOTS)]
        self.rings[sid] = {"meas": mk(torch.uint8), "mask": mk(torch.uint8), "out": mk(torch.float32),
                           "out_u8": mk(torch.uint8)}

    def close(self, sid):
        del self.rings[sid]

    def _frame(self, s, r, nref):
        ring = self.rings[s.sid]
        t = s.t
        slot = t % SLOTS
        ring["meas"][slot].copy_(r.meas, non_blocking=True)
        ring["mask"][slot].copy_(r.mask, non_blocking=True)
        refs = tuple((ring["out_u8"][(t - k) % SLOTS], ring["meas"][(t - k) % SLOTS],
                      ring["mask"][(t - k) % SLOTS]) for k in range(1, nref + 1))
        r.out, r.out_u8 = ring["out"][slot], ring["out_u8"][slot]
        return self.R.BatchFrame(ring["meas"][slot], ring["mask"][slot], refs, r.out, r.out_u8)

    def launch(self, items, slot):
        torch, R = self.torch, self.R
        hs = self.hs[slot]
        keep = []
        with torch.cuda.stream(hs):
            frames = [self._frame(s, r, nref) for s, r, nref in items]
            if self.mode == "batch":
                b = R.Batch(frames, self.me, self.fsr, stream=hs)   # workspace from the caching allocator
                b.run(stream=hs)
                keep.append(b)
            else:
                for f in frames:
                    R.reconstruct_frame(f.cur, f.mask, list(f.refs), self.me, self.fsr, out=f.out,
                                        out_u8=f.out_u8, workspace=self._frame_ws[slot], stream=hs)
            if self.on_launch is not None:
                self.on_launch([r for _, r, _ in items], hs)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(hs)
        return (ev, keep)

    def poll(self, handle):
        ev, _ = handle
        if not ev.query():
            return None
        return self.t0_host + self.t0_ev.elapsed_time(ev) / 1e3

    def eta(self, handle):
        return None


def batch_bytes(shapes, me=None, fsr=None) -> int:
    """Device bytes a batch of frames (H, W, nref) takes: workspace plus job
    tables (computed by the library from descriptors with placeholder
    addresses, which it does not dereference)."""
    import ctypes
    from . import _lib as R
    n = len(shapes)
    ds = (R.FrameDesc * n)()
    for d, (H, W, nref) in zip(ds, shapes):
        d.cur = d.cur_mask = d.out = 256
        for k in range(nref):
            d.ref_recon[k] = d.ref_meas[k] = d.ref_mask[k] = 256
        d.nref, d.H, d.W, d.pitch = nref, H, W, W
    mc, fc = (me or R.MEParams()).c(), (fsr or R.FSRParams()).c()
    L = R.lib()
    ws = L.rfsr_batch_workspace_bytes(ds, n, ctypes.byref(mc), ctypes.byref(fc))
    tb = L.rfsr_batch_table_bytes(ds, n)
    if ws == 0 or tb == 0:
        raise R.RfsrError(f"invalid batch shapes {shapes}")
    return int(ws + tb)


# ------------------------------------------------------------------ traces --
def poisson_trace(n_streams: int, frames: int, fps: float, rng, sizes=None, size_choices=None):
    """Arrival times: per stream, exponential inter-arrival times of mean
    1/fps, `frames` frames.  Returns (sizes per stream, sorted list of
    (arrival, stream, index))."""
    if sizes is None:
        idx = rng.integers(0, len(size_choices), n_streams)
        sizes = [tuple(size_choices[i]) for i in idx]
    ev = []
    for s in range(n_streams):
        t = 0.0
        for i in range(frames):
            t += rng.exponential(1.0 / fps)
            ev.append((t, s, i))
    ev.sort()
    return sizes, ev


def run_trace(server: Server, trace, payload, sids, clock: str = "real", sim=None, progress=None,
              t_start=None):
    """Feed `trace` ([(arrival, stream index, frame index)]) to `server` and
    run until every request has finished.  payload(stream, index) -> (meas,
    mask); sids[stream] is the server's id of the (open) stream.
    clock="real" runs against the wall clock (arrivals replayed in real time
    from t_start, default now); clock="sim" advances a virtual clock to the
    next arrival or completion (`sim` is the SimExecutor).  Returns the
    requests (all finished)."""
    reqs = [Request(sids[s], i, t) for t, s, i in trace]
    finished = []
    k = 0
    n = len(reqs)
    if clock == "sim":
        now = 0.0
        sim.clock = lambda: now
        while len(finished) < n:
            while k < n and reqs[k].arrival <= now:
                r = reqs[k]
                r.meas, r.mask = payload(trace[k][1], r.index)
                server.submit(r)
                k += 1
            finished += server.step(now)
            nxt = [reqs[k].arrival] if k < n else []
            c = server.next_completion()
            if c is not None:
                nxt.append(c)
            if not nxt:
                if len(finished) < n:
                    raise RuntimeError("scheduler stalled with work pending")
                break
            now = max(now, min(nxt))
        return reqs
    t0 = time.perf_counter() if t_start is None else t_start
    last_print = t0
    while len(finished) < n:
        now = time.perf_counter() - t0
        while k < n and reqs[k].arrival <= now:
            r = reqs[k]
            r.meas, r.mask = payload(trace[k][1], r.index)
            r.arrival += t0          # absolute host time
            server.submit(r)
            k += 1
        done = server.step(time.perf_counter())
        finished += done
        if not done and not server.inflight and k == n and len(finished) < n:
            raise RuntimeError("scheduler stalled with work pending")
        if progress and time.perf_counter() - last_print > 10.0:
            last_print = time.perf_counter()
            progress(f"t={now:.1f}s: {len(finished)}/{n} done, {server.pending()} pending")
        if not done:
            wait = 2e-4
            if k < n:
                wait = min(wait, max(reqs[k].arrival - (time.perf_counter() - t0), 0.0))
            time.sleep(wait)
    return reqs


def summarize(reqs, px_of):
    import numpy as np
    lat = np.array([r.latency for r in reqs]) * 1e3
    first = min(r.arrival for r in reqs)
    last = max(r.done for r in reqs)
    px = sum(px_of(r) for r in reqs)
    span = max(r.arrival for r in reqs) - first
    return {"frames": len(reqs), "hr_mpix": round(px / 1e6, 3),
            "offered_mpix_per_s": round(px / span / 1e6, 3) if span > 0 else None,
            "sustained_mpix_per_s": round(px / (last - first) / 1e6, 3),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "max": round(float(lat.max()), 3)}}


# -------------------------------------------------------------------- main --
SIZES = [(288, 352), (720, 1280), (1080, 1920), (2160, 3840)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--streams", type=int, default=32)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--fps", type=float, default=30.0)
    ap.add_argument("--load", type=float, default=1.0, help="scale of the arrival rate")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--max-inflight", type=int, default=2)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--pool", type=int, default=8, help="distinct synthetic frames per size and mask kind")
    ap.add_argument("--precision", choices=["fp64", "bf16x3", "fp16x3", "fp32", "mixed"], default="mixed",
                    help="FSR arithmetic of the batched server (default mixed: the float64 model's result; "
                         "the plain loops are fp64 and fp32)")
    a = ap.parse_args(argv)

    import numpy as np
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    from . import _lib as R

    if not torch.cuda.is_available():
        print("serving: no GPU visible", file=sys.stderr)
        return 1
    R.lib()
    dev = torch.device("cuda:0")
    log = lambda m: print(f"# {m}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(synth.seed_for(5))
    sizes, trace = poisson_trace(a.streams, a.frames, a.fps * a.load, rng, size_choices=SIZES)
    # frame pool: per size and mask kind, `pool` frames of the 1080p generator
    pool = {}
    t_gen = time.perf_counter()
    for (h, w) in sorted(set(sizes)):
        for kind in ("fixed", "dynamic"):
            prng = np.random.default_rng(synth.seed_for(5, 1000 + 2 * SIZES.index((h, w)) + (kind == "dynamic")))
            f = synth.video_regions(a.pool, h, w, prng)
            m = synth.mask_sequence(kind, a.pool, h, w, prng)
            pool[(h, w, kind)] = ([torch.from_numpy(x).to(dev) for x in synth.measured(f, m)],
                                  [torch.from_numpy(x).to(dev) for x in m])
    log(f"frame pool generated in {time.perf_counter() - t_gen:.1f} s")
    kinds = ["fixed" if s % 2 == 0 else "dynamic" for s in range(a.streams)]
    offs = rng.integers(0, a.pool, a.streams)

    def payload(s, i):
        fm, mm = pool[(*sizes[s], kinds[s])]
        return fm[(i + offs[s]) % a.pool], mm[(i + offs[s]) % a.pool]

    me = R.MEParams()
    px_of = lambda r: r.out.numel()
    results = {}
    modes = [("batched", "batch", a.max_batch, a.max_inflight, a.precision)]
    if not a.no_plain:
        modes.append(("plain", "frame", 1, 1, "fp64"))
        modes.append(("plain_fp32", "frame", 1, 1, "fp32"))
    budget = int(a.budget_gib * 2**30)
    for name, mode, mb, mi, prec in modes:
        fsr = R.FSRParams(iters=a.iters, precision=prec)
        ex = GpuExecutor(me, fsr, dev, mode=mode, max_inflight=mi)
        # warm-up outside the trace: four frames per stream (kernels loaded, allocator primed)
        warm_srv = Server(ex, budget, max_batch=mb, max_inflight=mi)
        wsids = [warm_srv.open_stream(h, w) for h, w in sizes]
        run_trace(warm_srv, [(0.0, s, i) for i in range(4) for s in range(a.streams)], payload, wsids)
        for sid in wsids:
            warm_srv.close_stream(sid)
        srv = Server(ex, budget, max_batch=mb, max_inflight=mi)
        sids = [srv.open_stream(h, w) for h, w in sizes]
        log(f"{name}: replaying {len(trace)} requests")
        t0 = ex.reset_clock()
        reqs = run_trace(srv, trace, payload, sids, clock="real", progress=lambda m: log(f"{name} {m}"),
                         t_start=t0)
        results[name] = summarize(reqs, px_of)
        results[name]["mean_batch"] = round(float(np.mean([n for _, n in srv.batches])), 2)
        results[name]["peak_mem_gib"] = round(srv.peak / 2**30, 3)
        log(f"{name}: {json.dumps(results[name])}")
        del srv, warm_srv, ex
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    out = {"metric": "serving: HR Mpix/s sustained and p50/p99 frame latency (arrival -> result on device)",
           "streams": a.streams, "frames_per_stream": a.frames, "fps": a.fps * a.load,
           "sizes": {f"{h}x{w}": sizes.count((h, w)) for h, w in SIZES},
           "iters": a.iters, "precision": a.precision, "max_batch": a.max_batch,
           "max_inflight": a.max_inflight,
           "budget_gib": a.budget_gib, **results}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
