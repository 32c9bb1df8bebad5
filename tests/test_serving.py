"""Scheduling rules of the serving loop on the CPU (simulated device):
per-stream order and dependencies, continuous batching, memory admission
and backpressure, latency statistics."""
import numpy as np
import pytest

from paper_2203_09200_amd import serving as S


def run(sizes, trace, budget=1 << 40, max_batch=64, max_inflight=2, **sim_kw):
    sim = S.SimExecutor(**sim_kw)
    srv = S.Server(sim, budget, max_batch=max_batch, max_inflight=max_inflight)
    sids = [srv.open_stream(h, w) for h, w in sizes]
    reqs = S.run_trace(srv, trace, lambda s, i: (None, None), sids, clock="sim", sim=sim)
    return srv, sim, reqs


def test_poisson_trace_shape():
    rng = np.random.default_rng(0)
    sizes, tr = S.poisson_trace(6, 200, 30.0, rng, size_choices=S.SIZES)
    assert len(sizes) == 6 and all(s in S.SIZES for s in sizes)
    assert len(tr) == 1200
    assert all(a[0] <= b[0] for a, b in zip(tr, tr[1:]))
    for s in range(6):
        ts = [t for t, st, _ in tr if st == s]
        idx = [i for _, st, i in tr if st == s]
        assert idx == list(range(200))
        assert abs(np.mean(np.diff([0.0] + ts)) - 1 / 30) < 0.2 / 30


def test_every_request_served_in_stream_order_with_its_references():
    rng = np.random.default_rng(1)
    sizes = [(288, 352), (720, 1280), (1080, 1920), (64, 64), (2160, 3840)]
    _, tr = S.poisson_trace(len(sizes), 20, 30.0, rng, sizes=sizes)
    srv, sim, reqs = run(sizes, tr)
    assert all(r.done is not None for r in reqs)
    last_end = {}
    seen = {}
    for slot, items, start, end in sim.launched:
        assert len({sid for sid, _, _ in items}) == len(items)     # one frame per stream per batch
        for sid, idx, nref in items:
            assert idx == seen.get(sid, -1) + 1                     # stream order
            assert nref == min(idx, 3)                              # ring references
            assert start >= last_end.get(sid, 0.0)                  # previous frame finished
            seen[sid] = idx
            last_end[sid] = end
    for r in reqs:
        assert r.launched >= r.arrival and r.done > r.launched


def test_continuous_batching_admits_arrivals_while_a_batch_runs():
    sizes = [(2160, 3840), (288, 352), (288, 352)]
    # stream 0 arrives first (a long frame); the others arrive while it runs
    tr = [(0.0, 0, 0), (0.001, 1, 0), (0.002, 2, 0)]
    srv, sim, reqs = run(sizes, tr, max_inflight=2)
    r0, r1, r2 = reqs
    assert r1.launched < r0.done            # admitted into a second batch slot
    assert r2.launched >= r1.launched
    # one slot: the second request waits for the first batch to retire
    srv, sim, reqs = run(sizes, tr, max_inflight=1)
    assert reqs[1].launched >= reqs[0].done


def test_batches_gather_waiting_streams():
    sizes = [(288, 352)] * 8
    tr = [(0.0, s, 0) for s in range(8)] + [(0.0, s, 1) for s in range(8)]
    srv, sim, reqs = run(sizes, tr, max_inflight=1)
    assert [n for _, n in srv.batches] == [8, 8]
    srv, sim, reqs = run(sizes, tr, max_inflight=1, max_batch=3)
    assert max(n for _, n in srv.batches) == 3


def test_memory_budget_bounds_batches_and_is_never_exceeded():
    sizes = [(288, 352)] * 6
    sim = S.SimExecutor()
    one = sim.batch_bytes([(288, 352, 3)])
    rings = sum(sim.ring_bytes(h, w) for h, w in sizes)
    budget = rings + 2 * one + 1000        # room for two frames in flight
    tr = [(0.0, s, i) for i in range(3) for s in range(6)]
    tr.sort()
    srv, sim, reqs = run(sizes, tr, budget=budget, max_inflight=2)
    assert all(r.done is not None for r in reqs)
    assert srv.peak <= budget
    assert max(n for _, n in srv.batches) <= 2
    assert srv.used == rings                # everything released


def test_stream_admission_by_memory():
    sim = S.SimExecutor()
    ring, one = sim.ring_bytes(720, 1280), sim.batch_bytes([(720, 1280, 3)])
    # two rings and one frame in flight fit; a third ring does not
    srv = S.Server(sim, 2 * ring + one + ring // 2)
    a = srv.open_stream(720, 1280)
    srv.open_stream(720, 1280)
    with pytest.raises(S.AdmissionError):
        srv.open_stream(720, 1280)
    srv.close_stream(a)
    srv.open_stream(720, 1280)


def test_submit_checks_stream_and_order():
    srv = S.Server(S.SimExecutor(), 1 << 40)
    sid = srv.open_stream(64, 64)
    with pytest.raises(KeyError):
        srv.submit(S.Request(sid + 1, 0, 0.0))
    with pytest.raises(ValueError):
        srv.submit(S.Request(sid, 1, 0.0))
    srv.submit(S.Request(sid, 0, 0.0))
    with pytest.raises(RuntimeError):
        srv.close_stream(sid)


def test_overload_queues_and_latency_grows():
    """Offered load twice the modelled device rate: everything is still
    served, in order, with latency growing over the trace."""
    rng = np.random.default_rng(3)
    sizes = [(720, 1280)] * 4
    _, tr = S.poisson_trace(4, 60, 30.0, rng, sizes=sizes)
    px_rate = 4 * 30 * 720 * 1280 / 2.0
    srv, sim, reqs = run(sizes, tr, px_per_s=px_rate)
    lat = [r.latency for r in sorted(reqs, key=lambda r: r.arrival)]
    assert np.mean(lat[-20:]) > 5 * np.mean(lat[:20])
    st = S.summarize(reqs, lambda r: 720 * 1280)
    assert st["offered_mpix_per_s"] > 1.5 * st["sustained_mpix_per_s"]


def test_summarize_percentiles():
    reqs = []
    for k in range(100):
        r = S.Request(0, k, float(k))
        r.done = k + (k + 1) * 1e-3      # latencies 1..100 ms
        reqs.append(r)
    st = S.summarize(reqs, lambda r: 1000)
    assert st["frames"] == 100
    assert st["latency_ms"]["p50"] == pytest.approx(50.5)
    assert st["latency_ms"]["p99"] == pytest.approx(99.01)
    assert st["latency_ms"]["max"] == pytest.approx(100.0)


def test_admission_keeps_room_for_the_largest_frame_of_any_stream():
    """A large stream opened first must still be able to run once smaller
    streams opened after it hold their rings.  Here the 64x64 stream's ring
    and frame fit, and the 8x8 stream's ring and frame would fit next to the
    64x64 ring, but both rings together leave less than the 64x64 frame
    needs: the second open is refused (admitted, the 64x64 frame could never
    launch)."""
    sim = S.SimExecutor()
    ring64, one64 = sim.ring_bytes(64, 64), sim.batch_bytes([(64, 64, 3)])
    ring8, one8 = sim.ring_bytes(8, 8), sim.batch_bytes([(8, 8, 3)])
    budget = ring64 + one64 + ring8 // 2
    assert ring64 + ring8 + one8 <= budget < ring64 + ring8 + one64
    srv = S.Server(sim, budget)
    srv.open_stream(64, 64)
    with pytest.raises(S.AdmissionError):
        srv.open_stream(8, 8)
    # with room for both rings and the large frame, both run to completion
    budget = ring64 + ring8 + one64
    tr = [(0.0, 1, 0), (0.0, 0, 0), (0.001, 1, 1), (0.001, 0, 1)]
    srv, sim2, reqs = run([(64, 64), (8, 8)], tr, budget=budget)
    assert all(r.done is not None for r in reqs)
    assert srv.peak <= budget


def test_open_stream_counts_batches_in_flight():
    """Opening a stream while batches hold memory never takes `used` past
    the budget: the ring must fit next to what is held now, and the stream
    is admitted once the batch has retired."""
    sim = S.SimExecutor()
    sim.clock = lambda: 0.0
    ring, one = sim.ring_bytes(288, 352), sim.batch_bytes([(288, 352, 3)])
    budget = 3 * ring + 2 * one - 1000
    srv = S.Server(sim, budget, max_inflight=1)
    a, b = srv.open_stream(288, 352), srv.open_stream(288, 352)
    srv.submit(S.Request(a, 0, 0.0))
    srv.submit(S.Request(b, 0, 0.0))
    srv.step(0.0)                           # one batch of both frames in flight
    assert len(srv.inflight) == 1 and len(srv.inflight[0].requests) == 2
    assert srv.used == 2 * ring + sim.batch_bytes([(288, 352, 0)] * 2)
    with pytest.raises(S.AdmissionError):
        srv.open_stream(288, 352)           # rings + largest frame fit, but not next to the batch
    assert srv.used <= budget
    sim.clock = lambda: 1.0
    srv.step(1.0)                           # the batch retires
    assert not srv.inflight
    srv.open_stream(288, 352)
    assert srv.used <= budget


@pytest.mark.timeout(60)
def test_real_clock_loop_reports_a_stall():
    """If nothing is in flight, nothing can launch and no arrivals are left,
    the real-clock loop raises instead of spinning."""
    class Stuck(S.SimExecutor):
        def batch_bytes(self, shapes):        # every batch larger than any budget
            return 1 << 60

    sim = Stuck()
    sim.clock = lambda: 0.0
    srv = S.Server(sim, 1 << 40)
    srv.streams[0] = S._Stream(0, 8, 8, 0)   # a stream admitted by an earlier rule
    with pytest.raises(RuntimeError, match="stalled"):
        S.run_trace(srv, [(0.0, 0, 0)], lambda s, i: (None, None), [0], clock="real")
