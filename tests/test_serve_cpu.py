"""The serving scheduler on the CPU: a fake executor runs the oracle and
advances a simulated clock, so admission, slot reuse, HBM-budget limits and
result identity (alone vs in the mix) are checked without a GPU."""
import numpy as np

from oracle import rsz_oracle as O
from paper_2206_11297_amd import serve, synth


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class CpuExecutor:
    """Runs a batch with the oracle when launched; it finishes after
    raw_bytes / bandwidth simulated seconds (slots run concurrently)."""

    def __init__(self, clock, bandwidth=1e9):
        self.clock, self.bw = clock, bandwidth
        self.max_in_flight_bytes = 0
        self.in_flight = {}
        self.launches = []

    def size_request(self, r):
        w, b, eb, mode = r.params
        st, cap = O.max_bytes(O.params(*r.frame.shape, w, b, eb, mode), r.peaks.shape[0])
        r.out_cap = cap
        r.ws_bytes = 10 * r.frame.size // (b * b) + 4096
        r.raw_bytes = r.frame.size * 4

    def fits(self, batch, limits):
        return (sum(r.out_cap for r in batch) <= limits.out_bytes and
                sum(r.ws_bytes for r in batch) <= limits.ws_bytes)

    def start(self):
        pass

    def launch(self, slot, batch, now):
        outs = []
        for r in batch:
            w, b, eb, mode = r.params
            st, s, n = O.compress(O.params(*r.frame.shape, w, b, eb, mode), r.frame, r.peaks)
            outs.append((st, n, s))
        dur = sum(r.raw_bytes for r in batch) / self.bw
        self.in_flight[slot] = sum(r.out_cap + r.ws_bytes for r in batch)
        self.max_in_flight_bytes = max(self.max_in_flight_bytes, sum(self.in_flight.values()))
        self.launches.append((slot, [r.rid for r in batch], now))
        return (now, now + dur, outs)

    def done(self, h):
        return self.clock() >= h[1]

    def finish(self, slot, h, batch, keep):
        del self.in_flight[slot]
        st = [o[0] for o in h[2]]
        n = [o[1] for o in h[2]]
        return st, n, h[0], h[1], [o[2] for o in h[2]] if keep else None

    def idle(self, pending, inflight, until_next):
        # advance simulated time to the next event
        nxt = [h[1] for (_, h, _) in inflight.values()]
        if until_next is not None:
            nxt.append(self.clock() + until_next)
        self.clock.t = max(self.clock.t, min(nxt)) if nxt else self.clock.t + 1e-6


def _requests(n, rate, seed=3):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    pool = [synth.tiny_case(50 + k, (2, 24 + 4 * k, 40 + 6 * k), 3, "normal") for k in range(4)]
    reqs = []
    for i in range(n):
        f, pk = pool[i % 4]
        eb = [5.0, 10.0, 20.0][i % 3]
        reqs.append(serve.Request(i, float(t[i]), f, pk, (5, 2, eb, 0)))
    return reqs


def test_every_request_served_and_identical_to_alone():
    clock = SimClock()
    ex = CpuExecutor(clock, bandwidth=2e6)
    limits = serve.SlotLimits(max_frames=4, out_bytes=1 << 20, ws_bytes=1 << 20)
    reqs = _requests(40, rate=2000.0)
    res = serve.Scheduler(ex, 3, limits, clock=clock).run(reqs, keep_streams=True)
    assert [r.rid for r in res] == list(range(40))
    for r, q in zip(res, reqs):
        assert r.status == 0 and r.done >= r.arrival and r.start >= r.arrival
        w, b, eb, mode = q.params
        st, alone, n = O.compress(O.params(*q.frame.shape, w, b, eb, mode), q.frame, q.peaks)
        np.testing.assert_array_equal(r.stream, alone)
    # batching happened (requests arrived while slots were busy)
    assert max(len(ids) for _, ids, _ in ex.launches) > 1
    assert all(len(ids) <= 4 for _, ids, _ in ex.launches)


def test_budget_limits_in_flight_memory():
    clock = SimClock()
    ex = CpuExecutor(clock, bandwidth=1e6)
    reqs = _requests(30, rate=1e5)
    for r in reqs:
        ex.size_request(r)
    per = max(r.out_cap for r in reqs)
    limits = serve.SlotLimits(max_frames=16, out_bytes=2 * per, ws_bytes=1 << 24)
    res = serve.Scheduler(ex, 2, limits, clock=clock).run(reqs)
    assert all(r.status == 0 for r in res)
    budget = 2 * (limits.out_bytes + limits.ws_bytes)
    assert ex.max_in_flight_bytes <= budget
    assert all(sum(reqs[i].out_cap for i in ids) <= limits.out_bytes for _, ids, _ in ex.launches)


def test_oversized_request_is_rejected_not_blocking():
    clock = SimClock()
    ex = CpuExecutor(clock)
    reqs = _requests(6, rate=1e4)
    limits = serve.SlotLimits(max_frames=4, out_bytes=1, ws_bytes=1)
    res = serve.Scheduler(ex, 1, limits, clock=clock).run(reqs)
    assert all(r.status == -1 for r in res)


def test_summary_fields():
    clock = SimClock()
    ex = CpuExecutor(clock, bandwidth=5e6)
    reqs = _requests(20, rate=500.0)
    res = serve.Scheduler(ex, 2, serve.SlotLimits(8, 1 << 22, 1 << 22), clock=clock).run(reqs)
    s = serve.summarize(res, reqs)
    assert s["ok"] == 20 and s["p99_ms"] >= s["p50_ms"] > 0 and s["gbps"] > 0


def test_collector_off_during_run_and_restored():
    """The loop holds Python's cyclic collector off while it runs and puts
    it back as it was, also when the executor raises."""
    import gc

    class Probe(CpuExecutor):
        def launch(self, slot, batch, now):
            self.seen = gc.isenabled()
            return super().launch(slot, batch, now)

    class Failing(CpuExecutor):
        def launch(self, slot, batch, now):
            raise RuntimeError("launch failed")

    def run(ex_cls):
        clock = SimClock()   # the simulated executor counts time from 0
        ex = ex_cls(clock)
        serve.Scheduler(ex, 1, serve.SlotLimits(8, 1 << 24, 1 << 24), clock=clock).run(
            _requests(2, rate=100.0, seed=5))
        return ex

    assert gc.isenabled()
    assert run(Probe).seen is False and gc.isenabled()
    gc.disable()
    try:
        run(CpuExecutor)
        assert not gc.isenabled()   # left off, as the caller had it
    finally:
        gc.enable()
    try:
        run(Failing)
    except RuntimeError:
        pass
    assert gc.isenabled()
