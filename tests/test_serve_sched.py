"""The serving scheduler on a fake device: a virtual clock advanced by a
cost model (cell-updates / rate + per-tick overhead), no GPU."""
import numpy as np
import pytest

from paper_1301_4539_amd import serve, workload as W


class Fake:
    def __init__(self, rate=1e9, overhead=1e-3, fail_once=()):
        self.t = 0.0
        self.rate, self.overhead = rate, overhead
        self.fail_once = set(fail_once)
        self.live = {}
        self.max_live = 0
        self.max_bytes = 0
        self.order = []

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def footprint(self, req):
        return req.nx * req.ny * req.nz * 49

    def create(self, req):
        if req.rid in self.fail_once:
            self.fail_once.discard(req.rid)
            raise serve.AdmissionError("fake allocation failure")
        self.live[req.rid] = self.footprint(req)
        self.max_live = max(self.max_live, len(self.live))
        self.max_bytes = max(self.max_bytes, sum(self.live.values()))
        self.order.append(req.rid)
        return req

    def step(self, handles, counts):
        self.t += self.overhead + sum(h.nx * h.ny * h.nz * c for h, c in zip(handles, counts)) / self.rate

    def sync(self):
        pass

    def finish(self, h, req):
        del self.live[req.rid]
        return np.full((req.n_steps, 8), float(req.rid))


def _reqs(n=40, rate=20.0, seed=5):
    return W.serving_requests(n=n, rate=rate, seed=seed, dim_lo=16, dim_hi=48, steps_lo=20, steps_hi=200)


def test_all_complete_in_arrival_order_within_limits():
    reqs = _reqs()
    fake = Fake()
    budget = 6 * 48 ** 3 * 49
    rep = serve.Engine(fake, budget_bytes=budget, max_slots=4, chunk=16).run(reqs)
    assert not rep.rejected
    assert all(np.isfinite(r.finished) for r in rep.records)
    assert fake.order == [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert fake.max_live <= 4 and fake.max_bytes <= budget
    for r, q in zip(rep.records, sorted(reqs, key=lambda r: r.rid)):
        assert r.admitted >= q.arrival - 1e-12
        assert r.finished >= r.admitted + q.nx * q.ny * q.nz * q.n_steps / fake.rate - 1e-9
        assert r.probes.shape == (q.n_steps, 8) and r.probes[0, 0] == q.rid
    s = rep.summary()
    lat = rep.latencies()
    assert s["p50_s"] == float(np.percentile(lat, 50)) and s["p99_s"] == float(np.percentile(lat, 99))
    assert s["requests"] == len(reqs)


def test_continuous_batching_admits_while_others_run():
    """A short request arriving while a long one runs joins at the next tick
    and finishes first (not a run-to-completion queue)."""
    long = W.Request(0, 0.0, 48, 48, 48, 5, 2000, W.FP32)
    short = W.Request(1, 0.01, 16, 16, 16, 5, 40, W.FP32)
    fake = Fake(rate=1e9)
    rep = serve.Engine(fake, budget_bytes=1 << 40, max_slots=8, chunk=32).run([long, short])
    r0, r1 = rep.records
    assert r1.admitted < r0.finished
    assert r1.finished < r0.finished


def test_allocation_failure_requeues():
    reqs = _reqs(n=10)
    fake = Fake(fail_once={3, 7})
    rep = serve.Engine(fake, budget_bytes=1 << 40, max_slots=3, chunk=16).run(reqs)
    assert all(np.isfinite(r.finished) for r in rep.records)
    assert rep.records[3].requeues == 1 and rep.records[7].requeues == 1
    assert rep.summary()["requeues"] == 2


def test_oversized_request_is_rejected_not_blocking():
    reqs = [W.Request(0, 0.0, 100, 100, 100, 5, 10, W.FP32), W.Request(1, 0.0, 10, 10, 10, 5, 10, W.FP32)]
    fake = Fake()
    rep = serve.Engine(fake, budget_bytes=10 ** 6, max_slots=2, chunk=8).run(reqs)
    assert rep.rejected == [0]
    assert np.isfinite(rep.records[1].finished)


def test_budget_limits_concurrency():
    reqs = [W.Request(i, 0.0, 32, 32, 32, 5, 64, W.FP32) for i in range(6)]
    fake = Fake()
    fp = 32 ** 3 * 49
    rep = serve.Engine(fake, budget_bytes=2 * fp, max_slots=64, chunk=16).run(reqs)
    assert fake.max_live == 2
    assert all(np.isfinite(r.finished) for r in rep.records)


def test_long_waiting_solves_get_larger_steps():
    """A solve that has waited longer than age_step is advanced by two chunks
    per tick, and never by more than max_boost chunks; every count is a
    multiple of the chunk until the solve's last tick."""
    long = W.Request(0, 0.0, 40, 40, 40, 5, 3000, W.FP32)
    fake = Fake(rate=1e8)
    counts = []
    step = fake.step

    def record(handles, cs):
        counts.append(list(cs))
        step(handles, cs)
    fake.step = record
    serve.Engine(fake, budget_bytes=1 << 40, max_slots=4, chunk=16, age_step=0.05, max_boost=3).run([long])
    flat = [c[0] for c in counts]
    assert flat[0] == 16 and max(flat) == 48 and 32 in flat
    assert all(c % 16 == 0 for c in flat[:-1]) and sum(flat) == 3000


class PipedFake(Fake):
    """A fake with a device timeline: submit() queues a tick behind the
    previous one (device time = cells / rate), host calls cost `host` each;
    wait() advances the host clock to the tick's end."""

    def __init__(self, host=2e-3, **kw):
        super().__init__(**kw)
        self.host = host
        self.dev_end = 0.0
        self.dev_busy = 0.0

    def create(self, req):
        self.t += self.host
        return super().create(req)

    def submit(self, handles, counts):
        cost = self.overhead + sum(h.nx * h.ny * h.nz * c for h, c in zip(handles, counts)) / self.rate
        start = max(self.dev_end, self.t)
        self.dev_end = start + cost
        self.dev_busy += cost
        self.t += self.host
        return (start, self.dev_end)

    def wait(self, token):
        self.t = max(self.t, token[1])
        return token[1] - token[0]


def test_pipelined_ticks_keep_the_device_busy():
    """With the next tick queued before the engine waits for the current one,
    host work (admission, read-back) hides behind device work: the device is
    busy nearly all the time some solve is pending, where the tick-by-tick
    loop leaves it idle for the host's share; every request completes and
    gets the probes of its own solve."""
    reqs = W.serving_requests(n=60, rate=200.0, seed=9, dim_lo=40, dim_hi=64, steps_lo=100, steps_hi=400)
    slow_host = dict(rate=2e9, overhead=1e-4)
    piped = PipedFake(host=3e-3, **slow_host)
    rep = serve.Engine(piped, budget_bytes=1 << 40, max_slots=8, chunk=16).run(reqs)
    s = rep.summary()
    assert s["requests"] == 60 and not rep.rejected
    assert all(np.all(r.probes == r.rid) for r in rep.records)
    assert s["busy_while_pending"] > 0.9
    # the same trace tick by tick: the host's time per tick is device idle time
    plain = Fake(**slow_host)
    plain.t = 0.0
    rep2 = serve.Engine(plain, budget_bytes=1 << 40, max_slots=8, chunk=16).run(reqs)
    assert rep2.summary()["requests"] == 60
