"""CPU tests of the serving scheduler with a simulated engine and clock:
admission by slots and memory footprint, FIFO order, rejection, backfill."""
import numpy as np
import pytest

from paper_2108_12188_amd.serve import Request, Scheduler, summarize
from seminputs import arrival_times


class FakeEngine:
    """Processor sharing on a fake clock: every step advances time by dt and
    every active request by dt of its service time."""

    def __init__(self, dt=1e-3):
        self.t = 0.0
        self.dt = dt
        self.left = {}
        self.admitted = []
        self.max_active = 0

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def footprint(self, r):
        return r.n_elem * (r.order + 1) ** 3 * 100

    def admit(self, r):
        self.left[r.tag] = r.payload["service"]
        self.admitted.append(r.tag)
        self.max_active = max(self.max_active, len(self.left))

    def step(self):
        self.t += self.dt
        done = []
        for tag in list(self.left):
            self.left[tag] -= self.dt
            if self.left[tag] <= 1e-12:
                done.append((tag, {"converged": 1}))
                del self.left[tag]
        return done

    def release(self, tag):
        pass


def _requests(n=50, rate=200.0, seed=5):
    rng = np.random.default_rng(seed)
    t = arrival_times(n, rate, seed)
    out = []
    for q in range(n):
        E = int(rng.integers(8, 200))
        out.append(Request(tag=q, arrival=float(t[q]), n_elem=E, order=5,
                           payload={"service": 1e-3 * (1 + E // 20)}))
    return out


def test_all_complete_fifo_and_latency_bounds():
    eng = FakeEngine()
    reqs = _requests()
    sch = Scheduler(eng, budget_bytes=10 ** 12, max_slots=8)
    out = sch.run(reqs)
    assert all(r.status == "done" for r in out)
    assert eng.admitted == sorted(eng.admitted, key=lambda t: (reqs[t].arrival, t))
    for r in out:
        assert r.done - r.arrival >= r.payload["service"] - 1e-9
        assert r.admitted >= r.arrival
    assert eng.max_active <= 8
    s = summarize(out)
    assert s["completed"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0


def test_budget_is_never_exceeded():
    eng = FakeEngine()
    reqs = _requests(80, rate=1000.0)
    budget = 3 * max(eng.footprint(r) for r in reqs)
    sch = Scheduler(eng, budget_bytes=budget, max_slots=64)
    used = 0
    fp = {r.tag: eng.footprint(r) for r in reqs}
    out = sch.run(reqs)
    for kind, tag, _ in sch.log:
        used += fp[tag] if kind == "admit" else (-fp[tag] if kind == "done" else 0)
        assert used <= budget
    assert sch.peak_used <= budget
    assert all(r.status == "done" for r in out)


def test_oversized_request_is_rejected():
    eng = FakeEngine()
    reqs = _requests(10)
    reqs[3].n_elem = 10 ** 6
    sch = Scheduler(eng, budget_bytes=10 ** 9, max_slots=4)
    out = sch.run(reqs)
    assert out[[r.tag for r in out].index(3)].status == "rejected"
    assert sum(r.status == "done" for r in out) == 9


def test_backfill_admits_small_request_behind_blocked_head():
    eng = FakeEngine()
    big = Request(tag=0, arrival=0.0, n_elem=1000, order=5, payload={"service": 0.05})
    big2 = Request(tag=1, arrival=0.001, n_elem=1000, order=5, payload={"service": 0.05})
    small = Request(tag=2, arrival=0.002, n_elem=10, order=5, payload={"service": 0.001})
    budget = eng.footprint(big) + eng.footprint(small)
    for backfill, first_done in ((False, 0), (True, 2)):
        eng = FakeEngine()
        reqs = [Request(**{k: getattr(r, k) for k in ("tag", "arrival", "n_elem", "order",
                                                       "payload")}) for r in (big, big2, small)]
        sch = Scheduler(eng, budget_bytes=budget, max_slots=8, backfill=backfill)
        out = sch.run(reqs)
        order = [tag for kind, tag, _ in sch.log if kind == "done"]
        assert order[0] == first_done
        assert all(r.status == "done" for r in out)
