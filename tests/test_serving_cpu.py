"""Scheduler logic of the continuous-batching server, on the CPU.

A fake executor stands in for the device: it keeps, per pool, an iteration
counter and per-slot stop points exactly as the library does (a slot runs
iteration k only while k < stop_at), and a serial virtual clock.  The checks:
every request runs exactly its own budget whatever else shares its pool,
arrival order is kept within a plan, the plan cache respects the byte
budget (evicting idle plans), impossible plans are rejected, queued requests
can be cancelled, and a pool never holds more frames than its slots.
"""
import numpy as np
import pytest

from paper_0908_3252_amd.serving import Executor, Request, Scheduler, summarize


class FakePool:
    def __init__(self, key, slots):
        self.key = key
        self.slots = slots
        self.k = 0
        self.stop = [0] * slots
        self.count = [0] * slots   # iterations each slot actually ran
        self.busy = [False] * slots
        self.max_busy = 0
        self.markers = []


class FakeExec(Executor):
    def __init__(self, plan_cost=100, pool_cost=10, t_iter=1e-4, t_admit=1e-4,
                 t_build=1e-3):
        self.plan_cost = plan_cost
        self.pool_cost = pool_cost
        self.t_iter, self.t_admit, self.t_build = t_iter, t_admit, t_build
        self.vnow = 0.0       # virtual host clock
        self.gpu_free = 0.0   # virtual device: serial work queue
        self.resident = set()
        self.max_resident_bytes = 0
        self.builds = []
        self.admitted = []

    def clock(self):
        return self.vnow

    def sleep(self, dt):
        self.vnow += dt

    def _work(self, dt):
        self.gpu_free = max(self.gpu_free, self.vnow) + dt
        self.vnow += 1e-6  # host cost of a launch

    def plan_bytes(self, key):
        return self.plan_cost(key) if callable(self.plan_cost) else self.plan_cost

    def pool_bytes(self, key, slots):
        return self.pool_cost * slots

    def build_plan(self, key):
        self.builds.append(key)
        self.resident.add(key)
        used = sum(self.plan_bytes(k) + self.pool_bytes(k, 2) for k in self.resident)
        self.max_resident_bytes = max(self.max_resident_bytes, used)
        self._work(self.t_build)
        return key

    def free_plan(self, plan):
        self.resident.discard(plan)

    def make_pool(self, plan, slots):
        return FakePool(plan, slots)

    def admit(self, pool, slot, req):
        assert not pool.busy[slot], "admitted into a busy slot"
        pool.busy[slot] = True
        pool.stop[slot] = pool.k + req.iters
        pool.count[slot] = 0
        pool.max_busy = max(pool.max_busy, sum(pool.busy))
        self.admitted.append(req.id)
        self._work(self.t_admit)

    def step(self, pool, iters):
        # the host never runs more than max_inflight (2) chunks ahead
        assert sum(m > self.vnow for m in pool.markers) < 2
        for _ in range(iters):
            for s in range(pool.slots):
                if pool.k < pool.stop[s]:
                    pool.count[s] += 1
            pool.k += 1
        self._work(iters * self.t_iter)

    def retire(self, pool, slot, req):
        assert pool.k >= pool.stop[slot], "retired before its budget was used"
        req.x = (req.id, pool.count[slot])
        pool.busy[slot] = False

    def mark(self, pool):
        pool.markers.append(self.gpu_free)
        return self.gpu_free

    def done(self, marker):
        return self.vnow >= marker

    def wait(self, marker):
        self.vnow = max(self.vnow, marker)

    def when(self, marker):
        return marker


def make_reqs(n, keys, rate=1000.0, seed=0, iters=None):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        it = int(rng.integers(0, 60)) if iters is None else iters
        out.append(Request(id=i, arrival=float(t[i]), key=keys[i % len(keys)], y=None,
                           lam=0.01, delta=0.02, iters=it))
    return out


def run(ex, reqs, budget=10 ** 9, slots=4, chunk=7):
    s = Scheduler(ex, budget, slots=slots, chunk=chunk, clock=ex.clock)
    s.submit(reqs)
    done = s.run(sleep=ex.sleep)
    return s, done


def test_every_request_runs_exactly_its_budget():
    ex = FakeExec()
    reqs = make_reqs(200, ["a", "b", "c"])
    s, done = run(ex, reqs)
    assert len(done) == 200 and all(r.state == "done" for r in done)
    for r in done:
        assert r.x == (r.id, r.iters)
        assert r.t_done >= r.arrival and r.t_admit >= r.arrival
    assert s.plans_built == 3 and s.plans_evicted == 0


def test_zero_iteration_requests_complete():
    ex = FakeExec()
    reqs = make_reqs(10, ["a"], iters=0)
    _, done = run(ex, reqs)
    assert all(r.state == "done" and r.x == (r.id, 0) for r in done)


def test_arrival_order_within_a_plan():
    ex = FakeExec(t_iter=1e-3)  # slow device: queues build up
    reqs = make_reqs(120, ["a", "b"], rate=5000.0)
    _, done = run(ex, reqs, slots=3)
    for key in ("a", "b"):
        mine = [r for r in reqs if r.key == key]
        adm = [ex.admitted.index(r.id) for r in sorted(mine, key=lambda r: r.arrival)]
        assert adm == sorted(adm)


def test_pool_never_exceeds_its_slots():
    ex = FakeExec(t_iter=1e-3)
    reqs = make_reqs(60, ["a"], rate=1e4)
    s, done = run(ex, reqs, slots=2)
    assert all(r.state == "done" for r in done)
    assert max(ps.pool.max_busy for ps in s.pools.values()) <= 2


def test_plan_cache_budget_and_eviction():
    # room for exactly one plan + pool at a time
    ex = FakeExec(plan_cost=100, pool_cost=10)
    reqs = make_reqs(90, ["a", "b", "c"], rate=200.0)
    s, done = run(ex, reqs, budget=100 + 10 * 2, slots=2)
    assert all(r.state == "done" and r.x == (r.id, r.iters) for r in done)
    assert s.plans_evicted > 0 and s.plans_built == s.plans_evicted + len(s.pools)
    assert ex.max_resident_bytes <= 120
    assert s.used <= 120


def test_plan_that_can_never_fit_is_rejected():
    ex = FakeExec(plan_cost=lambda k: 10 ** 6 if k == "huge" else 100, pool_cost=10)
    reqs = make_reqs(30, ["a", "huge"])
    _, done = run(ex, reqs, budget=1000)
    for r in done:
        if r.key == "huge":
            assert r.state == "rejected" and r.error
        else:
            assert r.state == "done" and r.x == (r.id, r.iters)


def test_cancel_queued_request():
    ex = FakeExec()
    reqs = make_reqs(20, ["a"])
    s = Scheduler(ex, 10 ** 9, slots=2, chunk=5, clock=ex.clock)
    s.submit(reqs)
    assert s.cancel(reqs[7]) and reqs[7].state == "cancelled"
    done = s.run(sleep=ex.sleep)
    assert reqs[7].id not in ex.admitted
    assert sum(r.state == "done" for r in done) == 19
    assert not s.cancel(reqs[3])  # already finished


def test_results_do_not_depend_on_the_mix():
    # the same request alone and inside a busy mix runs the same iterations
    ex1 = FakeExec()
    alone = make_reqs(1, ["a"], iters=37)
    run(ex1, alone)
    ex2 = FakeExec()
    mix = make_reqs(50, ["a"], iters=None, seed=3)
    mix[20].iters = 37
    run(ex2, mix, slots=5, chunk=4)
    assert alone[0].x[1] == mix[20].x[1] == 37


def test_summary_percentiles():
    ex = FakeExec()
    reqs = make_reqs(100, ["a", "b"])
    _, done = run(ex, reqs)
    out = summarize(done, t_first=reqs[10].arrival)
    assert out["completed"] == 90
    assert 0 < out["p50_ms"] <= out["p99_ms"] <= out["max_ms"]
    assert out["recons_per_sec"] > 0


def test_negative_budget_refused():
    s = Scheduler(FakeExec(), 10 ** 9)
    with pytest.raises(ValueError):
        s.submit([Request(id=0, arrival=0.0, key="a", y=None, lam=0.0, delta=1.0, iters=-1)])
