"""Continuous-batching reconstruction server on one GPU.

Requests (one k-space frame each: trajectory key, data y, lambda, delta,
iteration budget) arrive as a stream.  Requests that share a trajectory share
a plan (phasor tables and Gram spectrum, built once by exact NUDFT sums,
Section 3.4 of the paper) and a slot pool: a workspace of B frame slots in
which frames start and finish at different iterations.  The scheduler

  * keeps a plan cache under an HBM byte budget (plan + pool workspace bytes
    from the library's size queries); an idle plan (no running or queued
    request) is evicted least-recently-used when a new one does not fit, and a
    request whose plan can never fit is rejected;
  * admits queued requests in arrival order into free slots of their plan's
    pool (adjoint b = A^H y and initial state for that slot);
  * advances every pool that has running slots by a chunk of iterations, cut
    short at the earliest slot budget so finished frames leave promptly;
  * retires finished slots (image copied out, statistics) and records their
    completion time from device events.

Every frame follows exactly the operations of a standalone solve of that
frame, so its result does not depend on what else is in the pool.

The executor interface keeps the scheduling logic free of device code; the
GPU executor drives the C ABI through paper_0908_3252_amd.recon.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, Hashable, List, Optional


@dataclasses.dataclass
class Request:
    id: int
    arrival: float              # seconds since the start of the run
    key: Hashable               # trajectory identity (requests with equal keys share a plan)
    y: Any                      # device data [M] (executor-specific)
    lam: float
    delta: float
    iters: int
    # filled in by the scheduler
    state: str = "future"       # future -> queued -> running -> done | rejected | cancelled
    slot: int = -1
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    x: Any = None               # result image (executor-specific)
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


class Executor:
    """What the scheduler needs from a device back end."""

    def plan_bytes(self, key) -> int:
        raise NotImplementedError

    def pool_bytes(self, key, slots: int) -> int:
        raise NotImplementedError

    def build_plan(self, key) -> Any:
        raise NotImplementedError

    def free_plan(self, plan) -> None:
        raise NotImplementedError

    def make_pool(self, plan, slots: int) -> Any:
        raise NotImplementedError

    def admit(self, pool, slot: int, req: Request) -> None:
        raise NotImplementedError

    def step(self, pool, iters: int) -> None:
        raise NotImplementedError

    def retire(self, pool, slot: int, req: Request) -> None:
        raise NotImplementedError

    def mark(self, pool) -> Any:
        """A completion marker for the work issued so far on the pool."""
        raise NotImplementedError

    def done(self, marker) -> bool:
        raise NotImplementedError

    def wait(self, marker) -> None:
        raise NotImplementedError

    def when(self, marker) -> float:
        """Run-relative time (s) at which a completed marker finished."""
        raise NotImplementedError


@dataclasses.dataclass
class _PoolState:
    key: Hashable
    plan: Any
    pool: Any
    slots: int
    iteration: int = 0
    stop_at: List[int] = dataclasses.field(default_factory=list)
    owner: List[Optional[Request]] = dataclasses.field(default_factory=list)
    last_use: float = 0.0
    # issued chunks not yet known complete: (marker, [requests finished by it], issue seq)
    inflight: collections.deque = dataclasses.field(default_factory=collections.deque)
    bytes: int = 0

    def running(self) -> int:
        return sum(1 for r in self.owner if r is not None)

    def free_slot(self) -> int:
        for i, r in enumerate(self.owner):
            if r is None:
                return i
        return -1


class Scheduler:
    """Plan cache + per-plan slot pools + chunked stepping (see module doc)."""

    def __init__(self, executor: Executor, hbm_budget: int, slots: int | Callable = 32,
                 chunk: int = 25, max_inflight: int = 2,
                 clock: Callable[[], float] = time.perf_counter):
        if chunk < 1:
            raise ValueError("chunk must be >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.slots = slots
        self.chunk = int(chunk)
        self.max_inflight = int(max_inflight)
        self.clock = clock
        self.t0 = None
        self.pools: Dict[Hashable, _PoolState] = collections.OrderedDict()
        self.used = 0
        self.queue: collections.deque = collections.deque()
        self.future: collections.deque = collections.deque()
        self.finished: List[Request] = []
        self.plans_built = 0
        self.plans_evicted = 0
        self._seq = 0

    # -- submission ---------------------------------------------------------
    def submit(self, reqs):
        """Requests with arrival times (s, relative to start()); kept sorted."""
        for r in sorted(reqs, key=lambda r: (r.arrival, r.id)):
            if r.iters < 0:
                raise ValueError("iteration budget must be >= 0")
            r.state = "future"
            self.future.append(r)

    def cancel(self, req: Request) -> bool:
        """Cancel a request that has not started; returns False otherwise."""
        if req.state == "future":
            self.future.remove(req)
        elif req.state == "queued":
            self.queue.remove(req)
        else:
            return False
        req.state = "cancelled"
        self.finished.append(req)
        return True

    def now(self) -> float:
        return self.clock() - self.t0

    def start(self):
        self.t0 = self.clock()

    # -- plan cache -----------------------------------------------------------
    def _slots_for(self, key) -> int:
        return int(self.slots(key) if callable(self.slots) else self.slots)

    def _cost(self, key) -> int:
        return int(self.ex.plan_bytes(key)) + int(self.ex.pool_bytes(key, self._slots_for(key)))

    def _idle(self, ps: _PoolState) -> bool:
        return ps.running() == 0 and not ps.inflight and \
            not any(r.key == ps.key for r in self.queue)

    def _evict(self, ps: _PoolState):
        del self.pools[ps.key]
        self.ex.free_plan(ps.plan)
        self.used -= ps.bytes
        self.plans_evicted += 1

    def _ensure_pool(self, key) -> Optional[_PoolState]:
        ps = self.pools.get(key)
        if ps is not None:
            return ps
        cost = self._cost(key)
        if cost > self.budget:
            return None  # can never fit: caller rejects
        while self.used + cost > self.budget:
            victims = [p for p in self.pools.values() if self._idle(p)]
            if not victims:
                return _WAIT
            self._evict(min(victims, key=lambda p: p.last_use))
        plan = self.ex.build_plan(key)
        slots = self._slots_for(key)
        pool = self.ex.make_pool(plan, slots)
        ps = _PoolState(key=key, plan=plan, pool=pool, slots=slots,
                        stop_at=[0] * slots, owner=[None] * slots, bytes=cost)
        self.pools[key] = ps
        self.used += cost
        self.plans_built += 1
        return ps

    # -- one scheduling round -------------------------------------------------
    def _arrivals(self, now: float):
        while self.future and self.future[0].arrival <= now:
            r = self.future.popleft()
            r.state = "queued"
            self.queue.append(r)

    def _admit(self, now: float) -> bool:
        progressed = False
        blocked = set()
        for r in list(self.queue):
            if r.key in blocked:
                continue  # keep arrival order within a plan
            ps = self._ensure_pool(r.key)
            if ps is None:
                self.queue.remove(r)
                r.state = "rejected"
                r.error = "plan and pool exceed the device memory budget"
                self.finished.append(r)
                progressed = True
                continue
            if ps is _WAIT:
                blocked.add(r.key)
                continue
            slot = ps.free_slot()
            if slot < 0:
                blocked.add(r.key)
                continue
            self.queue.remove(r)
            self.ex.admit(ps.pool, slot, r)
            r.state = "running"
            r.slot = slot
            r.t_admit = now
            ps.owner[slot] = r
            ps.stop_at[slot] = ps.iteration + r.iters
            ps.last_use = now
            progressed = True
        return progressed

    def _step(self, now: float) -> bool:
        progressed = False
        for ps in list(self.pools.values()):
            if ps.running() == 0:
                continue
            # slots whose budget is already used up (iters == 0) leave at once
            progressed |= self._retire_done(ps)
            live = [ps.stop_at[i] - ps.iteration for i, r in enumerate(ps.owner) if r is not None]
            if not live:
                continue
            # Stay at most max_inflight chunks ahead of the device, so that new
            # frames join the pool at the next chunk boundary rather than
            # behind a long run of already-issued iterations.
            while len(ps.inflight) >= self.max_inflight and self._drain_one(ps, block=False):
                pass
            if len(ps.inflight) >= self.max_inflight:
                continue
            n = min(self.chunk, min(live))
            self.ex.step(ps.pool, n)
            ps.iteration += n
            ps.last_use = now
            self._retire_done(ps, force_mark=True)
            progressed = True
        return progressed

    def _retire_done(self, ps: _PoolState, force_mark: bool = False) -> bool:
        fin = []
        for i, r in enumerate(ps.owner):
            if r is not None and ps.stop_at[i] <= ps.iteration:
                self.ex.retire(ps.pool, i, r)
                ps.owner[i] = None
                fin.append(r)
        if fin or force_mark:
            self._seq += 1
            ps.inflight.append((self.ex.mark(ps.pool), fin, self._seq))
        return bool(fin)

    def _drain_one(self, ps: _PoolState, block: bool) -> bool:
        if not ps.inflight:
            return False
        marker, reqs, _ = ps.inflight[0]
        if block:
            self.ex.wait(marker)
        elif not self.ex.done(marker):
            return False
        ps.inflight.popleft()
        t = self.ex.when(marker)
        for r in reqs:
            r.t_done = t
            r.state = "done"
            self.finished.append(r)
        return True

    def _collect(self) -> bool:
        progressed = False
        for ps in self.pools.values():
            while self._drain_one(ps, block=False):
                progressed = True
        return progressed

    def pending(self) -> bool:
        return bool(self.future or self.queue or
                    any(ps.running() or ps.inflight for ps in self.pools.values()))

    def tick(self) -> bool:
        """One scheduling round; True if anything was admitted, stepped or completed."""
        now = self.now()
        self._arrivals(now)
        progressed = self._admit(now)
        progressed |= self._step(now)
        progressed |= self._collect()
        return progressed

    def run(self, sleep: Callable[[float], None] = time.sleep):
        """Serve every submitted request; returns the finished list."""
        if self.t0 is None:
            self.start()
        while self.pending():
            if self.tick():
                continue
            inflight = [ps for ps in self.pools.values() if ps.inflight]
            if inflight:
                # wait for the oldest issued chunk
                self._drain_one(min(inflight, key=lambda p: p.inflight[0][2]), block=True)
            elif self.future:
                dt = self.future[0].arrival - self.now()
                if dt > 0:
                    sleep(dt)
            elif self.queue:
                raise RuntimeError("scheduler stalled: queued requests can never be admitted")
        return self.finished


class _Wait:
    def __repr__(self):
        return "WAIT"


_WAIT = _Wait()


def summarize(reqs: List[Request], t_first: float = 0.0) -> dict:
    """Throughput and latency percentiles of the completed requests whose
    arrival is at or after t_first (warm-up excluded)."""
    import numpy as np
    done = [r for r in reqs if r.state == "done" and r.arrival >= t_first]
    if not done:
        return dict(completed=0)
    lat = np.array([r.latency for r in done])
    t_begin = min(r.arrival for r in done)
    t_end = max(r.t_done for r in done)
    return dict(completed=len(done),
                rejected=sum(1 for r in reqs if r.state == "rejected"),
                recons_per_sec=len(done) / max(t_end - t_begin, 1e-9),
                p50_ms=1e3 * float(np.percentile(lat, 50)),
                p99_ms=1e3 * float(np.percentile(lat, 99)),
                mean_ms=1e3 * float(lat.mean()),
                max_ms=1e3 * float(lat.max()))


# ---------------------------------------------------------------------------
# GPU back end


class GpuExecutor(Executor):
    """Executor on the C ABI: one plan per trajectory key, one slot pool per
    plan, pools spread round-robin over a few HIP streams (default priority)
    so that pools of different plans overlap on the device."""

    def __init__(self, trajectories: Dict[Hashable, tuple], prec: Optional[int] = None,
                 phi: str = "hyperbolic", streams: int = 4):
        import torch
        from . import recon
        self.torch = torch
        self.recon = recon
        self.lib = recon.load()
        self.tr = trajectories          # key -> (k [M,2] float64, N, L)
        self.prec = recon.FP64 if prec is None else int(prec)
        self.phi = phi
        self.streams = [torch.cuda.Stream() for _ in range(max(1, int(streams)))]
        self._rr = 0
        self._t0_event = None
        self._t0_rel = 0.0
        self.plans: Dict[Hashable, Any] = {}

    # sizes from the library's queries
    def plan_bytes(self, key) -> int:
        k, N, L = self.tr[key]
        M = int(k.shape[0])
        return int(self.lib.recon_plan_bytes(M, N, L, self.prec) +
                   self.lib.recon_gram_workspace_bytes(M, N, L))

    def pool_bytes(self, key, slots: int) -> int:
        k, N, L = self.tr[key]
        return int(self.lib.recon_workspace_bytes(int(k.shape[0]), N, L, slots, self.prec)) + \
            slots * self.recon.STATS_DTYPE.itemsize

    def build_plan(self, key):
        plan = self.plans.get(key)
        if plan is None:
            k, N, L = self.tr[key]
            plan = self.recon.Plan(k, N, L, prec=self.prec)
            plan.gram_kernel()  # synchronises: the plan is ready for every stream
            plan.key = key
        return plan

    def keep_plan(self, key, plan):
        """Pre-built plan to hand out on build_plan(key) (a warm cache)."""
        plan.key = key
        self.plans[key] = plan

    def free_plan(self, plan) -> None:
        self.plans.pop(getattr(plan, "key", None), None)

    def make_pool(self, plan, slots: int):
        s = self.streams[self._rr % len(self.streams)]
        self._rr += 1
        return self.recon.Pool(plan, slots, self.phi, stream=s)

    def admit(self, pool, slot: int, req: Request) -> None:
        pool.admit(slot, req.y, req.lam, req.delta, req.iters)

    def step(self, pool, iters: int) -> None:
        pool.step(iters)

    def retire(self, pool, slot: int, req: Request) -> None:
        torch = self.torch
        N = pool.plan.N
        with torch.cuda.stream(pool.stream):
            req.x = torch.empty((N, N), dtype=torch.complex64, device="cuda")
            req.stats = torch.empty(self.recon.STATS_DTYPE.itemsize, dtype=torch.uint8,
                                    device="cuda")
        pool.retire(slot, req.x, stats_out=req.stats)

    def start_clock(self, rel_now: float):
        """Anchor device timestamps to the scheduler's clock."""
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.torch.cuda.current_stream())
        ev.synchronize()
        self._t0_event = ev
        self._t0_rel = rel_now

    def mark(self, pool):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(pool.stream)
        return ev

    def done(self, marker) -> bool:
        return bool(marker.query())

    def wait(self, marker) -> None:
        marker.synchronize()

    def when(self, marker) -> float:
        return self._t0_rel + self._t0_event.elapsed_time(marker) * 1e-3


def default_slots(key) -> int:
    """Slots per pool: enough frames per launch to fill the device at the
    smaller images, bounded for the larger ones."""
    N = key[0]
    return 64 if N <= 128 else 32 if N <= 256 else 16


def make_workload(count: int, seed: int = 4):
    """Requests of the serving workload with device-resident data.

    Request contents (trajectory key, phantom, noise, lambda, delta) do not
    depend on the arrival rate; arrival times are drawn at rate 1 and scaled
    by 1/rate per run (exponential gaps scale exactly that way).  Data
    synthesis: y = A x_true + sigma * noise with the library's forward model
    (one plan per trajectory, kept as the warm plan cache), sigma =
    c * max|A x_true|.  Returns (base requests, trajectories, plans).
    """
    import numpy as np
    import torch
    import synthetic
    from . import recon
    raw = synthetic.serving_requests(count, 1.0, seed)
    traj, plans = {}, {}
    for q in raw:
        key = (q["N"], q["I"])
        if key not in traj:
            k = synthetic.spiral_trajectory(q["N"], q["I"], q["S"], q["R"], "clv")
            traj[key] = (np.ascontiguousarray(k), q["N"], recon.default_L(q["N"]))
    for key, (k, N, L) in traj.items():
        plan = recon.Plan(k, N, L, prec=recon.FP64)
        plan.gram_kernel()
        plans[key] = plan
    base = []
    for q in raw:
        key = (q["N"], q["I"])
        x = torch.from_numpy(q["x_true"].astype(np.complex64)).cuda()[None]
        y0 = plans[key].forward(x)[0]
        sig = q["noise_c"] * float(y0.abs().max())
        nz = torch.from_numpy(q["noise"].astype(np.complex64)).cuda()
        base.append(dict(id=q["id"], arrival=q["arrival"], key=key,
                         y=(y0 + sig * nz).contiguous(), lam=q["lam"], delta=q["delta"],
                         iters=q["iters"]))
    torch.cuda.synchronize()
    return base, traj, plans


# fp64i: FP64 adjoint and FP64 iteration (state, FFTs, stencil, spectrum)
PRECS = {"fp64i": 3 | 16, "fp64": 3, "fp32": 0, "fp16x3": 2, "bf16x3": 1}


def serve(rate: float, workload, warmup_frac: float = 0.1, hbm_budget: Optional[int] = None,
          chunk: int = 25, streams: int = 4, verify: int = 3, seed: int = 4, prec: str = "fp64",
          reference: Optional[Dict[int, Any]] = None, keep_results: bool = False,
          log=None) -> dict:
    """Serve the workload's requests arriving at `rate` req/s on the GPU with
    plans of precision `prec`; returns throughput, p50/p99 latency (warm-up
    requests excluded), a check that `verify` served results equal
    standalone solves bitwise and, given `reference` (request id -> image of
    another run), the relative L2 distance of every result to it."""
    import numpy as np
    import torch
    base, traj, plans = workload
    reqs = [Request(id=b["id"], arrival=b["arrival"] / rate, key=b["key"], y=b["y"],
                    lam=b["lam"], delta=b["delta"], iters=b["iters"]) for b in base]
    ex = GpuExecutor(traj, prec=PRECS[prec], streams=streams)
    if PRECS[prec] == ex.recon.FP64:
        for key, plan in plans.items():
            ex.keep_plan(key, plan)
    else:  # plans of this precision, built before the clock starts
        for key in traj:
            ex.keep_plan(key, ex.build_plan(key))
    if hbm_budget is None:
        free, _total = torch.cuda.mem_get_info()
        hbm_budget = int(0.8 * free) + sum(ex.plan_bytes(k) for k in ex.plans)
    sched = Scheduler(ex, hbm_budget, slots=default_slots, chunk=chunk)
    sched.submit(reqs)
    sched.start()
    ex.start_clock(sched.now())
    done = sched.run()
    torch.cuda.synchronize()
    t_first = sorted(r.arrival for r in reqs)[int(warmup_frac * len(reqs))] if reqs else 0.0
    out = summarize(done, t_first)
    out.update(rate=rate, prec=prec, requests=len(reqs), plans_built=sched.plans_built,
               plans_evicted=sched.plans_evicted, chunk=chunk, streams=streams)
    st = [r for r in done if r.state == "done"]
    ok = 0
    if st:
        stats = np.frombuffer(torch.cat([r.stats for r in st]).cpu().numpy().tobytes(),
                              dtype=ex.recon.STATS_DTYPE)
        ok = int(np.sum(stats["status"] == 0))
    out["status_ok"] = ok
    if verify:
        rng = np.random.default_rng(seed)
        pick = rng.choice(len(st), size=min(verify, len(st)), replace=False) if st else []
        same = 0
        for i in pick:
            r = st[int(i)]
            plan = ex.build_plan(r.key)
            x1, _ = plan.solve(r.y[None], r.lam, r.delta, r.iters)
            torch.cuda.synchronize()
            same += int(torch.equal(x1[0].view(torch.float32), r.x.view(torch.float32)))
        out["bitwise_equal_standalone"] = f"{same}/{len(pick)}"
    if reference is not None:
        errs = []
        for r in st:
            xr = reference.get(r.id)
            if xr is not None:
                errs.append(float(torch.linalg.vector_norm(r.x - xr) /
                                  torch.linalg.vector_norm(xr)))
        if errs:
            out["rel_l2_vs_reference"] = {"median": float(np.median(errs)),
                                          "p99": float(np.percentile(errs, 99)),
                                          "max": float(np.max(errs)), "n": len(errs)}
    results = {r.id: r.x for r in st} if keep_results else None
    for r in reqs:  # release result buffers
        r.stats = None
        if not keep_results:
            r.x = None
    if log:
        log(f"rate {rate} prec {prec}: {out}")
    return (out, results) if keep_results else out


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="continuous-batching reconstruction server")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--precs", default="fp64i",
                    help="comma list of precisions (fp64i, fp64, fp32, fp16x3, bf16x3); with "
                         "several, each later one is compared with the first's results")
    ap.add_argument("--count", type=int, default=2200)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=25)
    ap.add_argument("--streams", type=int, default=4)
    args = ap.parse_args(argv)

    def log(m):
        print(f"[serve] {m}", file=sys.stderr, flush=True)

    log(f"synthesising {args.count} requests")
    wl = make_workload(args.count, args.seed)
    precs = args.precs.split(",")
    res = []
    for rate in [float(r) for r in args.rates.split(",")]:
        ref = None
        for i, prec in enumerate(precs):
            if len(precs) > 1 and i == 0:
                out, ref = serve(rate, wl, chunk=args.chunk, streams=args.streams,
                                 seed=args.seed, prec=prec, keep_results=True, log=log)
            else:
                out = serve(rate, wl, chunk=args.chunk, streams=args.streams, seed=args.seed,
                            prec=prec, reference=ref, log=log)
            res.append(out)
        ref = None
    print(json.dumps({"serving": res}), flush=True)


if __name__ == "__main__":
    main()
