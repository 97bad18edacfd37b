"""Serving loop: many independent solve-plus-gradient requests on one GPU.

A request is one simulation (its own size, amplitude, step count T) that has to be rolled
out for T fixed steps with a checkpoint every K steps and then differentiated: the loss is
sum_i |v_i(T)|^2 and the answer is the cotangent of the initial state (x0, v0, rho0), as in
the checkpointed scheme of Sec. 3.3 (store every K-th state, recompute the rest).

The scheduler works in ticks.  Within a tick a request advances by one checkpoint segment:
in its forward phase it steps to its next checkpoint boundary, in its backward phase it runs
the adjoint of one segment (recompute it from its checkpoint, then its adjoint steps in
reverse).  Requests in the same phase, of the same dimension and with the same segment
length are packed back to back into one batched plan (one library call per group), so the
batch changes at every segment boundary: requests join as soon as they are admitted and
leave as soon as their gradient is done (continuous batching).  Which requests take part in
a tick is decided by cost-fair sharing (see Scheduler).  Admission is first-come first-served under an HBM budget: a request
is admitted when its footprint (its states, checkpoints and cotangent plus the workspace of
a plan of its size) fits beside the requests already running; the head of the queue is
always admitted into an empty server so that every request makes progress.

2D neighbour lists are rebuilt every R steps (the largest R <= 8 dividing K, so every segment
starts with a build) with a skin per request that covers R steps at 1.3 times the largest speed
of its initial state; 3D lists are rebuilt every step.  The plain path uses the same settings.

The segment boundaries of a request are the same (every K steps from its step 0, the last
segment possibly shorter) whether it runs alone or in a mix, and the library's results do
not depend on the batch composition, so a served request returns bitwise the gradient that
the plain path (one plan per request, sph_step with checkpoints then sph_rollout_backward)
returns.

Time is kept on a clock that advances by the measured wall time of each tick and jumps to
the next arrival when the server is idle; latency of a request is its completion time minus
its arrival time on that clock.  The plain path is timed per request (service time) and its
first-come first-served latencies follow from the same arrival times.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from .inputs import Request


@dataclass
class Job:
    req: Request
    footprint: int
    state: object = None                       # engine-owned current state (forward phase)
    ckpts: List[object] = field(default_factory=list)
    cot: object = None                         # engine-owned cotangent (backward phase)
    pos: int = 0                               # forward steps done
    seg: int = -1                              # next backward segment
    phase: str = "fwd"
    admitted: float = math.nan
    finished: float = math.nan
    error: int = 0                             # device status word if the request failed
    vtime: float = 0.0                         # estimated device time received so far
    large: bool = False                        # served one at a time, in admission order
    promoted: bool = False                     # a large request whose turn has come

    @property
    def dim(self) -> int:
        return self.req.spec.dim

    def seg_len(self, K: int) -> int:
        """Length of the segment this job works on next."""
        T = self.req.steps
        if self.phase == "fwd":
            return min(K, T - self.pos)
        return min(K, T - self.seg * K)


class Scheduler:
    """First-come first-served admission under a byte budget; continuous batching by segment
    with cost-fair sharing of the device.

    Every admitted request carries a virtual time: the estimated device time of the segments it
    has run so far (engine.segment_cost).  Each tick runs one segment of every request whose
    virtual time is within `quantum` seconds of the smallest one, grouped into batched calls by
    (phase, dimension, segment length).  A request that has just run an expensive segment (a
    large 3D simulation) therefore sits out while cheaper ones catch up, so small requests are
    not held at the pace of the largest one, and the largest one still gets its share.  A request
    admitted mid-way starts at the current smallest virtual time.

    Fair sharing alone stretches the largest requests: they share the device with every request
    that arrives during their long lives, and with each other, which sets the tail of the latency
    distribution.  Two rules bound that stretch:
    * A request whose estimated cost exceeds `large_factor` times the mean estimated cost of the
      requests admitted so far is large.  Large requests take part in the sharing one at a time,
      in admission order, so several large requests do not all finish at the end of their
      combined work; small ones still share the device with the one that runs.  A waiting large
      request is left out of the smallest virtual time that newcomers start from, and when its
      turn comes it starts from the smallest virtual time of the others.
    * A request that has waited longer than a grace period gains priority: its sharing key is
      vtime - age_weight * (age - grace), with the age converted to estimated device time (by
      the ratio of the estimated to the measured time of the ticks so far) and the grace equal
      to `age_after` mean estimated costs.  Small requests finish well within the grace.
    With large_factor = 0 and age_weight = 0 the scheduler is plain cost-fair sharing.

    The engine supplies footprint(req), segment_cost(job, n), admit(job), forward(jobs, n),
    backward(jobs, n), finish(jobs) and sync(); sync() ends a tick and may return {rid: status}
    for requests whose device status reports a failure (non-finite values, list overflow):
    those leave the server at once with job.error set.  The scheduler owns the clock and the
    queues and never touches device memory itself.

    An engine with `lookahead` = 1 (and a drain() method) lets its device run one tick behind the
    host: sync() of tick t waits only for tick t - 1 and reports its failures, so the host work
    of a tick (deciding, packing, enqueueing) overlaps the device work of the previous one.  A
    request whose last segment ran in tick t is then finished (finish(), completion time, budget
    released) when tick t is known to be complete, at the end of tick t + 1 or at drain().
    """

    def __init__(self, engine, ckpt_every: int = 8, budget_bytes: int = 64 << 30,
                 clock: Optional[Callable[[], float]] = None, quantum: float = 5e-3,
                 progress: Optional[Callable[[str], None]] = None, progress_every: float = 10.0,
                 large_factor: float = 5.0, age_weight: float = 0.5, age_after: float = 16.0):
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1")
        self.engine = engine
        self.K = int(ckpt_every)
        self.budget = int(budget_bytes)
        self.clock_fn = clock if clock is not None else time.perf_counter
        self.quantum = float(quantum)
        self.age_weight = float(age_weight)
        self.age_after = float(age_after)
        self.large_factor = float(large_factor)
        self.est_total = 0.0        # estimated device time of the ticks run so far
        self.wall_total = 0.0       # their measured time
        self.cost_sum = 0.0         # estimated cost of the requests admitted so far
        self.admitted_count = 0
        self.now = 0.0
        self.used = 0
        self.peak_used = 0
        self.ticks = 0
        self.batch_sizes: List[int] = []
        self.progress = progress
        self.progress_every = progress_every

    def _request_cost(self, j: Job) -> float:
        """Estimated device time of a whole request: all its forward and backward steps."""
        phase = j.phase
        j.phase = "fwd"
        c = self.engine.segment_cost(j, j.req.steps)
        j.phase = "bwd"
        c += self.engine.segment_cost(j, j.req.steps)
        j.phase = phase
        return c

    @staticmethod
    def _sharing(active: Sequence[Job]) -> List[Job]:
        """The requests that share the device now: every small one and the first large one (by
        admission).  A large request that becomes first after waiting starts from the smallest
        virtual time of the others, so it joins the sharing instead of running alone until its
        frozen virtual time catches up."""
        large = [j for j in active if j.large]
        if not large:
            return list(active)
        first = min(large, key=lambda j: (j.admitted, j.req.rid))
        cand = [j for j in active if not j.large or j is first]
        if not first.promoted:
            first.promoted = True
            others = [j.vtime for j in cand if j is not first]
            if others:
                first.vtime = max(first.vtime, min(others))
        return cand

    def _groups(self, jobs: Sequence[Job]) -> Dict[Tuple[str, int, int], List[Job]]:
        groups: Dict[Tuple[str, int, int], List[Job]] = {}
        for j in jobs:
            groups.setdefault((j.phase, j.dim, j.seg_len(self.K)), []).append(j)
        return groups

    def _finalize(self, jobs: List[Job], done: List[Job]) -> None:
        if jobs:
            self.engine.finish(jobs)
        for j in jobs:
            j.finished = self.now
            self.used -= j.footprint
            done.append(j)

    @staticmethod
    def _mark_failed(failed: Dict[int, int], jobs) -> None:
        for j in jobs:
            if j.req.rid in failed:
                j.error = int(failed[j.req.rid])
                j.phase = "done"

    def run(self, trace: Sequence[Request]) -> List[Job]:
        pending = deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
        queue: deque = deque()
        active: List[Job] = []
        done: List[Job] = []
        K = self.K
        lag = int(getattr(self.engine, "lookahead", 0))
        inflight: deque = deque()   # per tick the device may still be running: its finished jobs

        def drain():
            # the device finishes the ticks still running; the wait is device time on the clock
            t0 = self.clock_fn()
            failed = self.engine.drain() or {}
            self.wall_total += self.clock_fn() - t0
            self.now += self.clock_fn() - t0
            waiting = [j for batch in inflight for j in batch]
            self._mark_failed(failed, waiting + active)
            self._finalize(waiting, done)
            inflight.clear()

        last_report = time.perf_counter()
        while pending or queue or active:
            if self.progress is not None and time.perf_counter() - last_report > self.progress_every:
                last_report = time.perf_counter()
                self.progress("serving: tick %d, clock %.2f s, done %d, active %d, queued %d, pending %d"
                              % (self.ticks, self.now, len(done), len(active), len(queue), len(pending)))
            while pending and pending[0].arrival <= self.now:
                r = pending.popleft()
                queue.append(Job(r, int(self.engine.footprint(r))))
            if not queue and not active:
                if inflight:
                    drain()
                self.now = max(self.now, pending[0].arrival)
                continue
            # new requests start at the smallest virtual time among the requests that may run
            # now: a large request waiting for its turn keeps a frozen, lower virtual time and
            # is left out, so that newcomers do not start below the running set and run alone
            vmin = min((j.vtime for j in self._sharing(active)), default=0.0)
            while queue and (self.used + queue[0].footprint <= self.budget or not active):
                j = queue.popleft()
                self.used += j.footprint
                self.peak_used = max(self.peak_used, self.used)
                j.admitted = self.now
                j.vtime = vmin
                rc = self._request_cost(j)
                self.cost_sum += rc
                self.admitted_count += 1
                j.large = self.large_factor > 0 and rc > self.large_factor * self.cost_sum / self.admitted_count
                active.append(j)
            rate = self.est_total / self.wall_total if self.wall_total > 0 else 1.0
            grace = self.age_after * self.cost_sum / max(1, self.admitted_count)
            key = {id(j): j.vtime - self.age_weight * max(0.0, rate * (self.now - j.admitted) - grace)
                   for j in active}
            cand = self._sharing(active)
            kmin = min(key[id(j)] for j in cand)
            runnable = [j for j in cand if key[id(j)] <= kmin + self.quantum]
            t0 = self.clock_fn()
            for j in [j for j in runnable if j.state is None and j.phase == "fwd" and j.pos == 0]:
                self.engine.admit(j)
            groups = self._groups(runnable)
            for (phase, _, n), jobs in sorted(groups.items(), key=lambda kv: kv[0]):
                for j in jobs:
                    c = self.engine.segment_cost(j, n)
                    j.vtime += c
                    self.est_total += c
                if phase == "fwd":
                    self.engine.forward(jobs, n)
                    for j in jobs:
                        j.pos += n
                        if j.pos == j.req.steps:
                            j.phase = "bwd"
                            j.seg = (j.req.steps + K - 1) // K - 1
                else:
                    self.engine.backward(jobs, n)
                    for j in jobs:
                        j.seg -= 1
                        if j.seg < 0:
                            j.phase = "done"
            failed = self.engine.sync() or {}
            self._mark_failed(failed, active + [j for batch in inflight for j in batch])
            self.wall_total += self.clock_fn() - t0
            self.now += self.clock_fn() - t0
            self.ticks += 1
            self.batch_sizes.append(len(runnable))
            inflight.append([j for j in active if j.phase == "done"])
            active = [j for j in active if j.phase != "done"]
            while len(inflight) > lag:
                self._finalize(inflight.popleft(), done)
        if inflight:
            drain()
        return done


def fifo_latencies(arrivals: Sequence[float], service: Sequence[float]) -> np.ndarray:
    """Latencies of a single first-come first-served server with the given service times."""
    free = 0.0
    out = np.empty(len(arrivals))
    for k, (a, s) in enumerate(zip(arrivals, service)):
        start = max(a, free)
        free = start + s
        out[k] = free - a
    return out


def percentiles(lat_s: Sequence[float]) -> Dict[str, float]:
    a = np.asarray(lat_s, dtype=np.float64)
    if a.size == 0:
        return {"p50_ms": math.nan, "p99_ms": math.nan, "mean_ms": math.nan}
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "mean_ms": float(a.mean() * 1e3)}


# ---------------------------------------------------------------- GPU engine

def rebuild_intervals(ckpt_every: int, reuse: int = 8) -> Dict[int, int]:
    """List rebuild interval per dimension for served requests (and their plain-path twins)."""
    from .autotune import rebuild_for
    return {2: rebuild_for(ckpt_every, reuse), 3: rebuild_for(ckpt_every, min(reuse, 2))}


class GpuEngine:
    """Runs the scheduler's groups through batched plans of the HIP library.

    The device runs one tick behind the host (lookahead = 1): nothing in a tick waits for the
    device except sync(), which waits for the previous tick only.  Admission copies the
    request's initial state from page-locked host memory without waiting, and the status words
    and pair counts of every plan a tick used are read with sph_poll_async into page-locked
    buffers that are examined once that tick is complete."""

    lookahead = 1

    def __init__(self, dtype: str = "f32", ckpt_every: int = 8, device=None, tuned: bool = True,
                 reuse: int = 8):
        import torch
        self.torch = torch
        self.dtype = dtype
        self.tdt = torch.float32 if dtype == "f32" else torch.float64
        self.K = int(ckpt_every)
        # neighbour lists rebuilt every R steps (R divides K, so segments start with a build),
        # each request's skin from the largest speed of its own initial state; 3D lists every
        # second step at most, which keeps the 3D skin near 0.13 H at the largest amplitudes
        # (a skinned 3D list grows as (1 + skin)^3 and its sweeps with it)
        self.R = rebuild_intervals(self.K, reuse)
        self._skin: Dict[int, float] = {}
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.tuned = tuned
        self._plans: Dict[tuple, object] = {}
        self._used_plans: Dict[tuple, object] = {}
        self._ws_cache: Dict[tuple, int] = {}
        self.pairs = 0
        self.results: Dict[int, tuple] = {}
        self._host: Dict[int, list] = {}
        self._members: Dict[tuple, List[int]] = {}
        self.plan_seconds = 0.0         # host time spent creating and binding plans
        self._keep: List[object] = []   # page-locked sources of this tick's host-to-device copies
        self._ticks: deque = deque()    # ticks the device may still run: (event, readouts, sources)

    # -- accounting
    def workspace_bytes(self, spec) -> int:
        return self.workspace_bytes_skin(spec, 0.0)

    def workspace_bytes_skin(self, spec, skin: float) -> int:
        from .lib import workspace_bytes
        key = (spec.dim, spec.side, round(skin, 6))
        if key not in self._ws_cache:
            self._ws_cache[key] = workspace_bytes([spec.params()], [spec.n], self.dtype, self.K, skin=skin)
        return self._ws_cache[key]

    def footprint(self, req: Request) -> int:
        """Bytes the request holds while admitted.  Called when the request arrives, which is
        also when its initial state (the request's payload) is generated on the host."""
        from .inputs import make_state
        npdt = np.float32 if self.dtype == "f32" else np.float64
        from .autotune import skin_from_speed
        host = [a.astype(npdt) for a in make_state(req.spec, req.seed)]
        self._host[req.rid] = host
        vmax = float(np.sqrt((host[1].astype(np.float64) ** 2).sum(axis=0)).max())
        self._skin[req.rid] = skin_from_speed(vmax, req.spec.params(), self.R[req.spec.dim])
        spec = req.spec
        esz = 4 if self.dtype == "f32" else 8
        state = (2 * spec.dim + 1) * spec.n * esz
        nseg = (req.steps + self.K - 1) // self.K
        # checkpoints, current state, cotangent, and packed copies of both for a group call
        return (nseg + 4) * state + self.workspace_bytes_skin(spec, self._skin[req.rid])

    # neighbours per particle (self excluded) on the jittered lattices, and the cost model of
    # one simulation step used for fair sharing: a fixed launch cost per step plus the pair
    # interactions at a nominal rate; a backward step (recompute + adjoint) costs 2.5 forward
    NEIGHBOURS = {2: 47.0, 3: 256.0}
    STEP_LAUNCH_S = 60e-6
    PAIRS_PER_S = 100e9

    def segment_cost(self, job: Job, n: int) -> float:
        per_step = self.STEP_LAUNCH_S + job.req.spec.n * self.NEIGHBOURS[job.dim] / self.PAIRS_PER_S
        return n * per_step * (1.0 if job.phase == "fwd" else 2.5)

    # -- plans
    def _plan(self, key, jobs: Sequence[Job], tape: int):
        from .lib import Plan
        p = self._plans.get(key)
        if p is None:
            t0 = time.perf_counter()
            p = Plan([j.req.spec.params() for j in jobs], [j.req.spec.n for j in jobs], dtype=self.dtype,
                     tape_depth=tape, device=self.device, skin=[self._skin[j.req.rid] for j in jobs],
                     rebuild_every=self.R[jobs[0].dim], speed_skins=self.R[jobs[0].dim] > 1)
            if self.tuned:
                from .autotune import apply_cached
                apply_cached(p)
            self._plans[key] = p
            self.plan_seconds += time.perf_counter() - t0
        self._used_plans[key] = p
        self._members[key] = [j.req.rid for j in jobs]
        return p

    def _pack(self, parts: Sequence[tuple]):
        torch = self.torch
        if len(parts) == 1:
            return tuple(t.clone() for t in parts[0])
        return (torch.cat([p[0] for p in parts], 1), torch.cat([p[1] for p in parts], 1),
                torch.cat([p[2] for p in parts], 0))

    @staticmethod
    def _unpack(packed: tuple, jobs: Sequence[Job]) -> List[tuple]:
        out, a = [], 0
        for j in jobs:
            b = a + j.req.spec.n
            out.append((packed[0][:, a:b].contiguous(), packed[1][:, a:b].contiguous(),
                        packed[2][a:b].contiguous()))
            a = b
        return out

    # -- scheduler hooks
    def admit(self, job: Job):
        host = self._host.pop(job.req.rid)
        pinned = [self.torch.from_numpy(a).pin_memory() for a in host]
        job.state = tuple(t.to(self.device, non_blocking=True) for t in pinned)
        self._keep.extend(pinned)

    def forward(self, jobs: Sequence[Job], n: int):
        key = ("fwd", jobs[0].dim) + tuple(j.req.rid for j in jobs)
        plan = self._plan(key, jobs, 0)
        for j in jobs:
            j.ckpts.append(j.state)                     # the state at the start of this segment
        xs, vs, rs = self._pack([j.state for j in jobs])
        plan.step(xs, vs, rs, n)
        for j, st in zip(jobs, self._unpack((xs, vs, rs), jobs)):
            j.state = st
            if j.pos + n == j.req.steps:
                # loss sum_i |v_i(T)|^2: seed v-bar = 2 v(T), x-bar = rho-bar = 0
                j.cot = (self.torch.zeros_like(st[0]), 2.0 * st[1], self.torch.zeros_like(st[2]))
                j.state = None

    def backward(self, jobs: Sequence[Job], n: int):
        key = ("bwd", jobs[0].dim) + tuple(j.req.rid for j in jobs)
        plan = self._plan(key, jobs, self.K)
        ck = self._pack([j.ckpts[j.seg] for j in jobs])
        gx, gv, gr = self._pack([j.cot for j in jobs])
        plan.rollout_backward([ck], n, n, gx, gv, gr)
        for j, c in zip(jobs, self._unpack((gx, gv, gr), jobs)):
            j.cot = c
            j.ckpts[j.seg] = None

    def finish(self, jobs: Sequence[Job]):
        for j in jobs:
            self.results[j.req.rid] = None if j.error else j.cot
            j.cot = None
            j.ckpts = []

    def sync(self):
        """End the tick: enqueue the status reads of its plans, then wait for the previous tick
        and return the failures it reported."""
        torch = self.torch
        used = list(self._used_plans.items())
        total = sum(p.nsims for _, p in used)
        status = torch.empty(max(total, 1), dtype=torch.int32, pin_memory=True)
        pairs = torch.empty(max(len(used), 1), dtype=torch.int64, pin_memory=True)
        reads, a = [], 0
        for k, (key, p) in enumerate(used):
            p.poll_async(status[a:a + p.nsims], pairs[k:k + 1])
            reads.append((key[0], list(self._members[key]), a, p.nsims, k))
            a += p.nsims
        ev = torch.cuda.Event()
        ev.record()
        self._ticks.append((ev, reads, status, pairs, self._keep))
        self._keep = []
        failed = {}
        while len(self._ticks) > self.lookahead:
            failed.update(self._complete(self._ticks.popleft()))
        # plans not used in this tick belong to compositions that no longer exist (the ticks
        # that used them are complete)
        self._plans = dict(self._used_plans)
        self._members = {k: self._members[k] for k in self._plans}
        self._used_plans = {}
        return failed

    def drain(self):
        """Wait for every tick still running; their failures."""
        failed = {}
        while self._ticks:
            failed.update(self._complete(self._ticks.popleft()))
        return failed

    def _complete(self, tick) -> Dict[int, int]:
        # work is counted on the forward states only (each is also the start of one adjoint
        # step); the recompute builds of the backward plans are not work and are discarded
        ev, reads, status, pairs, _sources = tick
        ev.synchronize()
        st, pr = status.numpy(), pairs.numpy()
        failed = {}
        for phase, members, a, n, k in reads:
            if phase == "fwd":
                self.pairs += int(pr[k])
            for rid, word in zip(members, st[a:a + n]):
                if word:
                    failed[rid] = int(word)
        for rid in failed:
            self.results[rid] = None
        return failed


def serve(trace: Sequence[Request], dtype: str = "f32", ckpt_every: int = 8, budget_bytes: int = 64 << 30,
          device=None, tuned: bool = True, progress: Optional[Callable[[str], None]] = None,
          quantum: float = 5e-3, reuse: int = 8, **policy):
    """Serve `trace` with continuous batching; returns (scheduler, engine, finished jobs).
    `policy` holds the Scheduler's sharing options."""
    eng = GpuEngine(dtype, ckpt_every, device, tuned, reuse)
    sch = Scheduler(eng, ckpt_every, budget_bytes, quantum=quantum, progress=progress, **policy)
    done = sch.run(trace)
    return sch, eng, done


def plain_request(req: Request, dtype: str = "f32", ckpt_every: int = 8, device=None, tuned: bool = True,
                  reuse: int = 8):
    """The plain path for one request: its own plan, sph_step with checkpoints, sph_rollout_backward.

    Returns (service seconds, gradient tuple)."""
    import torch
    from .inputs import make_state
    from .lib import Plan
    spec = req.spec
    npdt = np.float32 if dtype == "f32" else np.float64
    host = [a.astype(npdt) for a in make_state(spec, req.seed)]
    from .autotune import skin_from_speed
    R = rebuild_intervals(ckpt_every, reuse)[spec.dim]
    skin = skin_from_speed(float(np.sqrt((host[1].astype(np.float64) ** 2).sum(axis=0)).max()), spec.params(), R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    x, v, r = (torch.tensor(a, device=dev) for a in host)
    plan = Plan([spec.params()], [spec.n], dtype=dtype, tape_depth=ckpt_every, device=dev, skin=skin,
                rebuild_every=R, speed_skins=R > 1)
    if tuned:
        from .autotune import apply_cached
        apply_cached(plan)
    T, K = req.steps, ckpt_every
    ck = [plan.empty_state() for _ in range((T + K - 1) // K)]
    plan.step(x, v, r, T, ck, K)
    gx, gv, gr = torch.zeros_like(x), 2.0 * v, torch.zeros_like(r)
    plan.rollout_backward(ck, T, K, gx, gv, gr)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, (gx, gv, gr)
