"""Host logic of the serving loop: admission, continuous batching by segment, FIFO latencies.

The scheduler runs against a recording engine on a simulated clock (no GPU); the GPU engine
and its bitwise agreement with the plain path are covered by the GPU tests.
"""
import math

import numpy as np
import pytest

from paper_2507_21684_amd.inputs import Request, SimSpec, serving_trace
from paper_2507_21684_amd.serving import Scheduler, fifo_latencies, percentiles


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class RecordingEngine:
    """Footprint = particle count; every group call costs 1 ms + 1 us per particle-step."""

    def __init__(self, clock):
        self.clock = clock
        self.calls = []
        self.admitted = []
        self.finished = []
        self.fail = set()

    def footprint(self, req):
        return req.spec.n

    def segment_cost(self, job, n):
        return 1e-6 * n * job.req.spec.n * (1.0 if job.phase == "fwd" else 2.0)

    def admit(self, job):
        self.admitted.append(job.req.rid)
        job.state = "x0"

    def forward(self, jobs, n):
        self.calls.append(("fwd", [j.req.rid for j in jobs], n, [j.pos for j in jobs], [j.dim for j in jobs]))
        self.clock.t += 1e-3 + 1e-6 * n * sum(j.req.spec.n for j in jobs)

    def backward(self, jobs, n):
        self.calls.append(("bwd", [j.req.rid for j in jobs], n, [j.seg for j in jobs], [j.dim for j in jobs]))
        self.clock.t += 1e-3 + 2e-6 * n * sum(j.req.spec.n for j in jobs)

    def finish(self, jobs):
        self.finished.extend(j.req.rid for j in jobs)

    def sync(self):
        return {rid: 1 for rid in self.fail if any(rid in c[1] for c in self.calls)}


def small_trace(seed=7, count=40, rate=200.0):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        dim = 2 if rng.uniform() < 0.7 else 3
        side = int(rng.integers(16, 40)) if dim == 2 else int(rng.integers(16, 24))
        out.append(Request(k, t, SimSpec(dim, side), k, int(rng.integers(3, 30))))
    return out


def run(trace, K=8, budget=1 << 40):
    clock = FakeClock()
    eng = RecordingEngine(clock)
    sch = Scheduler(eng, K, budget, clock=clock)
    done = sch.run(trace)
    return sch, eng, done


@pytest.mark.parametrize("K", [1, 3, 8])
def test_every_request_runs_its_segments_in_order(K):
    trace = small_trace()
    sch, eng, done = run(trace, K)
    assert sorted(j.req.rid for j in done) == list(range(len(trace)))
    assert sorted(eng.finished) == list(range(len(trace)))
    for r in trace:
        fwd = [(n, c[3][c[1].index(r.rid)]) for c in eng.calls if c[0] == "fwd" and r.rid in c[1] for n in [c[2]]]
        bwd = [(n, c[3][c[1].index(r.rid)]) for c in eng.calls if c[0] == "bwd" and r.rid in c[1] for n in [c[2]]]
        # forward: segments of K from step 0, the last one shorter, positions increasing
        pos = 0
        for n, p in fwd:
            assert p == pos and n == min(K, r.steps - pos)
            pos += n
        assert pos == r.steps
        # backward: the same segments in reverse
        nseg = (r.steps + K - 1) // K
        assert [s for _, s in bwd] == list(range(nseg - 1, -1, -1))
        assert [n for n, _ in bwd] == [min(K, r.steps - s * K) for s in range(nseg - 1, -1, -1)]
        # the backward starts after the last forward segment
        first_b = min(i for i, c in enumerate(eng.calls) if c[0] == "bwd" and r.rid in c[1])
        last_f = max(i for i, c in enumerate(eng.calls) if c[0] == "fwd" and r.rid in c[1])
        assert first_b > last_f


def test_groups_are_homogeneous_and_batched():
    trace = small_trace(count=60, rate=2000.0)
    sch, eng, done = run(trace)
    for phase, rids, n, _, dims in eng.calls:
        assert len(set(dims)) == 1
        assert len(set(rids)) == len(rids)
    # with a dense arrival trace the batches hold several requests
    assert max(len(c[1]) for c in eng.calls) >= 5
    assert max(sch.batch_sizes) >= 5


def test_budget_and_fifo_admission():
    trace = small_trace(count=50, rate=5000.0)
    budget = 30000      # above every single footprint, below the sum of a few
    sch, eng, done = run(trace, 8, budget)
    assert max(r.spec.n for r in trace) <= budget
    assert sch.peak_used <= budget
    assert sch.peak_used > budget // 2
    # admitted in arrival order
    by_rid = {j.req.rid: j for j in done}
    adm = [by_rid[r.rid].admitted for r in sorted(trace, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert eng.admitted == sorted(eng.admitted, key=lambda rid: trace[rid].arrival)
    for j in done:
        assert j.admitted >= j.req.arrival - 1e-12
        assert j.finished > j.admitted


def test_oversized_request_runs_alone():
    trace = [Request(0, 0.0, SimSpec(2, 64), 0, 8), Request(1, 0.0, SimSpec(2, 16), 1, 8)]
    sch, eng, done = run(trace, 8, budget=100)
    assert len(done) == 2
    for c in eng.calls:
        assert len(c[1]) == 1


def test_idle_server_jumps_to_next_arrival():
    trace = [Request(0, 0.0, SimSpec(2, 16), 0, 4), Request(1, 10.0, SimSpec(2, 16), 1, 4)]
    sch, eng, done = run(trace)
    j1 = [j for j in done if j.req.rid == 1][0]
    assert j1.admitted == pytest.approx(10.0)
    assert j1.finished - 10.0 < 0.1


def test_fifo_latencies_closed_form():
    # arrivals every 1 s, service 2 s: the k-th request waits k seconds in the queue
    lat = fifo_latencies([0, 1, 2, 3], [2, 2, 2, 2])
    assert np.allclose(lat, [2, 3, 4, 5])
    # idle gaps do not accumulate
    assert np.allclose(fifo_latencies([0, 10], [1, 1]), [1, 1])
    p = percentiles([0.001, 0.002, 0.003])
    assert p["p50_ms"] == pytest.approx(2.0) and p["mean_ms"] == pytest.approx(2.0)
    assert math.isnan(percentiles([])["p50_ms"])


def test_serving_trace_recipe():
    tr = serving_trace(seed=2026, count=400, rate=10.0)
    assert [r.rid for r in tr] == list(range(400))
    arr = np.array([r.arrival for r in tr])
    assert np.all(np.diff(arr) > 0)
    assert abs(np.mean(np.diff(arr)) - 0.1) < 0.02
    dims = np.array([r.spec.dim for r in tr])
    assert 0.24 < np.mean(dims == 3) < 0.36
    for r in tr:
        assert 16 <= r.steps <= 128 and 0.5 <= r.spec.amplitude <= 2.0
        if r.spec.dim == 2:
            assert 32 <= r.spec.side <= 256
        else:
            assert 20 <= r.spec.side <= 100


def test_failed_request_leaves_at_once():
    trace = [Request(0, 0.0, SimSpec(2, 16), 0, 64), Request(1, 0.0, SimSpec(2, 16), 1, 64)]
    clock = FakeClock()
    eng = RecordingEngine(clock)
    eng.fail = {0}
    sch = Scheduler(eng, 8, 1 << 40, clock=clock)
    done = {j.req.rid: j for j in sch.run(trace)}
    assert done[0].error == 1 and done[1].error == 0
    assert sum(1 for c in eng.calls if 0 in c[1]) == 1        # dropped after its first tick
    assert sum(1 for c in eng.calls if 1 in c[1]) == 16       # 8 forward + 8 backward segments


def test_small_request_is_not_held_at_the_pace_of_a_large_one():
    # a large request is running when a small one arrives: with cost-fair sharing the small
    # one finishes long before the large one, and in far fewer ticks than the large one needs
    trace = [Request(0, 0.0, SimSpec(3, 40), 0, 128), Request(1, 1e-9, SimSpec(2, 16), 1, 128)]
    clock = FakeClock()
    eng = RecordingEngine(clock)
    sch = Scheduler(eng, 8, 1 << 40, clock=clock, quantum=1e-3)
    done = {j.req.rid: j for j in sch.run(trace)}
    small, large = done[1], done[0]
    assert small.finished < 0.2 * large.finished
    ticks_with_large = sum(1 for c in eng.calls if 0 in c[1])
    assert ticks_with_large == 32
    # in plain segment-per-tick sharing the small request would have taken 32 ticks of the large one
    ticks_before_small_done = sum(1 for c in eng.calls[:max(i for i, c in enumerate(eng.calls) if 1 in c[1]) + 1]
                                  if 0 in c[1])
    assert ticks_before_small_done <= 3


def test_rebuild_intervals_divide_the_checkpoint_interval():
    from paper_2507_21684_amd.serving import rebuild_intervals
    assert rebuild_intervals(8) == {2: 8, 3: 2}
    assert rebuild_intervals(6) == {2: 6, 3: 2}
    assert rebuild_intervals(3) == {2: 3, 3: 1}
    assert rebuild_intervals(1) == {2: 1, 3: 1}
    assert rebuild_intervals(8, reuse=1) == {2: 1, 3: 1}
    for K in range(1, 17):
        for R in rebuild_intervals(K).values():
            assert K % R == 0


def _latencies(trace, **kw):
    clock = FakeClock()
    eng = RecordingEngine(clock)
    sch = Scheduler(eng, 8, 1 << 40, clock=clock, quantum=1e-3, **kw)
    done = {j.req.rid: j for j in sch.run(trace)}
    return {rid: j.finished - j.req.arrival for rid, j in done.items()}, eng


def test_aging_is_inactive_within_the_grace():
    # every request finishes within a few mean costs: aging changes nothing
    trace = small_trace(count=12, rate=20.0)
    lat_fair, eng_fair = _latencies(trace, age_weight=0.0, large_factor=0.0)
    lat_aged, eng_aged = _latencies(trace, age_weight=2.0, age_after=50.0, large_factor=0.0)
    assert eng_fair.calls == eng_aged.calls
    assert lat_fair == lat_aged


def test_aging_bounds_the_stretch_of_an_old_large_request():
    # a large request under a steady stream of small ones: fair sharing stretches it, aging
    # gives it a growing share once it has waited past the grace, and the small requests still
    # finish far sooner than it does
    rng = np.random.default_rng(3)
    trace = [Request(0, 0.0, SimSpec(3, 40), 0, 64)]
    t = 0.0
    for k in range(1, 200):
        t += rng.exponential(0.15)
        trace.append(Request(k, t, SimSpec(2, 24), k, 32))
    lat_fair, _ = _latencies(trace, age_weight=0.0, large_factor=0.0)
    lat_aged, _ = _latencies(trace, age_weight=2.0, age_after=8.0, large_factor=0.0)
    assert lat_aged[0] < 0.8 * lat_fair[0]
    small = [lat_aged[k] for k in range(1, 200)]
    assert np.median(small) < 0.1 * lat_aged[0]


def test_large_requests_share_one_at_a_time_in_admission_order():
    # three large requests among small ones: each large one runs alone among the large ones, in
    # admission order, so the first finishes long before the last instead of all at the end
    trace = [Request(k, 0.001 * k, SimSpec(2, 16), k, 16) for k in range(20)]
    trace += [Request(20 + k, 0.02 + 0.001 * k, SimSpec(3, 40), 20 + k, 64) for k in range(3)]
    lat, eng = _latencies(trace, large_factor=3.0, age_weight=0.0)
    fin = [lat[20 + k] + 0.02 + 0.001 * k for k in range(3)]
    assert fin[0] < fin[1] < fin[2]
    assert fin[0] < 0.5 * fin[2]
    for c in eng.calls:                       # never two large requests in one tick
        assert sum(1 for rid in c[1] if rid >= 20) <= 1
    ticks = {}
    for i, c in enumerate(eng.calls):
        for rid in c[1]:
            ticks.setdefault(rid, []).append(i)
    assert max(ticks[20]) < min(ticks[21]) and max(ticks[21]) < min(ticks[22])
    lat_fair, _ = _latencies(trace, large_factor=0.0, age_weight=0.0)
    fin_fair = [lat_fair[20 + k] + 0.02 + 0.001 * k for k in range(3)]
    assert fin_fair[0] > 0.8 * fin_fair[2]      # fair sharing: all three end together


def _tick_gaps(eng, rid, t_from=None):
    """Largest number of consecutive ticks (group calls) without `rid` while it was active."""
    idx = [i for i, c in enumerate(eng.calls) if rid in c[1]]
    return max(b - a - 1 for a, b in zip(idx, idx[1:])) if len(idx) > 1 else 0


def test_newcomers_do_not_freeze_the_running_set_while_a_large_request_waits():
    # two large requests (the second waits for the first) and a small request in flight; small
    # requests that arrive later start at the running set's smallest virtual time, not at the
    # frozen one of the waiting large request, so the in-flight small request keeps getting
    # ticks; and the second large request, when its turn comes, shares the device too
    trace = [Request(k, 0.0001 * k, SimSpec(2, 16), k, 16) for k in range(8)]
    trace += [Request(8, 0.001, SimSpec(2, 16), 8, 48), Request(9, 0.002, SimSpec(3, 40), 9, 64),
              Request(10, 0.003, SimSpec(3, 40), 10, 64)]
    t = 0.3
    for k in range(11, 60):
        trace.append(Request(k, t, SimSpec(2, 16), k, 32))
        t += 0.04 if k < 40 else 1.0
    clock = FakeClock()
    eng = RecordingEngine(clock)
    starts = []
    fwd, bwd = eng.forward, eng.backward
    eng.forward = lambda jobs, n: (starts.append(clock.t), fwd(jobs, n))
    eng.backward = lambda jobs, n: (starts.append(clock.t), bwd(jobs, n))
    sch = Scheduler(eng, 8, 1 << 40, clock=clock, quantum=1e-3, large_factor=3.0, age_weight=0.0)
    done = {j.req.rid: j for j in sch.run(trace)}
    assert sorted(done) == list(range(60))
    assert done[9].large and done[10].large and not done[8].large
    # the in-flight small request is never left out for more than a handful of group calls
    assert _tick_gaps(eng, 8) <= 4
    # once the first large request is done, the second does not run alone while small requests
    # that arrived meanwhile wait (at most the one call in which they are admitted)
    end9 = max(i for i, c in enumerate(eng.calls) if 9 in c[1])
    alone = longest = 0
    for i in range(end9 + 1, len(eng.calls)):
        t = starts[i]
        waiting = [k for k in range(11, 60) if done[k].admitted <= t < done[k].finished]
        alone = alone + 1 if eng.calls[i][1] == [10] and waiting else 0
        longest = max(longest, alone)
    assert any(done[k].finished > done[9].finished for k in range(11, 60))
    assert longest <= 2


class LaggedEngine(RecordingEngine):
    """The device runs one tick behind: sync() of tick t reports the failures of tick t - 1,
    drain() those of the last tick."""

    lookahead = 1

    def __init__(self, clock):
        super().__init__(clock)
        self.ticks = []          # per tick: the rids of its group calls
        self.reported = 0
        self.finish_tick = {}
        self._mark = 0

    def sync(self):
        self.ticks.append(sorted({rid for c in self.calls[self._mark:] for rid in c[1]}))
        self._mark = len(self.calls)
        out = self._report(len(self.ticks) - 1)
        return out

    def _report(self, upto):
        failed = {}
        while self.reported < upto:
            failed.update({rid: 1 for rid in self.fail if rid in self.ticks[self.reported]})
            self.reported += 1
        return failed

    def drain(self):
        return self._report(len(self.ticks))

    def finish(self, jobs):
        super().finish(jobs)
        for j in jobs:
            self.finish_tick[j.req.rid] = len(self.ticks)


def test_one_tick_lookahead_keeps_the_schedule_and_finishes_a_tick_later():
    trace = small_trace(seed=11, count=30)
    _, eng0, done0 = run(trace)
    clock = FakeClock()
    eng1 = LaggedEngine(clock)
    done1 = Scheduler(eng1, 8, 1 << 40, clock=clock).run(trace)
    # same group calls in the same order (the budget never binds here)
    assert eng1.calls == eng0.calls
    assert sorted(eng1.finished) == sorted(eng0.finished) == list(range(30))
    fin0 = {j.req.rid: j.finished for j in done0}
    for j in done1:
        # finished once the tick of its last segment is known to be complete: at the end of
        # the next tick (or when the device drains), never before the lag-free finish time
        last = max(t for t, rids in enumerate(eng1.ticks) if j.req.rid in rids)
        assert eng1.finish_tick[j.req.rid] >= last + 1
        assert j.finished >= fin0[j.req.rid] - 1e-12
        assert not j.error


def test_one_tick_lookahead_failure_is_reported_late_and_the_request_leaves_once():
    trace = small_trace(seed=5, count=12)
    clock = FakeClock()
    eng = LaggedEngine(clock)
    eng.fail = {3}
    done = Scheduler(eng, 4, 1 << 40, clock=clock).run(trace)
    assert sorted(j.req.rid for j in done) == list(range(12))
    bad = [j for j in done if j.req.rid == 3][0]
    assert bad.error == 1
    assert eng.finished.count(3) == 1
    # it ran at most one tick after the tick whose status reported the failure
    first = min(t for t, rids in enumerate(eng.ticks) if 3 in rids)
    ran = [t for t, rids in enumerate(eng.ticks) if 3 in rids]
    assert max(ran) <= first + 1
    assert all(not j.error for j in done if j.req.rid != 3)
