"""The forward tape: a plan with as many tape slots as a rollout has steps keeps every step's
sorted state and lists during sph_step, and sph_rollout_backward then runs its adjoint steps on
them without recomputing the checkpoint segments.  The gradient is bitwise the one of the
recomputing backward (a plan whose tape holds one segment), also when list reuse is on, and the
backward recomputes when a later call has overwritten part of the tape."""
import numpy as np
import pytest
import torch

from paper_2507_21684_amd.inputs import SimSpec, make_state
from paper_2507_21684_amd.lib import Plan

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _job(plan, st, T, K, between=None):
    x, v, r = (t.clone() for t in st)
    ck = [plan.empty_state() for _ in range((T + K - 1) // K)]
    plan.step(x, v, r, T, ck, K)
    if between is not None:
        between(plan)
    g = (torch.zeros_like(x), 2.0 * v, torch.zeros_like(r))
    plan.rollout_backward(ck, T, K, *g)
    torch.cuda.synchronize()
    assert np.all(plan.poll() == 0)
    return [t.clone() for t in (x, v, r) + g], ck


@pytest.mark.parametrize("dim,side,skin,R", [(2, 40, 0.0, 1), (2, 48, 0.2, 2), (3, 14, 0.15, 2)])
def test_taped_backward_equals_the_recomputing_one(dim, side, skin, R):
    spec = SimSpec(dim, side, amplitude=1.4)
    T, K = 12, 4
    st = [torch.tensor(a.astype(np.float32), device=DEV) for a in make_state(spec, 3)]
    kw = dict(device=DEV, skin=skin, rebuild_every=R)
    ref, _ = _job(Plan([spec.params()], [spec.n], "f32", tape_depth=K, **kw), st, T, K)
    taped = Plan([spec.params()], [spec.n], "f32", tape_depth=T, **kw)
    got, ck = _job(taped, st, T, K)
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    # a second backward on the same tape gives the same gradient
    g = (torch.zeros_like(st[0]), 2.0 * got[1], torch.zeros_like(st[2]))
    taped.rollout_backward(ck, T, K, *g)
    for a, b in zip(g, ref[3:]):
        assert torch.equal(a, b)


def test_overwritten_tape_is_recomputed():
    spec = SimSpec(2, 36, amplitude=1.1)
    T, K = 8, 4
    st = [torch.tensor(a.astype(np.float32), device=DEV) for a in make_state(spec, 4)]
    ref, _ = _job(Plan([spec.params()], [spec.n], "f32", tape_depth=K, device=DEV), st, T, K)
    taped = Plan([spec.params()], [spec.n], "f32", tape_depth=T, device=DEV)
    # a right-hand side between forward and backward sorts into the last slot, a tape slot here
    got, _ = _job(taped, st, T, K, between=lambda p: p.rhs(*[t.clone() for t in st]))
    for a, b in zip(got, ref):
        assert torch.equal(a, b)


def test_graph_replays_keep_the_forward_tape_and_the_results():
    """Graph mode on a taped plan: the forward and backward calls replayed, with eager work in
    between, give bitwise the direct path's results on every replay."""
    spec = SimSpec(2, 36, amplitude=1.2)
    T, K = 8, 4
    st = [torch.tensor(a.astype(np.float32), device=DEV) for a in make_state(spec, 6)]
    ref, _ = _job(Plan([spec.params()], [spec.n], "f32", tape_depth=T, device=DEV, skin=0.2, rebuild_every=2),
                  st, T, K)
    plan = Plan([spec.params()], [spec.n], "f32", tape_depth=T, device=DEV, skin=0.2, rebuild_every=2)
    plan.set_graphs(True)
    x, v, r = plan.empty_state()
    ck = [plan.empty_state() for _ in range(T // K)]
    gx, gv, gr = torch.empty_like(x), torch.empty_like(v), torch.empty_like(r)
    for rep in range(4):
        for b, a in zip((x, v, r), st):
            b.copy_(a)
        plan.step(x, v, r, T, ck, K)
        gx.zero_()
        gv.copy_(2.0 * v)
        gr.zero_()
        assert torch.isfinite(torch.randn(4096, device=DEV).sum())   # eager work between replays
        plan.rollout_backward(ck, T, K, gx, gv, gr)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip((x, v, r, gx, gv, gr), ref)):
            assert torch.equal(a, b), "replay %d, output %d" % (rep, k)
    assert np.all(plan.poll() == 0)


def test_graph_cache_follows_setting_changes():
    """Graph mode: after the reuse interval, the skin mode or the lanes change, the next calls
    give bitwise what a fresh plan with the new settings gives, not a replay of graphs captured
    under the old ones; returning to the first settings replays their graphs."""
    spec = SimSpec(2, 36, amplitude=1.2)
    T, K = 8, 8
    st = [torch.tensor(a.astype(np.float32), device=DEV) for a in make_state(spec, 6)]

    def fresh(R, speed, lanes):
        p = Plan([spec.params()], [spec.n], "f32", tape_depth=T, device=DEV, skin=0.3, rebuild_every=R,
                 speed_skins=speed)
        p.set_tuning(*lanes)
        return _job(p, st, T, K)[0]

    plan = Plan([spec.params()], [spec.n], "f32", tape_depth=T, device=DEV, skin=0.3, rebuild_every=2)
    plan.set_graphs(True)
    settings = [(2, False, (4, 4)), (4, False, (4, 4)), (4, True, (4, 4)), (4, True, (2, 8)), (2, False, (4, 4))]
    prev = None
    for R, speed, lanes in settings:
        plan.set_reuse(R)
        plan.set_skin_mode(speed)
        plan.set_tuning(*lanes)
        for rep in range(2):
            got = _job(plan, st, T, K)[0]
            want = fresh(R, speed, lanes)
            for k, (a, b) in enumerate(zip(got, want)):
                assert torch.equal(a, b), "R %d speed %s lanes %s replay %d output %d" % (R, speed, lanes, rep, k)
        if prev is not None and (R, speed) != prev[0]:
            # the settings change the summation order, so a stale graph would show
            assert any(not torch.equal(a, b) for a, b in zip(got, prev[1]))
        prev = ((R, speed), got)
