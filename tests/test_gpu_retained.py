"""Retained neighbour lists: the step and density adjoints reuse the sort and lists that the
forward call built for the same state (the paper's backward reuses the forward adjacency), and
give bitwise the results of the plain adjoints, which rebuild them; when the retained slot has
been overwritten since, the call falls back to the plain adjoint."""
import numpy as np
import pytest
import torch

from paper_2507_21684_amd.inputs import SimSpec, make_state
from paper_2507_21684_amd.lib import Plan

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _state(spec, seed, dtype="f32"):
    npdt = np.float32 if dtype == "f32" else np.float64
    return [torch.tensor(a.astype(npdt), device=DEV) for a in make_state(spec, seed)]


def _cot(st, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return [torch.randn(t.shape, generator=g, dtype=torch.float64).to(DEV, t.dtype) for t in st]


@pytest.mark.parametrize("dim,side,dtype,skin,R", [(2, 40, "f32", 0.0, 1), (2, 48, "f32", 0.2, 4),
                                                   (3, 14, "f32", 0.15, 2), (2, 24, "f64", 0.0, 1)])
def test_retained_adjoints_equal_the_plain_ones(dim, side, dtype, skin, R):
    spec = SimSpec(dim, side, amplitude=1.3)
    plan = Plan([spec.params()], [spec.n], dtype, tape_depth=1, device=DEV, skin=skin, rebuild_every=R)
    x0 = _state(spec, 5, dtype)
    # forward: one step (retains the input's sort in slot 0), then the density of the result
    # (retains the result's sort in the last slot)
    x1 = [t.clone() for t in x0]
    plan.step(*x1, 1)
    kept_step = plan.retained_lists()
    _, _, rs = plan.rhs(*x1, rho_sum=True)
    kept_rhs = plan.retained_lists()
    assert kept_step[0] == 0 and kept_rhs[0] >= 1 and kept_rhs[1] > kept_step[1]
    g = _cot([rs], 6)[0]
    xb_kept = plan.density_adjoint(*x1, g, retained=kept_rhs)
    c_kept = _cot(x0, 7)
    plan.step_adjoint(*x0, *c_kept, retained=kept_step)
    # the plain adjoints rebuild the sorts and lists of the same states
    xb_plain = plan.density_adjoint(*x1, g)
    c_plain = _cot(x0, 7)
    plan.step_adjoint(*x0, *c_plain)
    assert torch.equal(xb_kept, xb_plain)
    for a, b in zip(c_kept, c_plain):
        assert torch.equal(a, b)
    # the plain calls re-sorted slot 0: the step's retained pair is gone, and a retained call with
    # it falls back to the plain adjoint, with the same result
    c_again = _cot(x0, 7)
    plan.step_adjoint(*x0, *c_again, retained=kept_step)
    for a, b in zip(c_again, c_plain):
        assert torch.equal(a, b)
    assert np.all(plan.poll() == 0)


def test_retention_survives_graph_replays_and_is_off_for_other_schemes():
    spec = SimSpec(2, 32, amplitude=0.9)
    plan = Plan([spec.params()], [spec.n], "f32", tape_depth=1, device=DEV)
    plan.set_graphs(True)
    x0 = _state(spec, 8)
    buf = [torch.empty_like(t) for t in x0]
    ref = None
    for rep in range(3):
        for b, a in zip(buf, x0):
            b.copy_(a)
        plan.step(*buf, 1)                       # captured once, then replayed
        kept = plan.retained_lists()
        assert kept[0] == 0
        c = _cot(x0, 9)
        plan.step_adjoint(*x0, *c, retained=kept)
        torch.cuda.synchronize()
        if ref is None:
            ref = _cot(x0, 9)
            plan.step_adjoint(*x0, *ref)
        for a, b in zip(c, ref):
            assert torch.equal(a, b), "replay %d" % rep
    plan.set_graphs(False)
    rk = Plan([spec.params()], [spec.n], "f32", tape_depth=1, device=DEV, integrator="rk4")
    rk.step(*[t.clone() for t in x0], 1)
    assert rk.retained_lists()[0] == -1
