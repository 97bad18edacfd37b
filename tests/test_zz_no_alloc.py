"""The allocation-free binding: plans bound to the library's static per-device workspace
(sph_bind_scratch) give bitwise the results of the same plans bound to a workspace the caller
allocated (sph_bind), on two plans in a row, the second smaller, so the second runs on the
array the first left behind."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2507_21684_amd import lib as L
from paper_2507_21684_amd.inputs import SimSpec, make_state
from paper_2507_21684_amd.lib import Plan, SphError

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
NSTEPS, EVERY = 12, 4


def _job(plan, st):
    """Right-hand side, 12 steps with checkpoints every 4 and the checkpointed gradient of
    sum |v_T|^2; every output on the host."""
    x, v, r = [torch.tensor(a, device=DEV).contiguous() for a in st]
    drho, acc, rs = plan.rhs(x, v, r)
    ck = [tuple(t.clone() for t in (x, v, r)) for _ in range((NSTEPS + EVERY - 1) // EVERY)]
    plan.step(x, v, r, NSTEPS, ck, EVERY)
    gx, gv, gr = torch.zeros_like(x), 2.0 * v, torch.zeros_like(r)
    plan.rollout_backward(ck, NSTEPS, EVERY, gx, gv, gr)
    torch.cuda.synchronize()
    assert np.all(plan.poll() == 0)
    return [t.cpu().numpy() for t in (drho, acc, rs, x, v, r, gx, gv, gr)]


CASES = [  # (spec, seed, skin, rebuild interval); the second is smaller than the first
    (SimSpec(2, 64, amplitude=1.2), 3, 0.2, 4),
    (SimSpec(2, 36, amplitude=0.8), 4, 0.0, 1),
]


def test_scratch_binding_matches_the_callers_workspace():
    plans = []
    for spec, seed, skin, R in CASES:
        st = [a.astype(np.float32) for a in make_state(spec, seed)]
        kw = dict(tape_depth=EVERY, device=DEV, skin=skin, rebuild_every=R)
        ref = _job(Plan([spec.params()], [spec.n], "f32", **kw), st)
        plan = Plan([spec.params()], [spec.n], "f32", scratch=True, **kw)
        assert plan.workspace is None and plan.workspace_bytes <= L.SCRATCH_BYTES
        got = _job(plan, st)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        plans.append((plan, st, ref))
    # the second binding took the array over: the first plan's calls fail until it rebinds
    first, st, ref = plans[0]
    with pytest.raises(SphError, match="STATE"):
        first.poll()
    first.bind_scratch()
    for a, b in zip(_job(first, st), ref):
        np.testing.assert_array_equal(a, b)


def test_scratch_binding_rejects_a_plan_larger_than_the_array():
    spec = SimSpec(3, 32)
    assert L.workspace_bytes([spec.params()], [spec.n], "f32", 8) > L.SCRATCH_BYTES
    with pytest.raises(SphError, match="CAPACITY"):
        Plan([spec.params()], [spec.n], "f32", tape_depth=8, device=DEV, scratch=True)
