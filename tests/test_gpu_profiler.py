"""The library's HIP-event profiler (sph_profile_enable / sph_profile_read) on the GPU: launch
counts per kernel class, positive times for the classes asked for and none for the others,
reset on read, and results bitwise unchanged by profiling."""
import numpy as np
import pytest
import torch

from paper_2507_21684_amd.inputs import SimSpec, make_state
from paper_2507_21684_amd.lib import Plan

pytestmark = pytest.mark.gpu


def _gpu(arrs):
    return [torch.tensor(a.astype(np.float32), device=torch.device("cuda", 0)).contiguous() for a in arrs]


def test_profiler_counts_and_resets():
    spec = SimSpec(2, 32)
    st = make_state(spec, 2)
    plan = Plan([spec.params()], [spec.n], "f32")
    ref = _gpu(st)
    plan.step(*ref, 4)
    plan.profile(True)
    g = _gpu(st)
    plan.step(*g, 4)
    prof = plan.profile_read()
    assert prof["sweep"][1] == 4 and prof["sweep"][0] > 0
    assert prof["build"][1] == 4 and prof["build"][0] > 0
    assert prof["adjoint"][1] == 0 and prof["adjoint"][0] == 0
    for a, b in zip(g, ref):
        assert torch.equal(a, b)                     # profiling does not change the results
    c = _gpu([np.ones_like(a) for a in st])
    plan.step_adjoint(*_gpu(st), *c)
    prof = plan.profile_read()
    assert prof["adjoint"][1] == 1 and prof["adjoint"][0] > 0
    empty = plan.profile_read()                      # reset by the previous read
    assert all(n == 0 and ms == 0 for ms, n in empty.values())


def test_profiler_times_only_the_classes_asked_for():
    spec = SimSpec(2, 32)
    st = make_state(spec, 3)
    plan = Plan([spec.params()], [spec.n], "f32")
    plan.profile(True, classes=["sweep"])
    plan.step(*_gpu(st), 3)
    prof = plan.profile_read()
    assert prof["sweep"][1] == 3 and prof["sweep"][0] > 0
    assert all(prof[k][1] == 0 for k in prof if k != "sweep")
    plan.profile(False)
    plan.step(*_gpu(st), 3)
    assert all(n == 0 for _, n in plan.profile_read().values())
