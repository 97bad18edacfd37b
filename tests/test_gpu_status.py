"""Device-side status words on the GPU: a non-finite position and an overflowing neighbour list
are reported through sph_poll for their own simulation only, and the other simulations of the
batch are computed exactly as they are alone."""
import numpy as np
import pytest
import torch

from paper_2507_21684_amd.inputs import SimSpec, make_state
from paper_2507_21684_amd.lib import FLAG_NEIGHBOR_OVERFLOW, FLAG_NONFINITE, Plan

pytestmark = pytest.mark.gpu

SPECS = [SimSpec(2, 20), SimSpec(2, 24, amplitude=1.5)]


def _gpu(arrs):
    return [torch.tensor(a, dtype=torch.float32, device=torch.device("cuda", 0)).contiguous() for a in arrs]


def _states():
    return [[a.astype(np.float32) for a in make_state(s, 30 + k)] for k, s in enumerate(SPECS)]


def _run(states, steps=2):
    plan = Plan([s.params() for s in SPECS], [s.n for s in SPECS], "f32")
    cat = [np.concatenate([st[k] for st in states], axis=-1) for k in range(3)]
    g = _gpu(cat)
    plan.step(*g, steps)
    status = plan.poll()
    return status, [t.cpu().numpy() for t in g]


def _solo(spec, state, steps=2):
    plan = Plan([spec.params()], [spec.n], "f32")
    g = _gpu(state)
    plan.step(*g, steps)
    assert np.all(plan.poll() == 0)
    return [t.cpu().numpy() for t in g]


def _check_second(out, steps):
    ref = _solo(SPECS[1], _states()[1], steps)
    n0 = SPECS[0].n
    for k in range(3):
        np.testing.assert_array_equal(out[k][..., n0:], ref[k])


def test_nonfinite_position_is_reported_for_its_simulation_only():
    states = _states()
    states[0][0][0, 5] = np.nan
    status, out = _run(states)
    assert status[0] & FLAG_NONFINITE
    assert status[1] == 0
    assert not np.isfinite(out[0][0, 5])
    _check_second(out, 2)


def test_neighbor_overflow_is_reported_for_its_simulation_only():
    states = _states()
    x = states[0][0]
    rng = np.random.default_rng(3)
    # 150 particles within a tenth of the spacing of one point: each has more neighbours than
    # a list row holds (about 1.6 times the particles of a support disc, 80 here)
    x[:, :150] = (0.5 + 0.1 * SPECS[0].dx * rng.uniform(-1, 1, size=(2, 150))).astype(np.float32)
    status, out = _run(states, steps=1)
    assert status[0] & FLAG_NEIGHBOR_OVERFLOW
    assert status[1] == 0
    _check_second(out, 1)


def test_neighbor_export_keeps_its_overflow_apart_from_the_status_words():
    # an overflow left unpolled by a step does not fail a later export whose own lists fit, and
    # the export's own overflow is returned by the call, not added to the status words
    from paper_2507_21684_amd.lib import SphError
    states = _states()
    clean = _gpu([np.concatenate([st[k] for st in states], axis=-1) for k in range(3)])
    x = states[0][0]
    rng = np.random.default_rng(3)
    x[:, :150] = (0.5 + 0.1 * SPECS[0].dx * rng.uniform(-1, 1, size=(2, 150))).astype(np.float32)
    dense = _gpu([np.concatenate([st[k] for st in states], axis=-1) for k in range(3)])
    plan = Plan([s.params() for s in SPECS], [s.n for s in SPECS], "f32")
    d1 = [t.clone() for t in dense]
    plan.step(*d1, 1)                          # overflow flag left unpolled
    off, nbr = plan.neighbors(*clean)          # fits: must succeed
    assert int(off[-1]) == nbr.numel() > 0
    with pytest.raises(SphError) as e:
        plan.neighbors(*dense)                 # its own overflow: CAPACITY from the call
    assert e.value.code == -3
    status = plan.poll()
    assert status[0] == FLAG_NEIGHBOR_OVERFLOW  # the step's flag, kept
    assert status[1] == 0
    with pytest.raises(SphError):
        plan.neighbors(*dense)
    assert np.all(plan.poll() == 0)            # the export added nothing


def test_rollout_raises_on_a_device_flag():
    # the differentiable rollout reads the status words after its forward pass: a non-finite
    # position raises instead of returning a silently wrong state; check=False leaves the words
    # for the caller
    from paper_2507_21684_amd.lib import SphError
    from paper_2507_21684_amd.rollout import rollout
    states = _states()
    states[0][0][0, 5] = np.nan
    g = _gpu([np.concatenate([st[k] for st in states], axis=-1) for k in range(3)])
    plan = Plan([s.params() for s in SPECS], [s.n for s in SPECS], "f32", tape_depth=2)
    with pytest.raises(SphError) as e:
        rollout(plan, *g, 2, 2)
    assert e.value.code == -4
    rollout(plan, *g, 2, 2, check=False)
    status = plan.poll()
    assert status[0] & FLAG_NONFINITE and status[1] == 0
