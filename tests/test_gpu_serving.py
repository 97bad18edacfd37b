"""Serving loop on the GPU: a request served in a continuously batched mix returns bitwise the
gradient of the plain path (its own plan, forward with checkpoints, checkpointed backward),
whatever the mix and the HBM budget, and that gradient agrees with the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_2507_21684_amd.inputs import Request, SimSpec

pytestmark = pytest.mark.gpu


def _trace():
    specs = [(SimSpec(2, 24, amplitude=0.7), 9), (SimSpec(2, 33, amplitude=1.6), 16), (SimSpec(3, 12), 6),
             (SimSpec(2, 20), 13), (SimSpec(3, 14, amplitude=1.3), 11), (SimSpec(2, 40), 5),
             (SimSpec(2, 24, amplitude=0.7), 12)]
    arrivals = [0.0, 0.0, 0.001, 0.002, 0.002, 0.01, 0.05]
    return [Request(k, a, s, 100 + k, T) for k, ((s, T), a) in enumerate(zip(specs, arrivals))]


def _plain(trace, K):
    from paper_2507_21684_amd.serving import plain_request
    return {r.rid: plain_request(r, "f32", K, tuned=False)[1] for r in trace}


@pytest.mark.parametrize("budget", [1 << 34, 0])
def test_served_gradients_equal_plain_path(budget):
    from paper_2507_21684_amd.serving import serve
    K = 4
    trace = _trace()
    sch, eng, done = serve(trace, "f32", K, budget, tuned=False)
    assert sorted(j.req.rid for j in done) == [r.rid for r in trace]
    if budget:
        assert max(sch.batch_sizes) >= 3          # requests really were mixed
    else:
        assert max(sch.batch_sizes) == 1          # zero budget: one request at a time
    ref = _plain(trace, K)
    for r in trace:
        for got, want in zip(eng.results[r.rid], ref[r.rid]):
            assert torch.equal(got, want), "request %d differs from the plain path" % r.rid
    assert eng.pairs > 0


def test_served_gradient_matches_oracle(orc):
    from paper_2507_21684_amd.inputs import make_state
    from paper_2507_21684_amd.serving import serve
    trace = _trace()[:4]
    sch, eng, done = serve(trace, "f32", 4, 1 << 34, tuned=False)
    for r in (trace[1], trace[2]):
        x, v, rho = (a.astype(np.float32) for a in make_state(r.spec, r.seed))
        ref = orc.rollout(orc.Params(**r.spec.params()), x, v, rho, r.steps, 0)
        for got, want in zip(eng.results[r.rid], (ref["gx0"], ref["gv0"], ref["grho0"])):
            got = got.cpu().numpy().astype(np.float64)
            assert np.abs(got - want).max() <= 1e-3 * np.abs(want).max()
