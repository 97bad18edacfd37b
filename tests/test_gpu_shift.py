"""Particle shifting (sph_shift / sph_shift_adjoint) on the GPU against the FP64 oracle: the shift, its
VJP, a gradient through step-then-shift composed with autograd, and bitwise batch invariance."""
import numpy as np
import pytest
import torch

from paper_2507_21684_amd.inputs import SimSpec, make_state
from paper_2507_21684_amd.lib import Plan

pytestmark = pytest.mark.gpu


def _gpu(arrs, dtype):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    return [torch.tensor(a, dtype=tdt, device=torch.device("cuda", 0)).contiguous() for a in arrs]


def _state(spec, seed, dtype):
    npdt = np.float32 if dtype == "f32" else np.float64
    x, v, rho = make_state(spec, seed)
    rng = np.random.default_rng(seed + 50)
    rho = rho * (1 + 0.02 * rng.uniform(-1, 1, size=rho.shape))
    return [a.astype(npdt) for a in (x, v, rho)]


def _plan(specs, dtype, **kw):
    return Plan([s.params() for s in specs], [s.n for s in specs], dtype, **kw)


@pytest.mark.parametrize("dtype,dim,side,skin", [("f64", 2, 24, 0.0), ("f64", 3, 12, 0.0), ("f32", 2, 40, 0.2),
                                                 ("f32", 3, 16, 0.0)])
def test_shift_parity(orc, dtype, dim, side, skin):
    spec = SimSpec(dim, side, jitter=0.25)
    x, v, rho = _state(spec, 1, dtype)
    beta = 0.5
    plan = _plan([spec], dtype, skin=skin)
    g = _gpu([x, v, rho], dtype)
    plan.shift(*g, beta)
    dr = orc.shift(orc.Params(**spec.params()), x, rho, beta)
    got = g[0].cpu().numpy().astype(np.float64) - x.astype(np.float64)
    tol = 1e-10 if dtype == "f64" else 1e-4
    assert np.abs(got - dr).max() <= tol * np.abs(dr).max() + (0 if dtype == "f64" else 4e-7 * spec.box)
    np.testing.assert_array_equal(g[1].cpu().numpy(), v)
    np.testing.assert_array_equal(g[2].cpu().numpy(), rho)


@pytest.mark.parametrize("dtype,dim,side", [("f64", 2, 20), ("f32", 2, 32), ("f64", 3, 12), ("f32", 3, 12)])
def test_shift_adjoint_parity(orc, dtype, dim, side):
    spec = SimSpec(dim, side, jitter=0.25)
    x, v, rho = _state(spec, 3, dtype)
    rng = np.random.default_rng(4)
    c = [rng.normal(size=a.shape).astype(a.dtype) for a in (x, v, rho)]
    beta = 0.5
    plan = _plan([spec], dtype)
    g = _gpu([x, v, rho], dtype)
    cg = _gpu(c, dtype)
    plan.shift_adjoint(*g, *cg, beta)
    gx, gr = orc.shift_vjp(orc.Params(**spec.params()), x, rho, beta, c[0])
    tol = 1e-9 if dtype == "f64" else 1e-3
    got = [t.cpu().numpy().astype(np.float64) for t in cg]
    assert np.abs((got[0] - c[0]) - gx).max() <= tol * np.abs(gx).max()
    assert np.abs((got[2] - c[2]) - gr).max() <= tol * np.abs(gr).max()
    np.testing.assert_array_equal(cg[1].cpu().numpy(), c[1])
    np.testing.assert_array_equal(g[0].cpu().numpy(), x)     # the state is not modified


def test_step_then_shift_gradient(orc):
    """Two steps, each followed by a shift, composed with autograd; FP64 against the oracle's chain."""
    from paper_2507_21684_amd.rollout import rollout, shift
    spec = SimSpec(2, 20)
    x, v, rho = _state(spec, 5, "f64")
    beta = 0.3
    plan = _plan([spec], "f64", tape_depth=1)
    tx, tv, tr = _gpu([x, v, rho], "f64")
    for t in (tx, tv, tr):
        t.requires_grad_(True)
    s = (tx, tv, tr)
    for _ in range(2):
        s = rollout(plan, *s, 1, 1)
        s = shift(plan, *s, beta)
    loss = (s[1] ** 2).sum() + (s[0] * torch.linspace(0, 1, s[0].numel(), dtype=torch.float64,
                                                     device=s[0].device).view_as(s[0])).sum()
    loss.backward()
    # the oracle's chain: step, shift, step, shift; then the VJPs in reverse
    p = orc.Params(**spec.params())
    states = []
    cur = (x, v, rho)
    for _ in range(2):
        states.append(("step", cur))
        cur = orc.step(p, *cur, 1)
        states.append(("shift", cur))
        cur = (cur[0] + orc.shift(p, cur[0], cur[2], beta), cur[1], cur[2])
    w = np.linspace(0, 1, x.size).reshape(x.shape)
    cx, cv, cr = w.copy(), 2.0 * cur[1], np.zeros(rho.shape)
    for kind, st in reversed(states):
        if kind == "shift":
            gx, gr = orc.shift_vjp(p, st[0], st[2], beta, cx)
            cx, cr = cx + gx, cr + gr
        else:
            cx, cv, cr = orc.step_adjoint(p, *st, cx, cv, cr)
    for got, want in ((tx.grad, cx), (tv.grad, cv), (tr.grad, cr)):
        got = got.cpu().numpy()
        assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_shift_batch_invariance():
    specs = [SimSpec(2, 20, jitter=0.25), SimSpec(2, 29, jitter=0.25)]
    states = [_state(s, 40 + k, "f32") for k, s in enumerate(specs)]
    solo = []
    for s, st in zip(specs, states):
        p = _plan([s], "f32")
        g = _gpu(st, "f32")
        p.shift(*g, 0.5)
        solo.append(g[0].cpu().numpy())
    cat = [np.concatenate([st[k] for st in states], axis=-1) for k in range(3)]
    pb = _plan(specs, "f32")
    for lanes in ((4, 4), (2, 8)):
        pb.set_tuning(*lanes)
        g = _gpu(cat, "f32")
        pb.shift(*g, 0.5)
        out = g[0].cpu().numpy()
        off = 0
        for s, ref in zip(specs, solo):
            np.testing.assert_array_equal(out[..., off:off + s.n], ref)
            off += s.n
