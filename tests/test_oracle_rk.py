"""Pins of the oracle's explicit Runge-Kutta steps (Butcher tableaus) and their adjoints.

Independent checks: a one-stage tableau reproduces explicit Euler built from the oracle's
right-hand side; measured convergence orders match each tableau's order; the update
function's VJP and the RK step adjoint match central finite differences.
"""
import numpy as np
import pytest

from paper_2507_21684_amd.inputs import SimSpec, make_state


def _p(orc, spec, dt=None):
    d = spec.params()
    if dt is not None:
        d["dt"] = dt
    return orc.Params(**d)


def test_one_stage_tableau_is_explicit_euler(orc):
    spec = SimSpec(2, 16)
    x, v, rho = make_state(spec, 1)
    p = _p(orc, spec)
    drho, a, _ = orc.rhs(p, x, v, rho)
    x1, v1, r1 = orc.step_rk(p, x, v, rho, 1, "euler")
    np.testing.assert_allclose(x1, x + p.dt * v, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v1, v + p.dt * a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(r1, rho + p.dt * drho, rtol=0, atol=1e-15)


@pytest.mark.parametrize("scheme,order", [("euler", 1), ("midpoint", 2), ("heun", 2), ("rk4", 4)])
def test_convergence_order(orc, scheme, order):
    spec = SimSpec(2, 16)
    x, v, rho = make_state(spec, 2)
    t_end = 8 * spec.dt
    ref = orc.step_rk(_p(orc, spec, t_end / 256), x, v, rho, 256, "rk4")[1]
    errs = []
    for n in (8, 16, 32):
        vn = orc.step_rk(_p(orc, spec, t_end / n), x, v, rho, n, scheme)[1]
        errs.append(np.abs(vn - ref).max())
    rates = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    assert all(abs(r - order) < 0.35 for r in rates), (scheme, errs, rates)


def test_rhs_vjp_matches_finite_differences(orc):
    spec = SimSpec(2, 10)
    x, v, rho = make_state(spec, 3)
    rng = np.random.default_rng(4)
    rho = rho * (1 + 0.01 * rng.uniform(-1, 1, size=rho.shape))
    ab, rb = rng.normal(size=v.shape), rng.normal(size=rho.shape)
    p = _p(orc, spec)
    gx, gv, gr = orc.rhs_vjp(p, x, v, rho, ab, rb)

    def L(x, v, rho):
        drho, a, _ = orc.rhs(p, x, v, rho)
        return float((ab * a).sum() + (rb * drho).sum())

    h = 1e-6
    for arr, g, idx in ((x, gx, (0, 7)), (x, gx, (1, 55)), (v, gv, (1, 20)), (rho, gr, (33,))):
        ap, am = arr.copy(), arr.copy()
        ap[idx] += h * (spec.dx if arr is x else 1.0)
        am[idx] -= h * (spec.dx if arr is x else 1.0)
        args_p = [ap if arr is t else t for t in (x, v, rho)]
        args_m = [am if arr is t else t for t in (x, v, rho)]
        fd = (L(*args_p) - L(*args_m)) / (2 * h * (spec.dx if arr is x else 1.0))
        assert abs(fd - g[idx]) <= 1e-6 * np.abs(g).max(), (idx, fd, g[idx])


@pytest.mark.parametrize("scheme", ["rk4", "midpoint"])
def test_rk_step_adjoint_matches_finite_differences(orc, scheme):
    spec = SimSpec(2, 10)
    x, v, rho = make_state(spec, 5)
    rng = np.random.default_rng(6)
    wx, wv, wr = rng.normal(size=x.shape), rng.normal(size=v.shape), rng.normal(size=rho.shape)
    p = _p(orc, spec)
    gx, gv, gr = orc.step_rk_adjoint(p, x, v, rho, wx, wv, wr, scheme)

    def L(x, v, rho):
        x1, v1, r1 = orc.step_rk(p, x, v, rho, 1, scheme)
        return float((wx * x1).sum() + (wv * v1).sum() + (wr * r1).sum())

    for arr, g, idx, h in ((x, gx, (0, 11), 1e-7), (x, gx, (1, 90), 1e-7), (v, gv, (0, 42), 1e-6),
                           (rho, gr, (17,), 1e-6)):
        ap, am = arr.copy(), arr.copy()
        ap[idx] += h
        am[idx] -= h
        args_p = [ap if arr is t else t for t in (x, v, rho)]
        args_m = [am if arr is t else t for t in (x, v, rho)]
        fd = (L(*args_p) - L(*args_m)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(np.abs(gx).max(), np.abs(gv).max(), np.abs(gr).max()), (idx, fd, g[idx])
