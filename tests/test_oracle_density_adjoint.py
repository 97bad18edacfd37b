"""Pins of the oracle's summation-density vector-Jacobian product (the backward benchmark of
Sec. 4.1: summation density after one step, gradient with respect to the initial positions).

Each pin is independent of the function's own formula: central finite differences of the
loss sum_i g_i rho_i(x) computed by the oracle's forward density sum, the translation
invariance of that loss, and the symmetry of a perfect lattice.
"""
import numpy as np
import pytest

from paper_2507_21684_amd.inputs import SimSpec, make_state


def _params(orc, spec):
    return orc.Params(**spec.params())


def _loss(orc, p, x, g):
    _, _, rs = orc.rhs(p, x, np.zeros_like(x), np.ones(x.shape[1]))
    return float(np.dot(g, rs))


@pytest.mark.parametrize("dim,side", [(2, 12), (3, 10)])
def test_density_adjoint_matches_finite_differences(orc, dim, side):
    spec = SimSpec(dim, side)
    x, _, _ = make_state(spec, 3)
    rng = np.random.default_rng(11)
    x = x + 0.2 * spec.dx * rng.uniform(-1, 1, size=x.shape)   # break the lattice symmetry
    g = rng.normal(size=x.shape[1])
    p = _params(orc, spec)
    xbar = orc.density_adjoint(p, x, g)
    h = 1e-6 * spec.dx
    scale = np.abs(xbar).max()
    for k, i in [(0, 0), (1, 5), (0, 37), (dim - 1, x.shape[1] - 1), (1, x.shape[1] // 2)]:
        xp, xm = x.copy(), x.copy()
        xp[k, i] += h
        xm[k, i] -= h
        fd = (_loss(orc, p, xp, g) - _loss(orc, p, xm, g)) / (2 * h)
        assert abs(fd - xbar[k, i]) <= 1e-6 * scale, (k, i, fd, xbar[k, i])


def test_density_adjoint_translation_invariance(orc):
    # the loss does not change when every particle moves by the same vector
    spec = SimSpec(2, 16)
    x, _, _ = make_state(spec, 5)
    g = np.random.default_rng(2).normal(size=x.shape[1])
    xbar = orc.density_adjoint(_params(orc, spec), x, g)
    assert np.abs(xbar.sum(axis=1)).max() <= 1e-12 * np.abs(xbar).max() * x.shape[1]


def test_density_adjoint_vanishes_on_a_perfect_lattice(orc):
    # uniform cotangent on a perfect lattice: every particle sees a point-symmetric neighbourhood
    spec = SimSpec(2, 16, jitter=0.0)
    x, _, _ = make_state(spec, 0)
    p = _params(orc, spec)
    xbar = orc.density_adjoint(p, x, np.ones(x.shape[1]))
    ref = orc.density_adjoint(p, x + 0.3 * spec.dx * np.random.default_rng(1).uniform(-1, 1, x.shape),
                              np.ones(x.shape[1]))
    assert np.abs(xbar).max() <= 1e-12 * np.abs(ref).max()


def test_backward_benchmark_gradient_composition(orc):
    # L(x0) = sum_i rho_i(x1), x1 = step(x0): the gradient is the step adjoint of the density
    # adjoint with cotangent (xbar1, 0, 0); pinned by finite differences of the composed forward
    spec = SimSpec(2, 10)
    x0, v0, r0 = make_state(spec, 4)
    p = _params(orc, spec)
    x1, v1, r1 = orc.step(p, x0, v0, r0, 1)
    xb1 = orc.density_adjoint(p, x1, np.ones(x0.shape[1]))
    gx, gv, gr = orc.step_adjoint(p, x0, v0, r0, xb1, np.zeros_like(v0), np.zeros_like(r0))

    def L(x, v, r):
        xs, _, _ = orc.step(p, x, v, r, 1)
        return _loss(orc, p, xs, np.ones(x.shape[1]))

    h = 1e-6 * spec.dx
    for k, i in [(0, 3), (1, 50), (0, 99)]:
        xp, xm = x0.copy(), x0.copy()
        xp[k, i] += h
        xm[k, i] -= h
        fd = (L(xp, v0, r0) - L(xm, v0, r0)) / (2 * h)
        assert abs(fd - gx[k, i]) <= 1e-6 * np.abs(gx).max()
    hv = 1e-3    # the loss depends on v0 only through dt^2 a-terms: a larger step beats rounding
    for k, i in [(1, 7), (0, 42)]:
        vp, vm = v0.copy(), v0.copy()
        vp[k, i] += hv
        vm[k, i] -= hv
        fd = (L(x0, vp, r0) - L(x0, vm, r0)) / (2 * hv)
        assert abs(fd - gv[k, i]) <= 1e-6 * np.abs(gv).max()
