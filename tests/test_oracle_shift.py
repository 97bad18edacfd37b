"""Pins of the oracle's particle shifting (the delta-plus form, applied after a step) and of its VJP.

Independent checks: a perfect lattice is not shifted; for uniform volumes the shift is a descent
step on E = sum_i sum_j V [W_ij + R W_ij^5 / (5 W(dx)^4)], equal to -(beta H^2 / 2) dE/dx (against
central differences of E evaluated by brute force) and lowering E; it scales with the neighbours'
volumes V_j = m / rho_j and not with the particle's own; the VJP matches central differences.
"""
import numpy as np
import pytest

from paper_2507_21684_amd.inputs import SimSpec, make_state


def _p(orc, spec):
    return orc.Params(**spec.params())


def test_lattice_is_not_shifted(orc):
    spec = SimSpec(2, 16, jitter=0.0)
    x, _, rho = make_state(spec, 0)
    dr = orc.shift(_p(orc, spec), x, rho, 0.5)
    assert np.abs(dr).max() <= 1e-12 * spec.dx


def _energy(orc, p, x, V, w0):
    """E = sum_i sum_{j != i} V [W_ij + R W_ij^5 / (5 w0^4)] by brute force (periodic, minimum image)."""
    n = x.shape[1]
    E = 0.0
    for i in range(n):
        e = x[:, i:i + 1] - x
        e -= p.L * np.rint(e / p.L)
        r = np.sqrt((e ** 2).sum(axis=0))
        q = r / p.H
        Wv = np.array([orc.w(p.dim, p.H, e[:, j].copy()) if q[j] < 1 and j != i else 0.0 for j in range(n)])
        E += V * (Wv + 0.2 * Wv ** 5 / (5 * w0 ** 4)).sum()
    return E


def test_shift_is_a_descent_step(orc):
    spec = SimSpec(2, 12, jitter=0.3)
    x, _, rho = make_state(spec, 3)
    p = _p(orc, spec)
    V = p.m / p.rho0
    rho = np.full(rho.shape, p.rho0)
    w0 = orc.w(2, p.H, np.array([spec.dx, 0.0]))
    beta = 1e-3
    dr = orc.shift(p, x, rho, beta)
    # dr = -(beta H^2 / 2) dE/dx: compare with central differences of E
    h = 1e-6 * spec.dx
    for (k, i) in ((0, 3), (1, 17), (0, 40)):
        xp, xm = x.copy(), x.copy()
        xp[k, i] += h
        xm[k, i] -= h
        g = (_energy(orc, p, xp, V, w0) - _energy(orc, p, xm, V, w0)) / (2 * h)
        assert abs(dr[k, i] - (-beta * p.H ** 2 / 2) * g) <= 1e-6 * np.abs(dr).max()
    E0, E1 = _energy(orc, p, x, V, w0), _energy(orc, p, x + dr, V, w0)
    assert E1 < E0


def test_shift_uses_the_neighbours_volumes(orc):
    # dr_i = ... V_j ...: it scales as 1/rho for a uniform density, does not depend on the
    # particle's own density, and changes when a neighbour's does
    spec = SimSpec(2, 12, jitter=0.25)
    x, _, rho = make_state(spec, 5)
    p = _p(orc, spec)
    beta = 0.3
    d1 = orc.shift(p, x, np.full(rho.shape, p.rho0), beta)
    d2 = orc.shift(p, x, np.full(rho.shape, 2 * p.rho0), beta)
    np.testing.assert_allclose(d2, d1 / 2, rtol=1e-12, atol=1e-18)
    i = 37
    r2 = np.full(rho.shape, p.rho0)
    r2[i] = 1.5 * p.rho0
    d3 = orc.shift(p, x, r2, beta)
    np.testing.assert_allclose(d3[:, i], d1[:, i], rtol=1e-12, atol=1e-18)
    assert np.abs(d3 - d1).max() > 1e-3 * np.abs(d1).max()


def test_shift_vjp_matches_finite_differences(orc):
    spec = SimSpec(2, 10, jitter=0.2)
    x, _, rho = make_state(spec, 7)
    rng = np.random.default_rng(8)
    rho = rho * (1 + 0.02 * rng.uniform(-1, 1, size=rho.shape))
    xb = rng.normal(size=x.shape)
    p = _p(orc, spec)
    beta = 0.4
    gx, gr = orc.shift_vjp(p, x, rho, beta, xb)

    def L(x, rho):
        return float((xb * orc.shift(p, x, rho, beta)).sum())

    h = 1e-6
    for (k, i) in ((0, 7), (1, 55), (0, 80)):
        xp, xm = x.copy(), x.copy()
        xp[k, i] += h * spec.dx
        xm[k, i] -= h * spec.dx
        fd = (L(xp, rho) - L(xm, rho)) / (2 * h * spec.dx)
        assert abs(fd - gx[k, i]) <= 1e-6 * np.abs(gx).max(), (k, i, fd, gx[k, i])
    for i in (3, 33, 90):
        rp, rm = rho.copy(), rho.copy()
        rp[i] += h
        rm[i] -= h
        fd = (L(x, rp) - L(x, rm)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * np.abs(gr).max(), (i, fd, gr[i])
