"""Pins of the oracle's right-hand side and integrator (Sec. 2.3, Sec. 3.4, App. A.3)
against invariants, closed forms and physical sign checks."""
import math

import numpy as np
import pytest

from paper_2507_21684_amd.inputs import SimSpec, make_state


def _random_state(dim, side, seed, jitter=0.2, vscale=1.0, rho_noise=0.01):
    spec = SimSpec(dim, side, jitter=jitter)
    x, v, rho = make_state(spec, seed)
    rng = np.random.default_rng(seed + 100)
    v = vscale * rng.normal(size=v.shape)
    rho = spec.rho0 * (1.0 + rho_noise * rng.uniform(-1, 1, size=rho.shape))
    return spec, x, v, rho


def _params(orc, spec, **kw):
    d = spec.params()
    d.update(kw)
    return orc.Params(**d)


@pytest.mark.parametrize("dim,side", [(2, 24), (3, 12)])
def test_uniform_pressure_on_lattice_gives_no_force(orc, dim, side):
    # Perfect lattice, uniform rho != rho0, v = 0: p is uniform, every pair term is
    # balanced by its mirror image, so a = 0 and drho/dt = 0 (to rounding)
    spec = SimSpec(dim, side, jitter=0.0)
    x, v, rho = make_state(spec, 0)
    v[:] = 0.0
    rho[:] = 1.003
    drho, a, _ = orc.rhs(_params(orc, spec), x, v, rho)
    scale = spec.c0 ** 2 * 0.003 * 7 / spec.H  # |p|/H order of a single term
    assert np.abs(a).max() < 1e-10 * scale
    assert np.abs(drho).max() < 1e-12


@pytest.mark.parametrize("dim,side", [(2, 20), (3, 11)])
def test_momentum_conserved(orc, dim, side):
    # pressure (summation form) and artificial viscosity are antisymmetric per pair:
    # sum_i m a_i = 0 for any state
    spec, x, v, rho = _random_state(dim, side, 3)
    _, a, _ = orc.rhs(_params(orc, spec), x, v, rho)
    tot = (spec.mass * a).sum(axis=1)
    assert np.abs(tot).max() < 1e-12 * spec.mass * np.abs(a).sum()


@pytest.mark.parametrize("dim,side", [(2, 20), (3, 11)])
def test_density_diffusion_conserves_mass_and_smooths(orc, dim, side):
    # v = 0 leaves only the delta term: its flux is antisymmetric, so
    # sum_i V_i drho_i = 0, and it is diffusive: sum_i V_i rho_i drho_i <= 0
    spec, x, v, rho = _random_state(dim, side, 4, rho_noise=0.05)
    v[:] = 0.0
    drho, _, _ = orc.rhs(_params(orc, spec), x, v, rho)
    V = spec.mass / rho
    assert abs((V * drho).sum()) < 1e-12 * (V * np.abs(drho)).sum()
    assert (V * rho * drho).sum() < 0
    # without delta the density does not change
    drho0, _, _ = orc.rhs(_params(orc, spec, delta=0.0), x, v, rho)
    assert np.abs(drho0).max() == 0.0


@pytest.mark.parametrize("dim,side", [(2, 20), (3, 11)])
def test_artificial_viscosity_dissipates(orc, dim, side):
    # uniform density (no pressure force): the viscous power sum_i m v_i . a_i <= 0
    spec, x, v, rho = _random_state(dim, side, 5, rho_noise=0.0)
    _, a, _ = orc.rhs(_params(orc, spec), x, v, rho)
    assert (spec.mass * v * a).sum() < 0
    _, a0, _ = orc.rhs(_params(orc, spec, alpha=0.0), x, v, rho)
    assert np.abs(a0).max() == 0.0


@pytest.mark.parametrize("dim,side", [(2, 20), (3, 11)])
def test_galilean_translation_permutation(orc, dim, side):
    spec, x, v, rho = _random_state(dim, side, 6)
    p = _params(orc, spec)
    d0, a0, s0 = orc.rhs(p, x, v, rho)
    U = np.array([0.7, -1.3, 0.4][:dim])[:, None]
    d1, a1, s1 = orc.rhs(p, x, v + U, rho)
    np.testing.assert_allclose(d1, d0, rtol=1e-9, atol=1e-9 * np.abs(d0).max())
    np.testing.assert_allclose(a1, a0, rtol=1e-9, atol=1e-9 * np.abs(a0).max())
    shift = np.array([0.3711, -2.25, 5.125][:dim])[:, None]
    d2, a2, s2 = orc.rhs(p, x + shift, v, rho)
    np.testing.assert_allclose(d2, d0, rtol=1e-8, atol=1e-8 * np.abs(d0).max())
    np.testing.assert_allclose(a2, a0, rtol=1e-8, atol=1e-8 * np.abs(a0).max())
    np.testing.assert_allclose(s2, s0, rtol=1e-12)
    perm = np.random.default_rng(1).permutation(rho.shape[0])
    d3, a3, s3 = orc.rhs(p, x[:, perm], v[:, perm], rho[perm])
    np.testing.assert_allclose(d3, d0[perm], rtol=1e-12, atol=1e-13 * np.abs(d0).max())
    np.testing.assert_allclose(a3, a0[:, perm], rtol=1e-12, atol=1e-13 * np.abs(a0).max())


def test_continuity_sign_and_magnitude(orc):
    # v = (A sin 2 pi x, 0) on a lattice, rho = rho0: drho/dt = -rho div v
    # = -2 pi A rho0 cos(2 pi x), up to the discretisation error
    spec = SimSpec(2, 64, jitter=0.0)
    x, v, rho = make_state(spec, 0)
    A = 0.5
    v[0] = A * np.sin(2 * math.pi * x[0])
    v[1] = 0.0
    drho, _, _ = orc.rhs(_params(orc, spec), x, v, rho)
    exact = -2 * math.pi * A * spec.rho0 * np.cos(2 * math.pi * x[0])
    assert np.abs(drho - exact).max() < 0.02 * np.abs(exact).max()


def test_pressure_sign_and_magnitude(orc):
    # rho = rho0 (1 + e sin 2 pi x), v = 0: a = -grad p / rho with dp/drho = c0^2 (rho/rho0)^6
    spec = SimSpec(2, 64, jitter=0.0)
    x, v, rho = make_state(spec, 0)
    v[:] = 0.0
    e = 1e-3
    rho = spec.rho0 * (1 + e * np.sin(2 * math.pi * x[0]))
    _, a, _ = orc.rhs(_params(orc, spec, delta=0.0), x, v, rho)
    dpdx = spec.c0 ** 2 * (rho / spec.rho0) ** 6 * spec.rho0 * e * 2 * math.pi * np.cos(2 * math.pi * x[0])
    exact = -dpdx / rho
    assert np.abs(a[0] - exact).max() < 0.02 * np.abs(exact).max()
    assert np.abs(a[1]).max() < 1e-9 * np.abs(exact).max()


def test_integrator_kick_then_drift(orc):
    # semi-implicit Euler (Sec. 3.4): v' = v + dt a, rho' = rho + dt drho, x' = x + dt v'
    spec, x, v, rho = _random_state(2, 16, 7)
    p = _params(orc, spec)
    drho, a, _ = orc.rhs(p, x, v, rho)
    x1, v1, r1 = orc.step(p, x, v, rho, 1)
    dt = p.dt
    np.testing.assert_allclose(v1 - v, dt * a, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(r1 - rho, dt * drho, rtol=1e-10, atol=1e-16)
    np.testing.assert_allclose(x1 - x - dt * v, dt * dt * a, rtol=1e-6, atol=1e-15)
    # zero steps is the identity; two single steps equal one double step
    x0, v0, r0 = orc.step(p, x, v, rho, 0)
    assert np.array_equal(x0, x) and np.array_equal(v0, v) and np.array_equal(r0, rho)
    xa, va, ra = orc.step(p, x1, v1, r1, 1)
    xb, vb, rb = orc.step(p, x, v, rho, 2)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ra, rb)


def test_single_particle_drifts(orc):
    spec = SimSpec(2, 16)
    p = _params(orc, spec)
    x = np.array([[0.3], [0.9]])
    v = np.array([[0.5], [-0.25]])
    rho = np.array([1.2])
    x1, v1, r1 = orc.step(p, x, v, rho, 3)
    np.testing.assert_allclose(x1, x + 3 * p.dt * v, rtol=1e-15)
    assert np.array_equal(v1, v) and np.array_equal(r1, rho)


def test_rhs_sample_matches_full(orc):
    spec, x, v, rho = _random_state(3, 11, 8)
    p = _params(orc, spec)
    d, a, s = orc.rhs(p, x, v, rho)
    idx = np.array([0, 5, 17, 300, 1330])
    ds, as_, ss = orc.rhs_sample(p, x, v, rho, idx)
    np.testing.assert_allclose(ds, d[idx], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(as_, a[:, idx], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ss, s[idx], rtol=1e-13)


@pytest.mark.parametrize("dim,side,steps,amp", [(2, 64, 64, 1.0), (2, 32, 512, 2.0), (2, 32, 512, 0.5),
                                                 (3, 16, 32, 1.0), (3, 12, 96, 2.0)])
def test_taylor_green_stays_bounded_and_decays(orc, dim, side, steps, amp):
    # the time step dt = 0.25 h / c0 with h = H / 2: the TGV kinetic energy stays bounded
    # (never above its start, up to acoustic noise) and decays, also over rollouts several
    # times longer than the configured ones and at the largest amplitude of the batches
    spec = SimSpec(dim, side, amplitude=amp)
    x, v, rho = make_state(spec, 0)
    p = _params(orc, spec)
    ke0 = 0.5 * spec.mass * (v ** 2).sum()
    kes = []
    for _ in range(steps // 8):
        x, v, rho = orc.step(p, x, v, rho, 8)
        kes.append(0.5 * spec.mass * (v ** 2).sum())
    assert np.all(np.isfinite(kes))
    assert kes[-1] < ke0 and max(kes) < 1.01 * ke0
    assert np.abs(rho - spec.rho0).max() < 0.15


def test_time_step_with_h_equal_to_support_is_unstable(orc):
    # the rejected reading h = H in dt = 0.25 h / c0 (dt = dx / c0): the same flow blows up
    # within a few hundred steps, while the adopted step above stays bounded for 512
    spec = SimSpec(2, 32, amplitude=1.0, cfl=0.25)
    x, v, rho = make_state(spec, 0)
    p = _params(orc, spec)
    ke0 = (v ** 2).sum()
    grew = False
    for _ in range(256 // 8):
        x, v, rho = orc.step(p, x, v, rho, 8)
        ke = (v ** 2).sum()
        if not np.isfinite(ke) or ke > 10 * ke0:
            grew = True
            break
    assert grew