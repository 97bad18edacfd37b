"""Pins of the oracle's adjoint (Sec. 2.2 vector-Jacobian products, Sec. 3.3) against
central finite differences of its own forward step, which shares no code with the
hand-written reverse mode."""
import numpy as np
import pytest

from paper_2507_21684_amd.inputs import SimSpec, make_state


def _params(orc, spec, **kw):
    d = spec.params()
    d.update(kw)
    return orc.Params(**d)


@pytest.mark.parametrize("dim", [2, 3])
def test_pair_partials_fd(orc, dim):
    spec = SimSpec(dim, 16)
    p = _params(orc, spec, alpha=0.3, delta=0.2)  # large coefficients: every term matters
    rng = np.random.default_rng(11)
    h = 1e-7
    for _ in range(25):
        e = rng.uniform(-1, 1, dim)
        e *= rng.uniform(0.05, 0.97) * spec.H / np.linalg.norm(e)
        vi, vj = rng.normal(size=dim), rng.normal(size=dim)
        ri, rj = 1 + 0.02 * rng.uniform(-1, 1), 1 + 0.02 * rng.uniform(-1, 1)
        ab, rb = rng.normal(size=dim), rng.normal()

        def phi(e_, vi_, vj_, ri_, rj_):
            a, r = orc.pair_terms(p, e_, vi_, vj_, ri_, rj_)
            return float(ab @ a + rb * r)

        g = orc.pair_partials(p, e, vi, vj, ri, rj, ab, rb)
        scale = max(abs(phi(e, vi, vj, ri, rj)), 1e-30)
        for k in range(dim):
            dk = np.zeros(dim)
            dk[k] = h * spec.H
            fd = (phi(e + dk, vi, vj, ri, rj) - phi(e - dk, vi, vj, ri, rj)) / (2 * h * spec.H)
            assert g["de"][k] == pytest.approx(fd, rel=2e-6, abs=1e-7 * scale / spec.H)
            dk = np.zeros(dim)
            dk[k] = h
            fd = (phi(e, vi + dk, vj, ri, rj) - phi(e, vi - dk, vj, ri, rj)) / (2 * h)
            assert g["dvi"][k] == pytest.approx(fd, rel=2e-6, abs=1e-7 * scale)
            fd = (phi(e, vi, vj + dk, ri, rj) - phi(e, vi, vj - dk, ri, rj)) / (2 * h)
            assert g["dvj"][k] == pytest.approx(fd, rel=2e-6, abs=1e-7 * scale)
        fd = (phi(e, vi, vj, ri + h, rj) - phi(e, vi, vj, ri - h, rj)) / (2 * h)
        assert g["dri"] == pytest.approx(fd, rel=2e-6, abs=1e-7 * scale)
        fd = (phi(e, vi, vj, ri, rj + h) - phi(e, vi, vj, ri, rj - h)) / (2 * h)
        assert g["drj"] == pytest.approx(fd, rel=2e-6, abs=1e-7 * scale)


def _state(dim, side, seed):
    spec = SimSpec(dim, side, jitter=0.25)
    x, v, rho = make_state(spec, seed)
    rng = np.random.default_rng(seed)
    v = v + 0.3 * rng.normal(size=v.shape)
    rho = rho * (1 + 0.01 * rng.uniform(-1, 1, size=rho.shape))
    return spec, x, v, rho


@pytest.mark.parametrize("dim,side", [(2, 12), (3, 9)])
def test_step_vjp_dot_product(orc, dim, side):
    """<J du, w> from central differences of the forward step equals <du, J^T w>."""
    spec, x, v, rho = _state(dim, side, 21)
    p = _params(orc, spec, alpha=0.05, delta=0.1)
    rng = np.random.default_rng(22)
    for trial in range(3):
        dx_, dv_, dr_ = rng.normal(size=x.shape), rng.normal(size=v.shape), rng.normal(size=rho.shape)
        dx_ *= spec.dx
        dr_ *= 0.01
        wx, wv, wr = rng.normal(size=x.shape), rng.normal(size=v.shape), rng.normal(size=rho.shape)
        h = 1e-6
        xp, vp, rp = orc.step(p, x + h * dx_, v + h * dv_, rho + h * dr_, 1)
        xm, vm, rm = orc.step(p, x - h * dx_, v - h * dv_, rho - h * dr_, 1)
        jvp = (np.sum(wx * (xp - xm)) + np.sum(wv * (vp - vm)) + np.sum(wr * (rp - rm))) / (2 * h)
        gx, gv, gr = orc.step_adjoint(p, x, v, rho, wx, wv, wr)
        vjp = np.sum(gx * dx_) + np.sum(gv * dv_) + np.sum(gr * dr_)
        assert vjp == pytest.approx(jvp, rel=1e-7), (trial, vjp, jvp)


@pytest.mark.parametrize("dim,side", [(2, 12), (3, 9)])
def test_step_vjp_each_field(orc, dim, side):
    """Each input field's cotangent separately, against directional differences."""
    spec, x, v, rho = _state(dim, side, 31)
    p = _params(orc, spec)
    rng = np.random.default_rng(32)
    wx, wv, wr = rng.normal(size=x.shape), rng.normal(size=v.shape), rng.normal(size=rho.shape)
    gx, gv, gr = orc.step_adjoint(p, x, v, rho, wx, wv, wr)
    h = 1e-6

    def proj(xx, vv, rr):
        a, b, c = orc.step(p, xx, vv, rr, 1)
        return np.sum(wx * a) + np.sum(wv * b) + np.sum(wr * c)

    for field, g in (("x", gx), ("v", gv), ("rho", gr)):
        d = rng.normal(size=g.shape)
        if field == "x":
            fd = (proj(x + h * spec.dx * d, v, rho) - proj(x - h * spec.dx * d, v, rho)) / (2 * h * spec.dx)
        elif field == "v":
            fd = (proj(x, v + h * d, rho) - proj(x, v - h * d, rho)) / (2 * h)
        else:
            fd = (proj(x, v, rho + 1e-2 * h * d) - proj(x, v, rho - 1e-2 * h * d)) / (2e-2 * h)
        assert np.sum(g * d) == pytest.approx(fd, rel=1e-6), field


def test_rollout_gradient_fd(orc):
    """Gradient of L = sum |v_T|^2 after 4 steps with respect to v0, x0 and rho0."""
    spec, x, v, rho = _state(2, 12, 41)
    p = _params(orc, spec)
    T = 4
    out = orc.rollout(p, x, v, rho, T, 0)
    rng = np.random.default_rng(42)
    h = 1e-6

    def loss(xx, vv, rr):
        _, vT, _ = orc.step(p, xx, vv, rr, T)
        return float((vT ** 2).sum())

    assert out["loss"] == pytest.approx(loss(x, v, rho), rel=1e-14)
    for name, g, base in (("v", out["gv0"], 1.0), ("x", out["gx0"], spec.dx), ("rho", out["grho0"], 1e-2)):
        d = rng.normal(size=g.shape) * base
        args_p = [x, v, rho]
        args_m = [x, v, rho]
        k = {"x": 0, "v": 1, "rho": 2}[name]
        args_p = list(args_p)
        args_m = list(args_m)
        args_p[k] = args_p[k] + h * d
        args_m[k] = args_m[k] - h * d
        fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
        assert np.sum(g * d) == pytest.approx(fd, rel=1e-6), name


def test_rollout_ke_loss_seed(orc):
    spec, x, v, rho = _state(3, 9, 51)
    p = _params(orc, spec)
    out = orc.rollout(p, x, v, rho, 0, 1)
    np.testing.assert_allclose(out["gv0"], spec.mass * v, rtol=1e-15)
    assert out["loss"] == pytest.approx(0.5 * spec.mass * (v ** 2).sum(), rel=1e-14)
    assert np.all(out["gx0"] == 0) and np.all(out["grho0"] == 0)


def test_sampled_sweep_matches_step_adjoint(orc):
    """The sampled adjoint sweep (used for large-state checks) reproduces step_adjoint."""
    spec, x, v, rho = _state(3, 9, 61)
    p = _params(orc, spec)
    rng = np.random.default_rng(62)
    wx, wv, wr = rng.normal(size=x.shape), rng.normal(size=v.shape), rng.normal(size=rho.shape)
    gx, gv, gr = orc.step_adjoint(p, x, v, rho, wx, wv, wr)
    vt = wv + p.dt * wx
    abar, rbar = p.dt * vt, p.dt * wr
    idx = np.array([0, 3, 100, 728])
    sx, sv, sr = orc.adjoint_sweep_sample(p, x, v, rho, abar, rbar, idx)
    np.testing.assert_allclose(sx, (gx - wx)[:, idx], rtol=1e-9, atol=1e-12 * np.abs(gx).max())
    np.testing.assert_allclose(sv, (gv - vt)[:, idx], rtol=1e-9, atol=1e-12 * np.abs(gv).max())
    np.testing.assert_allclose(sr, (gr - wr)[idx], rtol=1e-9, atol=1e-12 * np.abs(gr).max())
