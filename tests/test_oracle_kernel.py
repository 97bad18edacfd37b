"""Pins of the oracle's Wendland-C4 kernel (App. A.1) against mathematics and printed values."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kernel_constants.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        name, dim, val = line.split()
        out[(name, int(dim))] = eval(val, {"pi": math.pi})
    return out


def _radial_moment(orc, dim, power, H=1.0):
    """int |r|^power W(r) dV over R^d, by adaptive quadrature of the radial integral."""
    surf = 2.0 * math.pi if dim == 2 else 4.0 * math.pi

    def f(r):
        e = [r] + [0.0] * (dim - 1)
        return surf * r ** (dim - 1) * r ** power * orc.w(dim, H, e)

    val, _ = integrate.quad(f, 0.0, H, epsabs=1e-15, epsrel=1e-13, limit=200)
    return val


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("H", [1.0, 0.125, 0.0625])
def test_normalisation(orc, dim, H):
    # A kernel is normalised: int W dV = 1 (App. A.1, kernel definition)
    assert abs(_radial_moment(orc, dim, 0, H) - 1.0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_printed_constants(orc, dim):
    g = _golden()
    assert orc.cd(dim) == pytest.approx(g[("C_d", dim)], rel=1e-15)
    sigma2 = _radial_moment(orc, dim, 2) / dim
    scale = 1.0 / (2.0 * math.sqrt(sigma2))
    # the paper prints six decimals; the 2D figure differs from the exact second
    # moment in its last digit (2.1712406 vs 2.171239)
    assert scale == pytest.approx(g[("kernel_scale", dim)], abs=2e-6)


def test_shape_endpoints(orc):
    assert orc.what(0.0) == 1.0
    for q in (1.0, 1.5, 7.0):
        assert orc.what(q) == 0.0 and orc.what_d1(q) == 0.0 and orc.what_d2(q) == 0.0
    # C4 smoothness at the support edge: value, slope and curvature vanish
    q = 1.0 - 1e-4
    assert abs(orc.what(q)) < 1e-20 and abs(orc.what_d1(q)) < 1e-16 and abs(orc.what_d2(q)) < 1e-12
    # monotone decreasing on [0, 1)
    qs = np.linspace(0, 0.999, 500)
    vals = np.array([orc.what(q) for q in qs])
    assert np.all(np.diff(vals) < 0)


def test_shape_derivatives_fd(orc):
    h = 1e-6
    for q in np.linspace(0.01, 0.99, 41):
        fd1 = (orc.what(q + h) - orc.what(q - h)) / (2 * h)
        fd2 = (orc.what_d1(q + h) - orc.what_d1(q - h)) / (2 * h)
        assert orc.what_d1(q) == pytest.approx(fd1, rel=1e-7, abs=1e-9)
        assert orc.what_d2(q) == pytest.approx(fd2, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_and_hessian_fd(orc, dim):
    rng = np.random.default_rng(5)
    H = 0.3
    h = 1e-7
    for _ in range(30):
        e = rng.uniform(-1, 1, dim)
        e *= rng.uniform(0.02, 0.98) * H / np.linalg.norm(e)
        g = orc.gradw(dim, H, e)
        Hm = orc.hessw(dim, H, e)
        for k in range(dim):
            d = np.zeros(dim)
            d[k] = h
            fd = (orc.w(dim, H, e + d) - orc.w(dim, H, e - d)) / (2 * h)
            assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.abs(g).max())
            fdg = (orc.gradw(dim, H, e + d) - orc.gradw(dim, H, e - d)) / (2 * h)
            np.testing.assert_allclose(Hm[:, k], fdg, rtol=1e-5, atol=1e-6 * np.abs(Hm).max())
        # the gradient points from the neighbour towards the particle's own side
        # with negative radial slope: grad W . e < 0 inside the support
        assert float(g @ e) < 0


@pytest.mark.parametrize("dim", [2, 3])
def test_hessian_regular_at_zero(orc, dim):
    # Sec. 3.3: the Hessian needs a well-defined zero-separation value; for C4 the
    # limit exists and equals C_d/H^(d+2) w''(0) Id
    H = 0.5
    h0 = orc.hessw(dim, H, np.zeros(dim))
    for s in (1e-5, 1e-7):
        e = np.full(dim, s)
        np.testing.assert_allclose(orc.hessw(dim, H, e), h0, rtol=1e-4, atol=1e-4 * abs(h0[0, 0]))
    np.testing.assert_allclose(h0, orc.cd(dim) / H ** (dim + 2) * orc.what_d2(0.0) * np.eye(dim))


# -- Poisson summation: lattice sums of W and of x (x) grad W from the kernel's Fourier transform

def _ft(orc, dim, kappa, H):
    """Radial Fourier transform phi(kappa) of W and its derivative d phi / d kappa."""
    if dim == 2:
        f = lambda r: 2 * math.pi * r * orc.w(2, H, [r, 0.0]) * special.j0(kappa * r)
        fp = lambda r: -2 * math.pi * r * r * orc.w(2, H, [r, 0.0]) * special.j1(kappa * r)
    else:
        def sinc(z):
            return math.sin(z) / z if z != 0 else 1.0

        def dsinc(z):
            return (z * math.cos(z) - math.sin(z)) / (z * z) if z != 0 else 0.0
        f = lambda r: 4 * math.pi * r * r * orc.w(3, H, [r, 0.0, 0.0]) * sinc(kappa * r)
        fp = lambda r: 4 * math.pi * r ** 3 * orc.w(3, H, [r, 0.0, 0.0]) * dsinc(kappa * r)
    opts = dict(epsabs=1e-16, epsrel=1e-13, limit=400)
    return integrate.quad(f, 0, H, **opts)[0], integrate.quad(fp, 0, H, **opts)[0]


def _shells(dim, kmax):
    """Reciprocal lattice vectors grouped by |k|^2: {k2: count}."""
    rng = range(-kmax, kmax + 1)
    out = {}
    if dim == 2:
        for a in rng:
            for b in rng:
                k2 = a * a + b * b
                if 0 < k2 <= kmax * kmax:
                    out[k2] = out.get(k2, 0) + 1
    else:
        for a in rng:
            for b in rng:
                for c in rng:
                    k2 = a * a + b * b + c * c
                    if 0 < k2 <= kmax * kmax:
                        out[k2] = out.get(k2, 0) + 1
    return out


@pytest.mark.parametrize("dim,k1,k2", [(2, 12, 16), (3, 10, 14)])
def test_lattice_sums_poisson(orc, dim, k1, k2):
    """Perfect lattice, H = 4 dx: the oracle's summation density and first moment of
    grad W equal their Poisson-summation values, an independent route through the
    kernel's Fourier transform (sum_n dx^d f(n dx) = sum_k f_hat(2 pi k / dx)).
    The transform of C4 decays as kappa^-(d+5), so the truncated series has a K^-5
    tail; two cutoffs K1 < K2 are combined by Richardson extrapolation."""
    from paper_2507_21684_amd.inputs import SimSpec, make_state
    side = 32 if dim == 2 else 16
    spec = SimSpec(dim, side, jitter=0.0)
    x, v, rho = make_state(spec, 0)
    v[:] = 0.0
    p = orc.Params(**spec.params())
    _, _, rs = orc.rhs(p, x, v, rho)
    dx, H = spec.dx, spec.H
    sums = {}
    for K in (k1, k2):
        dens, mom = 1.0, 1.0
        for kk, cnt in _shells(dim, K).items():
            kappa = 2 * math.pi * math.sqrt(kk) / dx
            phi, dphi = _ft(orc, dim, kappa, H)
            dens += cnt * phi
            mom += cnt * (phi + kappa * dphi / dim)
        sums[K] = (dens, mom)
    w1, w2 = k1 ** 5, k2 ** 5
    dens = (w2 * sums[k2][0] - w1 * sums[k1][0]) / (w2 - w1)
    mom = (w2 * sums[k2][1] - w1 * sums[k1][1]) / (w2 - w1)
    assert np.all(np.abs(rs / spec.rho0 - dens) < 5e-11), (rs[0], dens, sums)
    # first moment sum_j V_j (x_j - x_i) (x) grad_i W_ij on the lattice, via the oracle's gradw
    offs = np.array(np.meshgrid(*[np.arange(-4, 5)] * dim, indexing="ij")).reshape(dim, -1).T * dx
    M = np.zeros((dim, dim))
    for y in offs:
        g = orc.gradw(dim, H, -y)   # grad_i W_ij at x_ij = -(x_j - x_i)
        M += dx ** dim * np.outer(y, g)
    np.testing.assert_allclose(M, mom * np.eye(dim), atol=5e-10)
