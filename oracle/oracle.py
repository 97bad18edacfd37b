"""Python wrapper of the plain FP64 CPU oracle (``sph_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark.  The GPU library never imports it, and the
two share no code.  Every function takes and returns numpy float64 arrays in
SoA layout (``x[k, i]`` is coordinate ``k`` of particle ``i``).

What each function computes is documented in ``sph_oracle.c`` with the paper
passage it follows (diffSPH, arXiv 2507.21684: Sec. 2.3 governing equations,
Sec. 3.2 neighbourhood search and periodic domains, Sec. 3.4 integration,
App. A kernels and operators).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wno-unused-variable", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("renorm", ctypes.c_int32), ("L", ctypes.c_double),
                ("H", ctypes.c_double), ("m", ctypes.c_double), ("rho0", ctypes.c_double),
                ("c0", ctypes.c_double), ("delta", ctypes.c_double), ("alpha", ctypes.c_double),
                ("eps", ctypes.c_double), ("dt", ctypes.c_double)]


@dataclass
class Params:
    """Physical and numerical parameters of one simulation (all SI-free units)."""
    dim: int
    L: float
    H: float
    m: float
    rho0: float = 1.0
    c0: float = 10.0
    delta: float = 0.1
    alpha: float = 0.01
    eps: float = 0.01
    dt: float = 0.0
    renorm: int = 0      # 1: delta-diffusion with the renormalised density gradient

    def c(self) -> OrcParams:
        return OrcParams(self.dim, int(self.renorm), self.L, self.H, self.m, self.rho0, self.c0, self.delta,
                         self.alpha, self.eps, self.dt)


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_P = ctypes.POINTER(OrcParams)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_cd.restype = ctypes.c_double
        L.orc_cd.argtypes = [ctypes.c_int]
        for name in ("orc_what", "orc_what_d1", "orc_what_d2"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_double]
        L.orc_w.restype = ctypes.c_double
        L.orc_w.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.orc_gradw.restype = None
        L.orc_gradw.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_hessw.restype = None
        L.orc_hessw.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_neighbors.restype = ctypes.c_int64
        L.orc_neighbors.argtypes = [ctypes.c_int, ctypes.c_int64, _D, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, _I64, _I32, ctypes.c_int64]
        L.orc_pair_terms.restype = None
        L.orc_pair_terms.argtypes = [_P, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_pair_partials.restype = None
        L.orc_pair_partials.argtypes = [_P, _D, _D, _D, ctypes.c_double, ctypes.c_double, _D,
                                        ctypes.c_double, _D]
        L.orc_rhs.restype = ctypes.c_int
        L.orc_rhs.argtypes = [_P, ctypes.c_int64, _D, _D, _D, _D, _D, _D]
        L.orc_rhs_sample.restype = ctypes.c_int
        L.orc_rhs_sample.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int64, _I64, _D, _D, _D]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int32]
        L.orc_rhs_vjp.restype = ctypes.c_int
        L.orc_rhs_vjp.argtypes = [_P, ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_step_rk.restype = ctypes.c_int
        L.orc_step_rk.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int32, ctypes.c_int32, _D, _D]
        L.orc_step_rk_adjoint.restype = ctypes.c_int
        L.orc_step_rk_adjoint.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int32, _D, _D, _D, _D, _D]
        L.orc_step_symplectic.restype = ctypes.c_int
        L.orc_step_symplectic.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, _I64]
        L.orc_step_symplectic_adjoint.restype = ctypes.c_int
        L.orc_step_symplectic_adjoint.argtypes = [_P, ctypes.c_int64, _D, _D, _D, _D, _D, _D]
        L.orc_rollout_symplectic_adjoint.restype = ctypes.c_int
        L.orc_rollout_symplectic_adjoint.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.c_int32, _D, _D, _D]
        L.orc_shift.restype = ctypes.c_int
        L.orc_shift.argtypes = [_P, ctypes.c_int64, _D, _D, ctypes.c_double, _D]
        L.orc_shift_vjp.restype = ctypes.c_int
        L.orc_shift_vjp.argtypes = [_P, ctypes.c_int64, _D, _D, ctypes.c_double, _D, _D, _D]
        L.orc_renorm_gradient.restype = ctypes.c_int
        L.orc_renorm_gradient.argtypes = [_P, ctypes.c_int64, _D, _D, _D, _D]
        L.orc_density_adjoint.restype = ctypes.c_int
        L.orc_density_adjoint.argtypes = [_P, ctypes.c_int64, _D, _D, _D]
        L.orc_step_adjoint.restype = ctypes.c_int
        L.orc_step_adjoint.argtypes = [_P, ctypes.c_int64, _D, _D, _D, _D, _D, _D]
        L.orc_adjoint_sweep_sample.restype = ctypes.c_int
        L.orc_adjoint_sweep_sample.argtypes = [_P, ctypes.c_int64, _D, _D, _D, _D, _D, ctypes.c_int64,
                                               _I64, _D, _D, _D]
        L.orc_rollout.restype = ctypes.c_int
        L.orc_rollout.argtypes = [_P, ctypes.c_int64, _D, _D, _D, ctypes.c_int32, ctypes.c_int32,
                                  _D, _D, _D, _D, _D, _D, _D]
        L.orc_neighbors_adaptive.restype = ctypes.c_int64
        L.orc_neighbors_adaptive.argtypes = [ctypes.c_int, ctypes.c_int64, _D, ctypes.c_double, _D, ctypes.c_int,
                                             ctypes.c_int, _I64, _I32, ctypes.c_int64, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- kernel

def cd(dim: int) -> float:
    return lib().orc_cd(dim)


def what(q: float) -> float:
    return lib().orc_what(float(q))


def what_d1(q: float) -> float:
    return lib().orc_what_d1(float(q))


def what_d2(q: float) -> float:
    return lib().orc_what_d2(float(q))


def w(dim: int, H: float, e) -> float:
    e = _f64(e)
    return lib().orc_w(dim, H, _d(e))


def gradw(dim: int, H: float, e) -> np.ndarray:
    e = _f64(e)
    g = np.zeros(dim)
    lib().orc_gradw(dim, H, _d(e), _d(g))
    return g


def hessw(dim: int, H: float, e) -> np.ndarray:
    e = _f64(e)
    h = np.zeros(dim * dim)
    lib().orc_hessw(dim, H, _d(e), _d(h))
    return h.reshape(dim, dim)


# ---------------------------------------------------------------- neighbours

def neighbors(x, L: float, H: float, prec: str = "f64", brute: bool = False):
    """CSR neighbour lists (offsets int64[n+1], idx int32), rows ascending, self included.

    ``prec`` selects the precision of the predicate: ``"f64"`` or ``"f32"`` (positions
    rounded to float first; the wrap, minimum image and r^2 are then float operations)."""
    x = _f64(x)
    dim, n = x.shape
    off = np.zeros(n + 1, dtype=np.int64)
    p = 1 if prec == "f32" else 0
    total = lib().orc_neighbors(dim, n, _d(x), L, H, p, int(brute), off.ctypes.data_as(_I64), None, 0)
    if total < 0:
        raise ValueError("oracle neighbour search rejected its input")
    idx = np.zeros(max(total, 1), dtype=np.int32)
    total2 = lib().orc_neighbors(dim, n, _d(x), L, H, p, int(brute), off.ctypes.data_as(_I64),
                                 idx.ctypes.data_as(_I32), total)
    assert total2 == total
    return off, idx[:total]


def neighbors_adaptive(x, L: float, h, prec: str = "f64", brute: bool = False):
    """Neighbour lists with per-particle supports h (n values): the search radius
    s_k = max(h_k, max{h_i : r_ik < h_i}), then the pairs r_ij < max(h_i, h_j) found by searching
    with s_i.  Returns (offsets int64[n+1], idx int32, s float64[n]); rows ascending, self
    included; predicates in the working precision as for neighbors()."""
    x, h = _f64(x), _f64(h)
    dim, n = x.shape
    off = np.zeros(n + 1, dtype=np.int64)
    s = np.zeros(n)
    p = 1 if prec == "f32" else 0
    total = lib().orc_neighbors_adaptive(dim, n, _d(x), L, _d(h), p, int(brute), off.ctypes.data_as(_I64), None, 0,
                                         _d(s))
    if total < 0:
        raise ValueError("oracle adaptive neighbour search rejected its input")
    idx = np.zeros(max(total, 1), dtype=np.int32)
    total2 = lib().orc_neighbors_adaptive(dim, n, _d(x), L, _d(h), p, int(brute), off.ctypes.data_as(_I64),
                                          idx.ctypes.data_as(_I32), total, _d(s))
    assert total2 == total
    return off, idx[:total], s


# ---------------------------------------------------------------- physics

def pair_terms(p: Params, e, vi, vj, rhoi: float, rhoj: float):
    e, vi, vj = _f64(e), _f64(vi), _f64(vj)
    a = np.zeros(p.dim)
    r = np.zeros(1)
    pc = p.c()
    lib().orc_pair_terms(ctypes.byref(pc), _d(e), _d(vi), _d(vj), rhoi, rhoj, _d(a), _d(r))
    return a, float(r[0])


def pair_partials(p: Params, e, vi, vj, rhoi: float, rhoj: float, abar, rbar: float):
    e, vi, vj = _f64(np.pad(_f64(e), (0, 3 - p.dim))), _f64(np.pad(_f64(vi), (0, 3 - p.dim))), \
        _f64(np.pad(_f64(vj), (0, 3 - p.dim)))
    ab = _f64(np.pad(_f64(abar), (0, 3 - p.dim)))
    out = np.zeros(11)
    pc = p.c()
    lib().orc_pair_partials(ctypes.byref(pc), _d(e), _d(vi), _d(vj), rhoi, rhoj, _d(ab), rbar, _d(out))
    d = p.dim
    return {"de": out[0:d], "dvi": out[3:3 + d], "dvj": out[6:6 + d], "dri": out[9], "drj": out[10]}


def rhs(p: Params, x, v, rho):
    """(drho/dt, a, rho_sum) of one evaluation of the update function."""
    x, v, rho = _f64(x), _f64(v), _f64(rho)
    n = rho.shape[0]
    drho = np.zeros(n)
    acc = np.zeros((p.dim, n))
    rs = np.zeros(n)
    pc = p.c()
    rc = lib().orc_rhs(ctypes.byref(pc), n, _d(x), _d(v), _d(rho), _d(drho), _d(acc), _d(rs))
    if rc != 0:
        raise ValueError("oracle rhs rejected its input")
    return drho, acc, rs


def rhs_sample(p: Params, x, v, rho, sample):
    """rhs() for the listed particles only, each by a brute-force pass (large states)."""
    x, v, rho = _f64(x), _f64(v), _f64(rho)
    n = rho.shape[0]
    s = np.ascontiguousarray(np.asarray(sample, dtype=np.int64))
    ns = s.shape[0]
    drho = np.zeros(ns)
    acc = np.zeros((p.dim, ns))
    rs = np.zeros(ns)
    pc = p.c()
    rc = lib().orc_rhs_sample(ctypes.byref(pc), n, _d(x), _d(v), _d(rho), ns, s.ctypes.data_as(_I64),
                              _d(drho), _d(acc), _d(rs))
    if rc != 0:
        raise ValueError("oracle rhs_sample rejected its input")
    return drho, acc, rs


def step(p: Params, x, v, rho, nsteps: int = 1):
    """nsteps semi-implicit Euler steps; returns new copies (x, v, rho)."""
    x, v, rho = _f64(x).copy(), _f64(v).copy(), _f64(rho).copy()
    pc = p.c()
    rc = lib().orc_step(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho), nsteps)
    if rc != 0:
        raise ValueError("oracle step rejected its input")
    return x, v, rho


def step_adjoint(p: Params, x, v, rho, xb, vb, rb):
    """Cotangents of the state at the start of a step from those of its output."""
    x, v, rho = _f64(x), _f64(v), _f64(rho)
    xb, vb, rb = _f64(xb).copy(), _f64(vb).copy(), _f64(rb).copy()
    pc = p.c()
    rc = lib().orc_step_adjoint(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho), _d(xb), _d(vb), _d(rb))
    if rc != 0:
        raise ValueError("oracle step_adjoint rejected its input")
    return xb, vb, rb


# Butcher tableaus of the explicit schemes (A strictly lower triangular, weights b).
TABLEAUS = {
    "euler": ([[0.0]], [1.0]),
    "midpoint": ([[0.0, 0.0], [0.5, 0.0]], [0.0, 1.0]),
    "heun": ([[0.0, 0.0], [1.0, 0.0]], [0.5, 0.5]),
    "rk4": ([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]],
            [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
}


def _tableau(scheme):
    A, b = TABLEAUS[scheme] if isinstance(scheme, str) else scheme
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    return A.shape[0], A, b


def rhs_vjp(p: Params, x, v, rho, abar, rbar):
    """J^T terms (xbar, vbar, rhobar) of the update function for cotangents of (a, drho/dt)."""
    x, v, rho, abar, rbar = _f64(x), _f64(v), _f64(rho), _f64(abar), _f64(rbar)
    n = rho.shape[0]
    xb, vb, rb = np.zeros((p.dim, n)), np.zeros((p.dim, n)), np.zeros(n)
    pc = p.c()
    rc = lib().orc_rhs_vjp(ctypes.byref(pc), n, _d(x), _d(v), _d(rho), _d(abar), _d(rbar), _d(xb), _d(vb), _d(rb))
    if rc != 0:
        raise ValueError("oracle rhs_vjp rejected its input")
    return xb, vb, rb


def step_rk(p: Params, x, v, rho, nsteps: int, scheme="rk4"):
    """nsteps explicit Runge-Kutta steps of the named (or given (A, b)) tableau."""
    s, A, b = _tableau(scheme)
    x, v, rho = _f64(x).copy(), _f64(v).copy(), _f64(rho).copy()
    pc = p.c()
    rc = lib().orc_step_rk(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho), nsteps, s, _d(A), _d(b))
    if rc != 0:
        raise ValueError("oracle step_rk rejected its input")
    return x, v, rho


def step_rk_adjoint(p: Params, x, v, rho, xb, vb, rb, scheme="rk4"):
    """Cotangents of the state at the start of a Runge-Kutta step from those of its output."""
    s, A, b = _tableau(scheme)
    x, v, rho = _f64(x), _f64(v), _f64(rho)
    xb, vb, rb = _f64(xb).copy(), _f64(vb).copy(), _f64(rb).copy()
    pc = p.c()
    rc = lib().orc_step_rk_adjoint(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho), s, _d(A), _d(b),
                                   _d(xb), _d(vb), _d(rb))
    if rc != 0:
        raise ValueError("oracle step_rk_adjoint rejected its input")
    return xb, vb, rb


def step_symplectic(p: Params, x, v, rho, nsteps: int, reuse: bool = False, restart: int = 0):
    """nsteps steps of DualSPHysics' symplectic Euler; with reuse, the last substep's rates stand
    in for the next step's first substep, re-evaluated at every multiple of `restart` (0: only at
    the first step).  Returns (x, v, rho, evaluations of the update function)."""
    x, v, rho = _f64(x).copy(), _f64(v).copy(), _f64(rho).copy()
    ev = np.zeros(1, dtype=np.int64)
    pc = p.c()
    rc = lib().orc_step_symplectic(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho), nsteps,
                                   1 if reuse else 0, restart if restart > 0 else max(nsteps, 1),
                                   ev.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("oracle step_symplectic rejected its input")
    return x, v, rho, int(ev[0])


def step_symplectic_adjoint(p: Params, x, v, rho, xb, vb, rb):
    """Cotangents of the state at the start of a symplectic step (its first substep evaluated)
    from those of its output."""
    x, v, rho = _f64(x), _f64(v), _f64(rho)
    xb, vb, rb = _f64(xb).copy(), _f64(vb).copy(), _f64(rb).copy()
    pc = p.c()
    rc = lib().orc_step_symplectic_adjoint(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho),
                                           _d(xb), _d(vb), _d(rb))
    if rc != 0:
        raise ValueError("oracle step_symplectic_adjoint rejected its input")
    return xb, vb, rb


def rollout_symplectic_adjoint(p: Params, x, v, rho, nsteps: int, xb, vb, rb, reuse: bool = False,
                               restart: int = 0):
    """Cotangents of the initial state of a symplectic rollout from those of its final state."""
    x, v, rho = _f64(x), _f64(v), _f64(rho)
    xb, vb, rb = _f64(xb).copy(), _f64(vb).copy(), _f64(rb).copy()
    pc = p.c()
    rc = lib().orc_rollout_symplectic_adjoint(ctypes.byref(pc), rho.shape[0], _d(x), _d(v), _d(rho), nsteps,
                                              1 if reuse else 0, restart if restart > 0 else max(nsteps, 1),
                                              _d(xb), _d(vb), _d(rb))
    if rc != 0:
        raise ValueError("oracle rollout_symplectic_adjoint rejected its input")
    return xb, vb, rb


def shift(p: Params, x, rho, beta: float):
    """Particle shift dr = -beta H^2 sum_j [1 + 0.2 (W_ij / W(dx))^4] V_j grad_i W_ij (dim x n)."""
    x, rho = _f64(x), _f64(rho)
    n = rho.shape[0]
    dr = np.zeros((p.dim, n))
    pc = p.c()
    if lib().orc_shift(ctypes.byref(pc), n, _d(x), _d(rho), float(beta), _d(dr)) != 0:
        raise ValueError("oracle shift rejected its input")
    return dr


def shift_vjp(p: Params, x, rho, beta: float, xb):
    """(J_x^T xb, J_rho^T xb) of the shift, for cotangents xb of the shifted positions."""
    x, rho, xb = _f64(x), _f64(rho), _f64(xb)
    n = rho.shape[0]
    gx, gr = np.zeros((p.dim, n)), np.zeros(n)
    pc = p.c()
    if lib().orc_shift_vjp(ctypes.byref(pc), n, _d(x), _d(rho), float(beta), _d(xb), _d(gx), _d(gr)) != 0:
        raise ValueError("oracle shift_vjp rejected its input")
    return gx, gr


def renorm_gradient(p: Params, x, rho, A):
    """Renormalised gradient <grad A>_i = L_i sum_j V_j (A_j - A_i) grad_i W_ij (V_j = m / rho_j)."""
    x, rho, A = _f64(x), _f64(rho), _f64(A)
    n = rho.shape[0]
    G = np.zeros((p.dim, n))
    pc = p.c()
    rc = lib().orc_renorm_gradient(ctypes.byref(pc), n, _d(x), _d(rho), _d(A), _d(G))
    if rc != 0:
        raise ValueError("oracle renorm_gradient rejected its input")
    return G


def density_adjoint(p: Params, x, g):
    """Cotangent of the positions for cotangents g of the summation density:
    xbar_k = sum_{j != k} m (g_k + g_j) grad_k W_kj."""
    x, g = _f64(x), _f64(g)
    n = g.shape[0]
    xbar = np.zeros((p.dim, n))
    pc = p.c()
    rc = lib().orc_density_adjoint(ctypes.byref(pc), n, _d(x), _d(g), _d(xbar))
    if rc != 0:
        raise ValueError("oracle density_adjoint rejected its input")
    return xbar


def adjoint_sweep_sample(p: Params, x, v, rho, abar, rbar, sample):
    """Pair-sweep increments (x_bar, v_bar, rho_bar) of the listed particles."""
    x, v, rho, abar, rbar = _f64(x), _f64(v), _f64(rho), _f64(abar), _f64(rbar)
    n = rho.shape[0]
    s = np.ascontiguousarray(np.asarray(sample, dtype=np.int64))
    ns = s.shape[0]
    gx = np.zeros((p.dim, ns))
    gv = np.zeros((p.dim, ns))
    gr = np.zeros(ns)
    pc = p.c()
    rc = lib().orc_adjoint_sweep_sample(ctypes.byref(pc), n, _d(x), _d(v), _d(rho), _d(abar), _d(rbar), ns,
                                        s.ctypes.data_as(_I64), _d(gx), _d(gv), _d(gr))
    if rc != 0:
        raise ValueError("oracle adjoint_sweep_sample rejected its input")
    return gx, gv, gr


def rollout(p: Params, x0, v0, rho0, T: int, loss_kind: int):
    """Forward T steps then the full adjoint.  loss_kind 0: sum |v_T|^2, 1: 1/2 sum m |v_T|^2.

    Returns dict(x, v, rho, loss, gx0, gv0, grho0)."""
    x0, v0, rho0 = _f64(x0), _f64(v0), _f64(rho0)
    n = rho0.shape[0]
    xT, vT, rT = np.zeros_like(x0), np.zeros_like(v0), np.zeros_like(rho0)
    gx, gv, gr = np.zeros_like(x0), np.zeros_like(v0), np.zeros_like(rho0)
    loss = np.zeros(1)
    pc = p.c()
    rc = lib().orc_rollout(ctypes.byref(pc), n, _d(x0), _d(v0), _d(rho0), T, loss_kind, _d(xT), _d(vT), _d(rT),
                           _d(gx), _d(gv), _d(gr), _d(loss))
    if rc != 0:
        raise ValueError("oracle rollout rejected its input")
    return {"x": xT, "v": vT, "rho": rT, "loss": float(loss[0]), "gx0": gx, "gv0": gv, "grho0": gr}


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))
