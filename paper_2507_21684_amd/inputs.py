"""Seeded synthetic inputs: jittered periodic lattices with Taylor-Green velocity fields.

This module only draws initial states; it holds none of the method's arithmetic,
and it is the one piece of code that both the GPU path and the CPU oracle's tests
use (the oracle itself never imports it).

The paper's weakly compressible validation case is the periodic Taylor-Green
vortex (App. E, Taylor-Green subsection) and its scaling measurements use fully
occupied lattices with random noise on the positions (Sec. 4.1).  The workloads
here follow that recipe on the unit box: particles on a lattice of spacing dx
with uniform jitter of +-0.1 dx per coordinate, rest density 1, mass
rho0 dx^d, support H = 4 dx (Owen's neighbourhood size of App. A.1 gives
H ~ 4 dx in 2D) and velocity
    2D:  u =  A sin(2 pi x) cos(2 pi y),  v = -A cos(2 pi x) sin(2 pi y)
    3D:  u =  A sin(2 pi x) cos(2 pi y) cos(2 pi z),
         v = -A cos(2 pi x) sin(2 pi y) cos(2 pi z),  w = 0
evaluated at the jittered positions.  Everything is drawn in float64 with
numpy's PCG64 generator; float32 runs round the result once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np


@dataclass(frozen=True)
class SimSpec:
    """One periodic Taylor-Green simulation on the unit box."""
    dim: int
    side: int                 # particles per box side; N = side**dim
    amplitude: float = 1.0
    rho0: float = 1.0
    c0: float = 10.0
    delta: float = 0.1
    alpha: float = 0.01
    eps: float = 0.01
    support_factor: float = 4.0   # H = support_factor * dx
    cfl: float = 0.125            # dt = cfl * H / c0 = 0.25 h / c0 with smoothing length h = H / 2
    jitter: float = 0.1           # uniform jitter, fraction of dx
    box: float = 1.0

    @property
    def n(self) -> int:
        return self.side ** self.dim

    @property
    def dx(self) -> float:
        return self.box / self.side

    @property
    def H(self) -> float:
        return self.support_factor * self.dx

    @property
    def mass(self) -> float:
        return self.rho0 * self.dx ** self.dim

    @property
    def dt(self) -> float:
        return self.cfl * self.H / self.c0

    def params(self) -> dict:
        """Plain parameter dictionary understood by both the GPU binding and the oracle."""
        return dict(dim=self.dim, L=self.box, H=self.H, m=self.mass, rho0=self.rho0, c0=self.c0,
                    delta=self.delta, alpha=self.alpha, eps=self.eps, dt=self.dt)


def make_state(spec: SimSpec, seed: int):
    """Return (x[dim, N], v[dim, N], rho[N]) in float64 for one simulation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s, d, dx = spec.side, spec.dim, spec.dx
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64)] * d, indexing="ij")
    # particle index i = ((iz*s + iy)*s + ix): x varies fastest
    lat = np.stack([g.transpose(*reversed(range(d))).reshape(-1) for g in grids], axis=0)
    x = (lat + 0.5) * dx
    x = x + rng.uniform(-spec.jitter * dx, spec.jitter * dx, size=x.shape)
    tp = 2.0 * math.pi
    A = spec.amplitude
    v = np.zeros_like(x)
    if d == 2:
        v[0] = A * np.sin(tp * x[0]) * np.cos(tp * x[1])
        v[1] = -A * np.cos(tp * x[0]) * np.sin(tp * x[1])
    else:
        v[0] = A * np.sin(tp * x[0]) * np.cos(tp * x[1]) * np.cos(tp * x[2])
        v[1] = -A * np.cos(tp * x[0]) * np.sin(tp * x[1]) * np.cos(tp * x[2])
    rho = np.full(x.shape[1], spec.rho0, dtype=np.float64)
    return x, v, rho


@dataclass(frozen=True)
class Workload:
    """A named job: one or more simulations, a precision, a step count and a loss."""
    name: str
    sims: List[SimSpec]
    seeds: List[int]
    dtype: str            # "f32" or "f64"
    steps: int
    ckpt_every: int = 8
    adjoint: bool = True
    loss: str = "sum_v2"  # "sum_v2": sum |v_T|^2 ; "ke": 1/2 sum m |v_T|^2
    tape: int = 0         # plan tape depth (0: the checkpoint interval, so the backward recomputes)


def tgv2d_1k_f64() -> Workload:
    """2D, 32x32 = 1024 particles, FP64, 10 steps, forward only (seed 0)."""
    return Workload("tgv2d_1k_f64", [SimSpec(2, 32)], [0], "f64", 10, 10, False, "sum_v2")


def tgv2d_64k_f32() -> Workload:
    """2D, 256x256 = 65536 particles, FP32, 64 steps + adjoint of sum |v_T|^2, checkpoint every 8."""
    return Workload("tgv2d_64k_f32", [SimSpec(2, 256)], [0], "f32", 64, 8, True, "sum_v2")


def tgv3d_262k_f32() -> Workload:
    """3D, 64^3 = 262144 particles, FP32, 32 steps + adjoint of the kinetic energy; the plan keeps
    every step of the forward (32 tape slots), so the backward does not recompute."""
    return Workload("tgv3d_262k_f32", [SimSpec(3, 64)], [0], "f32", 32, 8, True, "ke", tape=32)


def batched_512_specs(seed: int = 1234, count: int = 512):
    """512 independent 2D simulations: N log-uniform in [256, 16384], side = clamp(round(sqrt N), 16, 128),
    amplitude uniform in [0.5, 2]; one derived seed per simulation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    logn = rng.uniform(math.log(256.0), math.log(16384.0), size=count)
    amp = rng.uniform(0.5, 2.0, size=count)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    sims, out_seeds = [], []
    for k in range(count):
        side = int(min(128, max(16, round(math.sqrt(math.exp(logn[k]))))))
        sims.append(SimSpec(2, side, amplitude=float(amp[k])))
        out_seeds.append(int(seeds[k]))
    return sims, out_seeds


def batched_512_f32() -> Workload:
    """The 512 simulations, 32 steps + adjoint of sum |v_T|^2; the plan keeps every step of the
    forward (32 tape slots), so the backward does not recompute."""
    sims, seeds = batched_512_specs()
    return Workload("batched_512_tgv2d_f32", sims, seeds, "f32", 32, 8, True, "sum_v2", tape=32)


@dataclass
class Request:
    """One solve-plus-gradient request of the serving workload."""
    rid: int
    arrival: float        # seconds after the start of the trace
    spec: SimSpec
    seed: int
    steps: int


def serving_trace(seed: int = 2026, count: int = 1000, rate: float = 50.0,
                  max_side_3d: int = 100, max_side_2d: int = 256) -> List[Request]:
    """Poisson arrivals at `rate` per second; 70 % 2D (N log-uniform in [1k, 64k]) and 30 % 3D
    (N log-uniform in [8k, 1M]); 16..128 steps; amplitude uniform in [0.5, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        is3d = rng.uniform() < 0.3
        if is3d:
            n = math.exp(rng.uniform(math.log(8e3), math.log(1e6)))
            side = int(min(max_side_3d, max(20, round(n ** (1.0 / 3.0)))))
            dim = 3
        else:
            n = math.exp(rng.uniform(math.log(1e3), math.log(64e3)))
            side = int(min(max_side_2d, max(32, round(math.sqrt(n)))))
            dim = 2
        steps = int(rng.integers(16, 129))
        amp = float(rng.uniform(0.5, 2.0))
        out.append(Request(k, t, SimSpec(dim, side, amplitude=amp), int(rng.integers(0, 2 ** 31 - 1)), steps))
    return out
