"""Thin ctypes binding of libsph.so (the C ABI declared in include/sph.h).

Argument marshalling only: every step of the hot path runs in the HIP library.  If the
library has not been built, loading raises; there is no other implementation to fall
back to.  Tensors are torch tensors on the GPU (PyTorch provides device memory and the
stream); states are (x[dim, N], v[dim, N], rho[N]) in the plan's dtype, contiguous.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK = 0
SPH_F32 = 0
SPH_F64 = 1
FLAG_NONFINITE = 1
FLAG_NEIGHBOR_OVERFLOW = 2
FLAG_SKIN = 4
ERR_NAMES = {-1: "INVALID_ARG", -2: "TOO_FEW_CELLS", -3: "CAPACITY", -4: "NONFINITE", -5: "DEVICE",
             -6: "UNSUPPORTED", -7: "STATE"}


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERR_NAMES.get(code, "?"), code, msg))
        self.code = code


class SphParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("box", ctypes.c_double),
                ("support", ctypes.c_double), ("mass", ctypes.c_double), ("rho0", ctypes.c_double),
                ("c0", ctypes.c_double), ("delta", ctypes.c_double), ("alpha", ctypes.c_double),
                ("eps", ctypes.c_double), ("dt", ctypes.c_double), ("skin", ctypes.c_double)]


class SphState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p * 3), ("v", ctypes.c_void_p * 3), ("rho", ctypes.c_void_p)]


_lib = None
_VP = ctypes.c_void_p


def lib():
    """Open libsph.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsph.so is not built (python -m paper_2507_21684_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int32
        L.sph_plan_create.restype = st
        L.sph_plan_create.argtypes = [ctypes.POINTER(SphParams), ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_VP)]
        L.sph_set_tuning.restype = st
        L.sph_set_tuning.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32]
        L.sph_get_tuning.restype = st
        L.sph_density_adjoint.restype = st
        L.sph_density_adjoint.argtypes = [_VP, ctypes.POINTER(SphState), _VP, _VP, _VP]
        L.sph_set_graphs.argtypes = [_VP, ctypes.c_int32]
        L.sph_set_integrator.restype = st
        L.sph_set_integrator.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.sph_shift.restype = st
        L.sph_shift.argtypes = [_VP, ctypes.POINTER(SphState), ctypes.c_double, _VP]
        L.sph_shift_adjoint.restype = st
        L.sph_shift_adjoint.argtypes = [_VP, ctypes.POINTER(SphState), ctypes.POINTER(SphState), ctypes.c_double,
                                        _VP]
        L.sph_set_diffusion.restype = st
        L.sph_set_diffusion.argtypes = [_VP, ctypes.c_int32]
        L.sph_set_symplectic.restype = st
        L.sph_set_symplectic.argtypes = [_VP, ctypes.c_int32]
        L.sph_set_reuse.restype = st
        L.sph_set_reuse.argtypes = [_VP, ctypes.c_int32]
        L.sph_set_skin_mode.restype = st
        L.sph_set_skin_mode.argtypes = [_VP, ctypes.c_int32]
        L.sph_set_graphs.restype = ctypes.c_int32
        L.sph_get_tuning.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.sph_rollout_backward.restype = st
        L.sph_rollout_backward.argtypes = [_VP, ctypes.POINTER(SphState), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(SphState), _VP]
        L.sph_plan_destroy.restype = None
        L.sph_plan_destroy.argtypes = [_VP]
        L.sph_workspace_size.restype = st
        L.sph_workspace_size.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
        L.sph_plan_info.restype = st
        L.sph_plan_info.argtypes = [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
        L.sph_bind.restype = st
        L.sph_bind.argtypes = [_VP, _VP, ctypes.c_size_t, _VP]
        L.sph_bind_scratch.restype = st
        L.sph_bind_scratch.argtypes = [_VP, _VP]
        L.sph_build_cells.restype = st
        L.sph_build_cells.argtypes = [_VP, ctypes.POINTER(SphState), _VP]
        L.sph_neighbors.restype = st
        L.sph_neighbors.argtypes = [_VP, ctypes.POINTER(SphState), _VP, _VP, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int64), _VP]
        L.sph_neighbors_adaptive.restype = st
        L.sph_neighbors_adaptive.argtypes = [_VP, ctypes.POINTER(SphState), _VP, _VP, _VP, _VP, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64), _VP]
        L.sph_retained_lists.restype = st
        L.sph_retained_lists.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]
        L.sph_step_adjoint_retained.restype = st
        L.sph_step_adjoint_retained.argtypes = [_VP, ctypes.POINTER(SphState), ctypes.POINTER(SphState),
                                                ctypes.c_int32, ctypes.c_uint64, _VP]
        L.sph_density_adjoint_retained.restype = st
        L.sph_density_adjoint_retained.argtypes = [_VP, ctypes.POINTER(SphState), _VP, _VP, ctypes.c_int32,
                                                   ctypes.c_uint64, _VP]
        L.sph_rhs.restype = st
        L.sph_rhs.argtypes = [_VP, ctypes.POINTER(SphState), _VP, _VP, _VP, _VP]
        L.sph_step.restype = st
        L.sph_step.argtypes = [_VP, ctypes.POINTER(SphState), ctypes.c_int32, ctypes.POINTER(SphState),
                               ctypes.c_int32, _VP]
        L.sph_step_adjoint.restype = st
        L.sph_step_adjoint.argtypes = [_VP, ctypes.POINTER(SphState), ctypes.POINTER(SphState), _VP]
        L.sph_poll.restype = st
        L.sph_poll.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32), _VP]
        L.sph_pair_count.restype = st
        L.sph_pair_count.argtypes = [_VP, ctypes.POINTER(ctypes.c_int64), _VP]
        L.sph_poll_async.restype = st
        L.sph_poll_async.argtypes = [_VP, _VP, _VP, _VP]
        L.sph_profile_enable.restype = st
        L.sph_profile_enable.argtypes = [_VP, ctypes.c_int32]
        L.sph_profile_read.restype = st
        L.sph_profile_read.argtypes = [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.sph_last_error.restype = ctypes.c_char_p
        L.sph_last_error.argtypes = []
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SPH_OK:
        raise SphError(rc, lib().sph_last_error().decode())


def exported_symbols() -> List[str]:
    """Names the binding expects libsph.so to export."""
    return ["sph_plan_create", "sph_plan_destroy", "sph_workspace_size", "sph_plan_info", "sph_bind",
            "sph_build_cells", "sph_neighbors", "sph_rhs", "sph_step", "sph_step_adjoint", "sph_poll",
            "sph_pair_count", "sph_profile_enable", "sph_profile_read", "sph_last_error", "sph_set_tuning",
            "sph_get_tuning", "sph_rollout_backward", "sph_set_graphs", "sph_density_adjoint", "sph_set_reuse",
            "sph_set_skin_mode",
            "sph_set_integrator", "sph_set_symplectic", "sph_set_diffusion", "sph_shift",
            "sph_shift_adjoint", "sph_bind_scratch", "sph_neighbors_adaptive", "sph_retained_lists",
            "sph_step_adjoint_retained", "sph_density_adjoint_retained", "sph_poll_async"]


# Bytes of the library's static per-device workspace (SPH_SCRATCH_BYTES in sph.h).
SCRATCH_BYTES = 64 << 20


KERNEL_CLASSES = ["sort", "build", "sweep", "adjoint", "other"]

# Explicit Runge-Kutta tableaus (A strictly lower triangular, weights b); None is the default
# semi-implicit Euler step.  The symplectic schemes are not tableaus and are named separately.
SYMPLECTIC = {"symplectic_euler": 0, "symplectic_euler_reuse": 1}
TABLEAUS = {
    "semi_implicit_euler": None,
    "explicit_euler": ([[0.0]], [1.0]),
    "midpoint": ([[0.0, 0.0], [0.5, 0.0]], [0.0, 1.0]),
    "heun": ([[0.0, 0.0], [1.0, 0.0]], [0.5, 0.5]),
    "rk4": ([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]],
            [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
}


def _set_integrator(handle, integrator):
    """integrator: a TABLEAUS or SYMPLECTIC name, (A, b), or None."""
    if isinstance(integrator, str) and integrator in SYMPLECTIC:
        _check(lib().sph_set_symplectic(handle, SYMPLECTIC[integrator]))
        return
    if isinstance(integrator, str) and integrator not in TABLEAUS:
        raise ValueError("unknown integrator %r" % integrator)
    tab = None if integrator is None else (TABLEAUS[integrator] if isinstance(integrator, str) else integrator)
    if tab is None:
        _check(lib().sph_set_integrator(handle, 0, None, None))
        return
    A = np.ascontiguousarray(np.asarray(tab[0], dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(tab[1], dtype=np.float64))
    n = int(b.shape[0])
    _check(lib().sph_set_integrator(handle, n, A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def _skins(skin, n: int) -> List[float]:
    """One list skin per simulation from a scalar or a sequence."""
    if isinstance(skin, (int, float)):
        return [float(skin)] * n
    out = [float(x) for x in skin]
    if len(out) != n:
        raise ValueError("need one skin per simulation")
    return out


def workspace_bytes(sims: Sequence[dict], counts: Sequence[int], dtype: str = "f32", tape_depth: int = 8,
                    max_neighbors: int = 0, skin=0.0) -> int:
    """Workspace bytes a plan for this batch needs (host-only query; allocates no device memory)."""
    L = lib()
    n = len(sims)
    arr = (SphParams * n)(*[make_params(p, dtype, k) for p, k in zip(sims, _skins(skin, n))])
    cnt = (ctypes.c_int64 * n)(*[int(c) for c in counts])
    h = _VP()
    _check(L.sph_plan_create(arr, n, cnt, int(max_neighbors), int(tape_depth), ctypes.byref(h)))
    try:
        size = ctypes.c_size_t()
        _check(L.sph_workspace_size(h, ctypes.byref(size)))
        return int(size.value)
    finally:
        L.sph_plan_destroy(h)


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_params(p: dict, dtype: str, skin: float = 0.0) -> SphParams:
    """dict with keys dim, L, H, m, rho0, c0, delta, alpha, eps, dt -> SphParams (list skin as a
    fraction of the support)."""
    return SphParams(int(p["dim"]), SPH_F64 if dtype == "f64" else SPH_F32, float(p["L"]), float(p["H"]),
                     float(p["m"]), float(p["rho0"]), float(p["c0"]), float(p["delta"]), float(p["alpha"]),
                     float(p["eps"]), float(p["dt"]), float(skin))


class Plan:
    """A bound plan: host plan + device workspace for a batch of simulations."""

    def __init__(self, sims: Sequence[dict], counts: Sequence[int], dtype: str = "f32",
                 max_neighbors: int = 0, tape_depth: int = 8, device: Optional[torch.device] = None,
                 stream=None, skin=0.0, rebuild_every: int = 1, integrator=None, renormalised_diffusion: bool = False,
                 scratch: bool = False, speed_skins: bool = False):
        """scratch=True binds the library's static workspace of the current device
        (sph_bind_scratch) instead of allocating one; speed_skins=True gives the lists
        speed-scaled half skins (sph_set_skin_mode)."""
        L = lib()
        self.dtype = dtype
        self.torch_dtype = torch.float64 if dtype == "f64" else torch.float32
        self.dim = int(sims[0]["dim"])
        n = len(sims)
        skins = _skins(skin, n)
        arr = (SphParams * n)(*[make_params(p, dtype, k) for p, k in zip(sims, skins)])
        cnt = (ctypes.c_int64 * n)(*[int(c) for c in counts])
        h = _VP()
        _check(L.sph_plan_create(arr, n, cnt, int(max_neighbors), int(tape_depth), ctypes.byref(h)))
        try:
            if integrator is not None:
                _set_integrator(h, integrator)   # before the workspace is sized
            if renormalised_diffusion:
                _check(L.sph_set_diffusion(h, 1))
        except Exception:
            L.sph_plan_destroy(h)
            raise
        self.renormalised_diffusion = bool(renormalised_diffusion)
        self.integrator = integrator or "semi_implicit_euler"
        self.tape_depth = int(tape_depth)
        self.skins = skins
        self.skin = max(skins) if skins else 0.0
        self._h = h
        self.counts = [int(c) for c in counts]
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.nsims = n
        size = ctypes.c_size_t()
        _check(L.sph_workspace_size(h, ctypes.byref(size)))
        tot, ns, mn = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.sph_plan_info(h, ctypes.byref(tot), ctypes.byref(ns), ctypes.byref(mn)))
        self.N = int(tot.value)
        self.max_neighbors = int(mn.value)
        self.workspace_bytes = int(size.value)
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.scratch = bool(scratch)
        if self.scratch:
            self.workspace = None
            self._ws_ptr = None
            try:
                with torch.cuda.device(self.device):
                    _check(L.sph_bind_scratch(h, _stream_ptr(stream)))
            except Exception:
                L.sph_plan_destroy(h)
                self._h = None
                raise
        else:
            self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            _check(L.sph_bind(h, self._ws_ptr, self.workspace_bytes, _stream_ptr(stream)))
        self.rebuild_every = 1
        if rebuild_every != 1:
            self.set_reuse(rebuild_every)
        self.speed_skins = False
        if speed_skins:
            self.set_skin_mode(True)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sph_plan_destroy(h)
            self._h = None

    # -- marshalling
    def state(self, x: torch.Tensor, v: torch.Tensor, rho: torch.Tensor) -> SphState:
        d, N = self.dim, self.N
        for name, t, shape in (("x", x, (d, N)), ("v", v, (d, N)), ("rho", rho, (N,))):
            if tuple(t.shape) != shape:
                raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shape))
            if t.dtype != self.torch_dtype or not t.is_cuda or not t.is_contiguous():
                raise ValueError("%s must be a contiguous %s GPU tensor" % (name, self.torch_dtype))
        s = SphState()
        es = x.element_size()
        for k in range(3):
            s.x[k] = x.data_ptr() + k * N * es if k < d else None
            s.v[k] = v.data_ptr() + k * N * es if k < d else None
        s.rho = rho.data_ptr()
        return s

    def empty_state(self):
        d, N = self.dim, self.N
        return (torch.empty((d, N), dtype=self.torch_dtype, device=self.device),
                torch.empty((d, N), dtype=self.torch_dtype, device=self.device),
                torch.empty((N,), dtype=self.torch_dtype, device=self.device))

    # -- calls
    def build_cells(self, x, v, rho, stream=None):
        s = self.state(x, v, rho)
        _check(lib().sph_build_cells(self._h, ctypes.byref(s), _stream_ptr(stream)))

    def neighbors(self, x, v, rho, capacity: Optional[int] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
        """CSR (offsets int64[N+1], nbr int32[total]) over original indices, rows ascending, self included."""
        s = self.state(x, v, rho)
        off = torch.empty(self.N + 1, dtype=torch.int64, device=self.device)
        cap = capacity if capacity is not None else self.N * self.max_neighbors
        nbr = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        total = ctypes.c_int64()
        _check(lib().sph_neighbors(self._h, ctypes.byref(s), off.data_ptr(), nbr.data_ptr(), int(cap),
                                   ctypes.byref(total), _stream_ptr(stream)))
        return off, nbr[: total.value]

    def neighbors_adaptive(self, x, v, rho, support: torch.Tensor, capacity: Optional[int] = None,
                           stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
        """Lists with a support per particle (0 < h_i <= H): CSR (offsets int64[N+1], nbr int32[total])
        over original indices of the pairs with r_ij < max(h_i, h_j), rows ascending, self included,
        and the search radii s[N]."""
        s = self.state(x, v, rho)
        h = support.contiguous()
        if tuple(h.shape) != (self.N,) or h.dtype != self.torch_dtype or not h.is_cuda:
            raise ValueError("support must be a %s GPU tensor of shape (%d,)" % (self.torch_dtype, self.N))
        off = torch.empty(self.N + 1, dtype=torch.int64, device=self.device)
        cap = capacity if capacity is not None else self.N * self.max_neighbors
        nbr = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        sr = torch.empty(self.N, dtype=self.torch_dtype, device=self.device)
        total = ctypes.c_int64()
        _check(lib().sph_neighbors_adaptive(self._h, ctypes.byref(s), h.data_ptr(), sr.data_ptr(), off.data_ptr(),
                                            nbr.data_ptr(), int(cap), ctypes.byref(total), _stream_ptr(stream)))
        return off, nbr[: total.value], sr

    def rhs(self, x, v, rho, rho_sum: bool = True, stream=None):
        """(drho[N], a[dim, N], rho_sum[N] or None), original order."""
        s = self.state(x, v, rho)
        drho = torch.empty(self.N, dtype=self.torch_dtype, device=self.device)
        acc = torch.empty((self.dim, self.N), dtype=self.torch_dtype, device=self.device)
        rs = torch.empty(self.N, dtype=self.torch_dtype, device=self.device) if rho_sum else None
        _check(lib().sph_rhs(self._h, ctypes.byref(s), drho.data_ptr(), acc.data_ptr(),
                             rs.data_ptr() if rs is not None else None, _stream_ptr(stream)))
        return drho, acc, rs

    def step(self, x, v, rho, nsteps: int, ckpt: Optional[List[tuple]] = None, ckpt_every: int = 0, stream=None):
        """Advance (x, v, rho) in place.  ckpt: list of ceil(nsteps/ckpt_every) (x, v, rho) slots."""
        s = self.state(x, v, rho)
        cp = None
        if ckpt is not None:
            need = (nsteps + ckpt_every - 1) // ckpt_every if ckpt_every > 0 else 0
            if len(ckpt) < need:
                raise ValueError("need %d checkpoint slots" % need)
            cp = (SphState * max(need, 1))(*[self.state(*c) for c in ckpt[:need]])
        _check(lib().sph_step(self._h, ctypes.byref(s), int(nsteps), cp, int(ckpt_every), _stream_ptr(stream)))

    def shift(self, x, v, rho, beta: float, stream=None):
        """Particle shifting of (x, v, rho) in place (x only)."""
        s = self.state(x, v, rho)
        _check(lib().sph_shift(self._h, ctypes.byref(s), float(beta), _stream_ptr(stream)))

    def shift_adjoint(self, x, v, rho, gx, gv, grho, beta: float, stream=None):
        """Cotangents of the shifted state (gx, gv, grho) -> those of (x, v, rho), in place."""
        s = self.state(x, v, rho)
        c = self.state(gx, gv, grho)
        _check(lib().sph_shift_adjoint(self._h, ctypes.byref(s), ctypes.byref(c), float(beta), _stream_ptr(stream)))

    def step_adjoint(self, x, v, rho, gx, gv, grho, stream=None, retained=None):
        """Map the output cotangents (gx, gv, grho) of one step started at (x, v, rho) to its inputs, in place.
        retained: a (slot, generation) pair from retained_lists() taken after the one-step call that
        started at this state; its sort and lists are reused while still in the workspace."""
        s = self.state(x, v, rho)
        c = self.state(gx, gv, grho)
        if retained is None:
            _check(lib().sph_step_adjoint(self._h, ctypes.byref(s), ctypes.byref(c), _stream_ptr(stream)))
        else:
            _check(lib().sph_step_adjoint_retained(self._h, ctypes.byref(s), ctypes.byref(c), int(retained[0]),
                                                   int(retained[1]), _stream_ptr(stream)))

    def retained_lists(self) -> Tuple[int, int]:
        """(slot, generation) of the sort and lists that the last rhs or step call kept for its input state
        (slot -1 when gone)."""
        sl, gen = ctypes.c_int32(), ctypes.c_uint64()
        _check(lib().sph_retained_lists(self._h, ctypes.byref(sl), ctypes.byref(gen)))
        return int(sl.value), int(gen.value)

    def rollout_backward(self, ckpt: List[tuple], nsteps: int, ckpt_every: int, gx, gv, grho, stream=None):
        """Cotangents (gx, gv, grho) of the state after nsteps steps -> those of the initial state, in place,
        from the checkpoints sph_step wrote."""
        need = (nsteps + ckpt_every - 1) // ckpt_every if nsteps > 0 else 0
        if len(ckpt) < need:
            raise ValueError("need %d checkpoint slots" % need)
        cp = (SphState * max(need, 1))(*[self.state(*c) for c in ckpt[:need]])
        c = self.state(gx, gv, grho)
        _check(lib().sph_rollout_backward(self._h, cp, int(nsteps), int(ckpt_every), ctypes.byref(c),
                                          _stream_ptr(stream)))

    def density_adjoint(self, x, v, rho, rho_sum_bar, stream=None, retained=None) -> torch.Tensor:
        """Cotangent of the positions for cotangents rho_sum_bar[N] of the summation density.
        retained: a (slot, generation) pair from retained_lists() taken after the rhs call at this state."""
        s = self.state(x, v, rho)
        g = rho_sum_bar.contiguous()
        if tuple(g.shape) != (self.N,) or g.dtype != self.torch_dtype or not g.is_cuda:
            raise ValueError("rho_sum_bar must be a %s GPU tensor of shape (%d,)" % (self.torch_dtype, self.N))
        xbar = torch.empty((self.dim, self.N), dtype=self.torch_dtype, device=self.device)
        if retained is None:
            _check(lib().sph_density_adjoint(self._h, ctypes.byref(s), g.data_ptr(), xbar.data_ptr(),
                                             _stream_ptr(stream)))
        else:
            _check(lib().sph_density_adjoint_retained(self._h, ctypes.byref(s), g.data_ptr(), xbar.data_ptr(),
                                                      int(retained[0]), int(retained[1]), _stream_ptr(stream)))
        return xbar

    def bind_scratch(self, stream=None):
        """(Re)bind the plan to the library's static workspace of the current device."""
        _check(lib().sph_bind_scratch(self._h, _stream_ptr(stream)))
        self.scratch = True

    def set_tuning(self, lanes_fwd: int, lanes_adj: int):
        _check(lib().sph_set_tuning(self._h, int(lanes_fwd), int(lanes_adj)))

    def set_reuse(self, rebuild_every: int):
        """Rebuild the cell list and neighbour lists every `rebuild_every` steps (needs a skin)."""
        _check(lib().sph_set_reuse(self._h, int(rebuild_every)))
        self.rebuild_every = int(rebuild_every)

    def set_skin_mode(self, speed_scaled: bool):
        """Speed-scaled (True) or uniform (False) half skins for the lists (needs a skin)."""
        _check(lib().sph_set_skin_mode(self._h, 1 if speed_scaled else 0))
        self.speed_skins = bool(speed_scaled)

    def set_graphs(self, enable: bool = True):
        """Issue step / rollout_backward calls as cached executable HIP graphs."""
        _check(lib().sph_set_graphs(self._h, 1 if enable else 0))

    def get_tuning(self) -> Tuple[int, int]:
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sph_get_tuning(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def pair_count(self, stream=None) -> int:
        """Directed neighbour pairs (j != i, r < H) counted since the last call, then reset."""
        v = ctypes.c_int64()
        _check(lib().sph_pair_count(self._h, ctypes.byref(v), _stream_ptr(stream)))
        return int(v.value)

    def profile(self, enable: bool = True, classes: Optional[Sequence[str]] = None):
        """Time launches with HIP events: every kernel class, or only those named in `classes`."""
        mask = 0
        if enable:
            names = KERNEL_CLASSES if classes is None else classes
            for c in names:
                mask |= 1 << KERNEL_CLASSES.index(c)
        _check(lib().sph_profile_enable(self._h, mask))

    def profile_read(self) -> dict:
        """{class: (milliseconds, launches)} accumulated since the last read."""
        ms = (ctypes.c_double * len(KERNEL_CLASSES))()
        n = (ctypes.c_int64 * len(KERNEL_CLASSES))()
        _check(lib().sph_profile_read(self._h, ms, n))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def poll(self, stream=None) -> np.ndarray:
        out = (ctypes.c_int32 * self.nsims)()
        _check(lib().sph_poll(self._h, out, _stream_ptr(stream)))
        return np.frombuffer(out, dtype=np.int32).copy()

    def poll_async(self, status: torch.Tensor, pairs: Optional[torch.Tensor] = None, stream=None):
        """Enqueue the status words (into `status`, host int32[nsims]) and the pair count (into
        `pairs`, host int64[1], optional) without waiting; both are valid once the stream has
        passed this point.  Pass page-locked tensors (pin_memory=True)."""
        if status.device.type != "cpu" or status.dtype != torch.int32 or status.numel() < self.nsims \
                or not status.is_contiguous():
            raise ValueError("status must be a contiguous host int32 tensor of at least nsims entries")
        if pairs is not None and (pairs.device.type != "cpu" or pairs.dtype != torch.int64 or pairs.numel() < 1):
            raise ValueError("pairs must be a host int64 tensor")
        _check(lib().sph_poll_async(self._h, status.data_ptr(), pairs.data_ptr() if pairs is not None else None,
                                    _stream_ptr(stream)))
