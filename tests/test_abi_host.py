"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol
include/sph.h declares, and plan creation validates its arguments."""
import ctypes
import os
import re

import pytest

from paper_2507_21684_amd import lib as L
from paper_2507_21684_amd.inputs import SimSpec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    declared = _declared()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(L.exported_symbols()) == declared


def _plan(params, counts, maxn=0, tape=0):
    arr = (L.SphParams * len(params))(*params)
    cnt = (ctypes.c_int64 * len(counts))(*counts)
    h = ctypes.c_void_p()
    rc = L.lib().sph_plan_create(arr, len(params), cnt, maxn, tape, ctypes.byref(h))
    return rc, h


def _p(spec, dtype="f32", **kw):
    d = spec.params()
    d.update(kw)
    return L.make_params(d, dtype)


def test_plan_create_and_sizes():
    spec = SimSpec(2, 256)
    rc, h = _plan([_p(spec)], [spec.n])
    assert rc == 0
    size = ctypes.c_size_t()
    assert L.lib().sph_workspace_size(h, ctypes.byref(size)) == 0
    tot, ns, mn = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    assert L.lib().sph_plan_info(h, ctypes.byref(tot), ctypes.byref(ns), ctypes.byref(mn)) == 0
    assert tot.value == 65536 and ns.value == 1
    # automatic width: 1.6 x (pi H^2 / dx^2) rounded up to 8
    assert mn.value == 88
    # two neighbour-list slots dominate: 2 x width x N x 4 bytes, plus O(N) arrays
    lists = 2 * mn.value * 65536 * 4
    assert lists < size.value < lists + 600 * 65536
    L.lib().sph_plan_destroy(h)
    # a tape of 8 steps holds 8 slots
    rc, h8 = _plan([_p(spec)], [spec.n], 0, 8)
    size8 = ctypes.c_size_t()
    L.lib().sph_workspace_size(h8, ctypes.byref(size8))
    assert 8 * mn.value * 65536 * 4 < size8.value < 8 * (mn.value * 65536 * 4 + 100 * 65536) + 300 * 65536
    lf, la = ctypes.c_int32(), ctypes.c_int32()
    assert L.lib().sph_get_tuning(h8, ctypes.byref(lf), ctypes.byref(la)) == 0
    assert (lf.value, la.value) == (4, 4)
    assert L.lib().sph_set_tuning(h8, 2, 8) == 0
    assert L.lib().sph_set_tuning(h8, 1, 4) == -1
    L.lib().sph_plan_destroy(h8)


@pytest.mark.parametrize("kw,code", [
    (dict(dim=4), -1),
    (dict(H=0.6), -1),          # 2H >= L
    (dict(m=-1.0), -1),
    (dict(eps=0.0), -1),
    (dict(H=0.4), -2),          # L/H < 3: fewer than 3 cells of side >= H
])
def test_plan_create_rejects(kw, code):
    spec = SimSpec(2, 16)
    d = spec.params()
    d.update(kw)
    p = L.make_params(d, "f32")
    rc, h = _plan([p], [spec.n])
    assert rc == code, L.lib().sph_last_error()
    assert L.lib().sph_last_error()


def test_plan_rejects_mixed_batches():
    a, b = SimSpec(2, 16), SimSpec(3, 16)
    rc, _ = _plan([_p(a), _p(b)], [a.n, b.n])
    assert rc == -1
    rc, _ = _plan([_p(a), _p(a, "f64")], [a.n, a.n])
    assert rc == -1
    rc, _ = _plan([_p(a)], [-5])
    assert rc == -1


def test_batched_plan():
    from paper_2507_21684_amd.inputs import batched_512_specs
    sims, _ = batched_512_specs()
    params = [_p(s) for s in sims]
    rc, h = _plan(params, [s.n for s in sims])
    assert rc == 0, L.lib().sph_last_error()
    tot = ctypes.c_int64()
    L.lib().sph_plan_info(h, ctypes.byref(tot), None, None)
    assert tot.value == sum(s.n for s in sims)
    L.lib().sph_plan_destroy(h)


def test_calls_need_bound_plan():
    spec = SimSpec(2, 16)
    rc, h = _plan([_p(spec)], [spec.n])
    st = L.SphState()
    assert L.lib().sph_build_cells(h, ctypes.byref(st), None) == -7
    assert L.lib().sph_rollout_backward(h, None, 4, 2, ctypes.byref(st), None) == -7
    words = (ctypes.c_int32 * 1)()
    assert L.lib().sph_poll_async(h, words, None, None) == -7
    L.lib().sph_plan_destroy(h)


def test_tape_depth_validation():
    spec = SimSpec(2, 16)
    rc, _ = _plan([_p(spec)], [spec.n], 0, -1)
    assert rc == -1


def test_integrator_settings_on_an_unbound_plan():
    """Tableau checks and the stage storage it reserves (host-only calls)."""
    import ctypes
    import numpy as np
    from paper_2507_21684_amd.inputs import SimSpec
    spec = SimSpec(2, 32)
    arr = (L.SphParams * 1)(L.make_params(spec.params(), "f32"))
    cnt = (ctypes.c_int64 * 1)(spec.n)
    h = L._VP()
    assert L.lib().sph_plan_create(arr, 1, cnt, 0, 4, ctypes.byref(h)) == 0
    size0 = ctypes.c_size_t()
    L.lib().sph_workspace_size(h, ctypes.byref(size0))
    dp = ctypes.POINTER(ctypes.c_double)

    def setp(A, b):
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        return L.lib().sph_set_integrator(h, len(b), A.ctypes.data_as(dp), b.ctypes.data_as(dp))

    A, b = L.TABLEAUS["rk4"]
    assert setp(A, b) == 0
    size1 = ctypes.c_size_t()
    L.lib().sph_workspace_size(h, ctypes.byref(size1))
    assert size1.value > size0.value
    assert setp([[0.0, 1.0], [0.0, 0.0]], [0.5, 0.5]) == -1     # not explicit
    assert setp([[0.5, 0.0], [0.5, 0.0]], [0.5, 0.5]) == -1     # diagonal entry
    assert setp(np.zeros((5, 5)), np.ones(5) / 5) == -1          # too many stages
    assert setp([[0.0]], [float("nan")]) == -1
    assert L.lib().sph_set_integrator(h, 0, None, None) == 0    # back to semi-implicit Euler
    L.lib().sph_plan_destroy(h)


def test_symplectic_setting_reserves_a_rate_tape():
    """sph_set_symplectic on an unbound plan: stage storage plus tape_depth rate blocks."""
    import ctypes
    from paper_2507_21684_amd.inputs import SimSpec
    spec = SimSpec(2, 32)
    arr = (L.SphParams * 1)(L.make_params(spec.params(), "f32"))
    cnt = (ctypes.c_int64 * 1)(spec.n)
    sizes = {}
    for name in ("euler", "rk", "symp", "symp_after_rk"):
        h = L._VP()
        assert L.lib().sph_plan_create(arr, 1, cnt, 0, 4, ctypes.byref(h)) == 0
        if name in ("rk", "symp_after_rk"):
            A, b = L.TABLEAUS["midpoint"]
            L._set_integrator(h, "midpoint")
        if name in ("symp", "symp_after_rk"):
            assert L.lib().sph_set_symplectic(h, 1) == 0
            assert L.lib().sph_set_symplectic(h, 0) == 0
        sz = ctypes.c_size_t()
        L.lib().sph_workspace_size(h, ctypes.byref(sz))
        sizes[name] = sz.value
        if name == "symp":
            # back to a tableau and to semi-implicit Euler; the reservation stays
            L._set_integrator(h, "rk4")
            L._set_integrator(h, None)
            L.lib().sph_workspace_size(h, ctypes.byref(sz))
            assert sz.value == sizes["symp"]
        L.lib().sph_plan_destroy(h)
    block = 4 * spec.n * 5               # FP32, 2D: x, v (2 each) and rho, aligned below
    assert sizes["rk"] > sizes["euler"]
    assert sizes["symp"] - sizes["rk"] >= 4 * block
    assert sizes["symp_after_rk"] == sizes["symp"]
    assert L.lib().sph_set_symplectic(None, 0) != 0


def test_diffusion_setting_reserves_records_in_any_order():
    """sph_set_diffusion and the integrator settings reserve disjoint regions whatever the order."""
    import ctypes
    from paper_2507_21684_amd.inputs import SimSpec
    spec = SimSpec(2, 32)
    arr = (L.SphParams * 1)(L.make_params(spec.params(), "f32"))
    cnt = (ctypes.c_int64 * 1)(spec.n)

    def size_after(steps):
        h = L._VP()
        assert L.lib().sph_plan_create(arr, 1, cnt, 0, 4, ctypes.byref(h)) == 0
        for st in steps:
            if st == "renorm":
                assert L.lib().sph_set_diffusion(h, 1) == 0
            elif st == "plain":
                assert L.lib().sph_set_diffusion(h, 0) == 0
            else:
                L._set_integrator(h, st)
        sz = ctypes.c_size_t()
        L.lib().sph_workspace_size(h, ctypes.byref(sz))
        L.lib().sph_plan_destroy(h)
        return sz.value

    base = size_after([])
    rn = size_after(["renorm"])
    assert rn - base >= 4 * 16 * spec.n                      # G, two L records and gbar per particle
    assert size_after(["plain"]) == base                     # the default reserves nothing
    assert size_after(["renorm", "plain", "renorm"]) == rn
    a = size_after(["renorm", "symplectic_euler_reuse"])
    b = size_after(["symplectic_euler_reuse", "renorm"])
    assert a == b == size_after(["symplectic_euler"]) + (rn - base)
    assert L.lib().sph_set_diffusion(None, 1) != 0


def test_scratch_binding_checks_before_any_device_call():
    """sph_bind_scratch rejects a null plan and a plan larger than the static workspace
    without touching a device; the binding's constant matches the header's."""
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    m = re.search(r"#define SPH_SCRATCH_BYTES \((\d+)ull << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == L.SCRATCH_BYTES
    assert L.lib().sph_bind_scratch(None, None) == -1
    spec = SimSpec(3, 32)
    rc, h = _plan([_p(spec)], [spec.n], 0, 8)
    assert rc == 0
    size = ctypes.c_size_t()
    L.lib().sph_workspace_size(h, ctypes.byref(size))
    assert size.value > L.SCRATCH_BYTES
    assert L.lib().sph_bind_scratch(h, None) == -3
    assert b"static workspace" in L.lib().sph_last_error()
    L.lib().sph_plan_destroy(h)


def test_skin_mode_setting_on_an_unbound_plan():
    """Speed-scaled half skins need a skin; uniform ones are always accepted (host-only calls)."""
    spec = SimSpec(2, 32)
    rc, h = _plan([_p(spec)], [spec.n])
    assert rc == 0
    assert L.lib().sph_set_skin_mode(h, 1) == -1
    assert L.lib().sph_set_skin_mode(h, 0) == 0
    L.lib().sph_plan_destroy(h)
    rc, h = _plan([L.make_params(spec.params(), "f32", 0.2)], [spec.n])
    assert rc == 0
    assert L.lib().sph_set_skin_mode(h, 1) == 0
    assert L.lib().sph_set_skin_mode(h, 0) == 0
    L.lib().sph_plan_destroy(h)
    assert L.lib().sph_set_skin_mode(None, 1) == -1
