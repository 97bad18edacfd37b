#!/usr/bin/env python3
"""Benchmark of the differentiable WCSPH hot path on one MI355X.

Metric: pair interactions per second, forward + adjoint.  A pair interaction is one
directed neighbour pair (i, j), j != i, in one right-hand-side evaluation of the forward
pass or in one adjoint step; recomputation during the backward pass is done but not
counted as work.  One benchmark "step" is one pass of the whole job: the forward rollout
with checkpoints, the loss seed and the checkpointed backward rollout.

Default workload (batched_512_tgv2d_f32, the largest single-GPU configuration): 512
independent 2D periodic Taylor-Green simulations in one plan, particle counts log-uniform in
[256, 16384] (1.96 M particles in all), amplitudes uniform in [0.5, 2], FP32, 32 steps of
dt = 0.125 H / c0 with a checkpoint every 8, loss sum |v_T|^2, gradient with respect to the
initial state.  Inputs are synthetic (seeded jittered lattices) and resident on the GPU
before the timed region.

The JSON line carries, for the headline workload: the roofline of its dominant pair kernel
(device time from HIP events that the library hands to that kernel's launches in the timed
region, which hold each launch's own start and end); the per-simulation completion latency
p50/p99 of the batched job against the plain path (one plan per simulation, run one after
the other); and the CPU oracle timed on a bounded sample on all host threads and on one.
Legs: the 3D 64^3 and 2D 256^2 fwd+adjoint jobs and the 2D 32^2 FP64 forward job, each
with its own roofline and oracle baseline; the backward benchmark, the renormalised
diffusion, particle shifting, the neighbour export, RK4 and symplectic jobs on the 2D 256^2
state; and the served workload (Poisson arrivals of uneven 2D/3D solve-plus-gradient
requests under continuous batching) against the plain first-come first-served path on the
same arrival trace.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s fwd+adjoint; batched p50/p99 latency vs plain path"

# Algorithmic FP work per directed pair (FMA = 2 flops; add, mul, division, sqrt, rint = 1),
# counted from the operations each sweep performs per pair.
FLOPS_PER_PAIR = {("sweep", 2): 54, ("sweep", 3): 64, ("adjoint", 2): 149, ("adjoint", 3): 178}
# Vector ALU ceilings of MI355X (published): FP32 157.3 TFLOP/s, which counts packed FP32 (two
# FP32 operations per lane per instruction), and FP64 78.6 TFLOP/s.  The library is built with
# packed FP32 instructions disabled, which caps its FP32 code at 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s; the JSON gives the fraction of that ceiling as well.
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
PEAK_TFLOPS_UNPACKED_F32 = 78.6
PEAK_HBM_GBS = 8000.0
STAGE_SKIN = 0.05      # list skin of the multistage legs (stage list reuse)


def workloads():
    from paper_2507_21684_amd import inputs as I
    return {"tgv2d_64k_f32": I.tgv2d_64k_f32, "tgv3d_262k_f32": I.tgv3d_262k_f32,
            "tgv2d_1k_f64": I.tgv2d_1k_f64, "batched_512_tgv2d_f32": I.batched_512_f32}


def packed_inputs(wl, dev):
    """Seeded initial state of every simulation of the workload, packed back to back."""
    import numpy as np
    import torch
    from paper_2507_21684_amd.inputs import make_state
    npdt = np.float32 if wl.dtype == "f32" else np.float64
    parts = [[a.astype(npdt) for a in make_state(s, sd)] for s, sd in zip(wl.sims, wl.seeds)]
    host = [np.concatenate([p[k] for p in parts], axis=-1) for k in range(3)]
    return host, [torch.tensor(a, device=dev).contiguous() for a in host]


_MASS_CACHE = {}


def plan_masses(plan, wl, like):
    """Per-particle mass row (for the kinetic-energy loss)."""
    import torch
    key = id(plan)
    if key not in _MASS_CACHE:
        _MASS_CACHE[key] = torch.cat([torch.full((c,), s.mass, dtype=like.dtype, device=like.device)
                                      for s, c in zip(wl.sims, plan.counts)])
    return _MASS_CACHE[key]


def run_job(plan, x0, v0, rho0, wl, adjoint=None):
    """One pass of the job: forward rollout with checkpoints, loss, checkpointed backward."""
    from paper_2507_21684_amd.rollout import rollout
    adjoint = wl.adjoint if adjoint is None else adjoint
    x = x0.clone()
    v = v0.clone().requires_grad_(adjoint)
    r = rho0.clone()
    # the device status is polled once after the timed jobs, not after every forward and backward
    xT, vT, rT = rollout(plan, x, v, r, wl.steps, wl.ckpt_every, check=False)
    if not adjoint:
        return None
    if wl.loss == "ke":
        loss = (0.5 * plan_masses(plan, wl, v0) * vT ** 2).sum()
    else:
        loss = (vT ** 2).sum()
    loss.backward()
    return v.grad


def count_pairs(plan, x0, v0, r0, wl):
    """Directed pairs (j != i) of every forward state n = 0..T-1, from a step-by-step forward pass."""
    import torch
    per_state = []
    xs, vs, rs = x0.clone(), v0.clone(), r0.clone()
    plan.pair_count()
    for _ in range(wl.steps):
        plan.step(xs, vs, rs, 1)
        per_state.append(plan.pair_count())
    torch.cuda.synchronize()
    return per_state


def count_pairs_schedule(plan, x0, v0, r0, wl):
    """Directed pairs (j != i) of the forward states n = 0..T-1 along the job's own trajectory:
    calls of one rebuild interval each keep the job's schedule of list builds."""
    import torch
    R = getattr(plan, "rebuild_every", 1)
    xs, vs, rs = x0.clone(), v0.clone(), r0.clone()
    plan.pair_count()
    done = 0
    while done < wl.steps:
        n = min(R, wl.steps - done)
        plan.step(xs, vs, rs, n)
        done += n
    torch.cuda.synchronize()
    return plan.pair_count()


def host_info():
    """Logical CPUs, the CPUs this process may run on, and the CPU model of the host."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def sample_pairs(dev, specs, parts, steps, dtype):
    """Directed pairs (j != i) of the states n = 0..steps-1 of the listed simulations, counted by
    the library's exact list builds (one plan of the sample, lists rebuilt every step)."""
    import numpy as np
    import torch
    from paper_2507_21684_amd.lib import Plan
    plan = Plan([s.params() for s in specs], [s.n for s in specs], dtype, tape_depth=0, device=dev)
    x, v, r = (torch.tensor(np.concatenate([p[k] for p in parts], axis=-1), device=dev) for k in range(3))
    plan.pair_count()
    total = 0
    for _ in range(steps):
        plan.step(x, v, r, 1)
        total += plan.pair_count()
    assert all(plan.poll() == 0)
    return total


def oracle_seconds(wl, parts, steps, threads=None):
    """Wall time of the oracle over the listed simulations: `steps` forward steps keeping every
    state and, for jobs with an adjoint, the adjoint steps back to the initial state (FP64)."""
    from oracle import oracle as O
    spec_parts = parts
    old = O.num_threads()
    if threads is not None:
        O.set_num_threads(threads)
    try:
        used = O.num_threads()
        t0 = time.perf_counter()
        for spec, (x, v, r) in spec_parts:
            p = O.Params(**spec.params())
            xd, vd, rd = (a.astype("float64") for a in (x, v, r))
            if wl.adjoint:
                O.rollout(p, xd, vd, rd, steps, 1 if wl.loss == "ke" else 0)
            else:
                O.step(p, xd, vd, rd, steps)
        return time.perf_counter() - t0, used
    finally:
        O.set_num_threads(old)


def cpu_baseline(dev, wl, parts_all, pick, steps, pick_1t=None, steps_1t=None):
    """The oracle as it stands on this host's cores over a bounded sample of the workload: the
    simulations `pick` for `steps` steps (forward and adjoint) with every OpenMP thread, and
    `pick_1t` for `steps_1t` steps with one thread (None: not run).  Rates are the sample's
    pair interactions (counted as in the GPU figure) over the oracle's wall time."""
    factor = 2 if wl.adjoint else 1
    sel = [(wl.sims[k], parts_all[k]) for k in pick]
    pairs = factor * sample_pairs(dev, [s for s, _ in sel], [p for _, p in sel], steps, wl.dtype)
    secs, threads = oracle_seconds(wl, sel, steps)
    what = "%d simulation%s, %d step%s%s" % (len(sel), "s" if len(sel) > 1 else "", steps, "s" if steps > 1 else "",
                                           " forward + adjoint" if wl.adjoint else " forward")
    out = {"value": round(pairs / secs, 1), "unit": "pair interactions/s", "cores": threads, "kind": "oracle",
           "sample": "%s, FP64, %d OpenMP threads, %.1f s, %d pair interactions" % (what, threads, secs, pairs),
           **host_info()}
    if pick_1t is not None:
        sel1 = [(wl.sims[k], parts_all[k]) for k in pick_1t]
        pairs1 = factor * sample_pairs(dev, [s for s, _ in sel1], [p for _, p in sel1], steps_1t, wl.dtype)
        secs1, _ = oracle_seconds(wl, sel1, steps_1t, threads=1)
        out["value_1thread"] = round(pairs1 / secs1, 1)
        out["sample_1thread"] = "%d simulation%s, %d step%s, 1 OpenMP thread, %.1f s, %d pair interactions" % (
            len(sel1), "s" if len(sel1) > 1 else "", steps_1t, "s" if steps_1t > 1 else "", secs1, pairs1)
    else:
        out["value_1thread"] = None
    return out


def timed_jobs(plan, x0, v0, r0, wl, reps, classes=None):
    """Wall time of `reps` jobs with library-side HIP-event timing of the kernel classes named
    (all when None); returns (seconds, profile)."""
    import torch
    plan.profile_read()
    plan.profile(True, classes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run_job(plan, x0, v0, r0, wl)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    return t1 - t0, plan.profile_read()


def source_hash():
    """sha256 prefix of the kernel sources, the key of the committed counter tables."""
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2507_21684_amd/csrc/sph_device.hpp", "paper_2507_21684_amd/csrc/sph_api.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel_symbol):
    """HBM bytes per dispatch of a kernel from the committed rocprofv3 counter summary, or None when
    the summary has no line for it or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_and_counters.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    h = source_hash()
    for ln in lines:
        f = ln.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == workload and f[2] == kernel_symbol and f[3] == h:
            return int(f[4])
    return None


def roofline(prof, dom, wl, per_state, reps, dim, n_particles, lanes=(4, 4), taped=False, speed_skins=False):
    """Roofline of the dominant kernel from its HIP-event launch times in the timed region.

    k_sweep / k_adj_sweep: ALU-bound; algorithmic flops per launch = flops per directed pair x
    pairs per launch.  k_build_list: bound by its HBM output; algorithmic bytes per launch =
    4 B per list entry (pairs plus the self entry) + 4 B per count + the 16 B record read per
    particle."""
    K = wl.ckpt_every
    # states whose forward sweep the backward recomputes (none when it runs on the forward's tape)
    recompute = [] if taped else [n for n in range(wl.steps) if wl.adjoint and (n + 1) % K != 0
                                  and n != wl.steps - 1]
    p_fwd = sum(per_state)
    ms_dom, n_dom = prof[dom]
    mean_launch_s = ms_dom / n_dom * 1e-3
    kernel = {"sweep": "k_sweep", "adjoint": "k_adj_sweep", "build": "k_build_list"}[dom]
    if dom == "build":
        # one build per rebuild interval, forward and again in the backward's recomputation
        # (with a list skin the lists hold more entries than the pairs counted here)
        R = lanes[2] if len(lanes) > 2 else 1
        states = [n for n in range(wl.steps) if n % R == 0] * (2 if wl.adjoint and not taped else 1)
        entries = sum(per_state[n] + n_particles for n in states) * reps
        launches = len(states) * reps
        bytes_per_launch = (4 * entries + launches * n_particles * (4 + (16 if wl.dtype == "f32" else 32))) / launches
        achieved = bytes_per_launch / mean_launch_s / 1e9
        peak = PEAK_HBM_GBS
        tdt = "float" if wl.dtype == "f32" else "double"
        # the build kernel's last template argument: built by groups of 2 x 2 cells (large 2D plans)
        sym = "sph::k_build_list<%s,%d,%s,%%s>" % (tdt, dim, "true" if speed_skins else "false")
        traffic = measured_traffic(wl.name, sym % "true")
        if traffic is None:
            traffic = measured_traffic(wl.name, sym % "false")
        return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": peak, "unit": "GB/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "mean_launch_us": round(mean_launch_s * 1e6, 2), "launches": n_dom,
                "algorithmic_bytes_per_launch": int(bytes_per_launch)}
    if dom == "sweep":
        pairs = (p_fwd + sum(per_state[n] for n in recompute)) * reps
    else:
        pairs = p_fwd * reps
    flops_per_launch = FLOPS_PER_PAIR[(dom, dim)] * pairs / n_dom
    achieved = flops_per_launch / mean_launch_s / 1e12
    peak = PEAK_TFLOPS[wl.dtype]
    tdt = "float" if wl.dtype == "f32" else "double"
    # the kernels of the plain delta-diffusion (the last template argument is the renormalised one)
    sym = ("sph::k_sweep<%s,%d,0,%d,false>" % (tdt, dim, lanes[0]) if dom == "sweep"
           else "sph::k_adj_sweep<%s,%d,%d,false>" % (tdt, dim, lanes[1]))
    traffic = measured_traffic(wl.name, sym)
    out = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": traffic, "mean_launch_us": round(mean_launch_s * 1e6, 2),
           "launches": n_dom, "pairs_per_launch": int(pairs / n_dom)}
    if wl.dtype == "f32":
        out["frac_of_unpacked_fp32_peak"] = round(achieved / PEAK_TFLOPS_UNPACKED_F32, 4)
    if traffic is not None:
        # the HBM view of the same launches: counted bytes over the live launch time
        gbs = traffic / mean_launch_s / 1e9
        out["hbm_gbs"] = round(gbs, 1)
        out["hbm_frac"] = round(gbs / PEAK_HBM_GBS, 4)
    return out


def plain_path(dev, wl, x0, v0, r0, skins, R):
    """The plain path of a batched workload: one plan per simulation (the batch's own list
    skins and rebuild interval, lanes tuned per plan), run one after the other.  Returns the
    wall time of all of them and each simulation's completion time (ms) from events after its
    job."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import autotune
    from paper_2507_21684_amd.inputs import Workload
    from paper_2507_21684_amd.lib import Plan
    offs = np.concatenate([[0], np.cumsum([s.n for s in wl.sims])])
    plains = []
    for k, s in enumerate(wl.sims):
        sub = Workload("one", [s], [wl.seeds[k]], wl.dtype, wl.steps, wl.ckpt_every, wl.adjoint, wl.loss)
        st = (x0[:, offs[k]:offs[k + 1]].contiguous(), v0[:, offs[k]:offs[k + 1]].contiguous(),
              r0[offs[k]:offs[k + 1]].contiguous())
        p = Plan([s.params()], [s.n], wl.dtype, tape_depth=max(wl.ckpt_every, wl.tape), device=dev, skin=skins[k],
                 rebuild_every=R, speed_skins=R > 1)
        autotune.tune(p, *st)
        run_job(p, *st, sub)
        plains.append((p, sub, st))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    evs = []
    t0 = time.perf_counter()
    ev0.record()
    for p, sub, st in plains:
        run_job(p, *st, sub)
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        evs.append(e)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for p, _, _ in plains:
        assert all(p.poll() == 0)
    return t_plain, np.array([ev0.elapsed_time(e) for e in evs])


def bench_density_backward(dev, reps=20):
    """The paper's backward benchmark (Sec. 4.1): one step of the 2D 256^2 FP32 state, the
    summation density of all particles after it, and the gradient of its sum with respect to
    the initial positions.  Reports the forward and backward device times and the backward
    share of the total (the paper measured 32 % at 64 Ki particles), with the backward reusing
    the sort and lists that the forward built (as the paper's backward reuses the forward's
    adjacency, and as the autograd path does) and with the backward rebuilding them."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import inputs as I
    from paper_2507_21684_amd.lib import Plan
    spec = I.SimSpec(2, 256)
    host = [a.astype(np.float32) for a in I.make_state(spec, 0)]
    x0, v0, r0 = (torch.tensor(a, device=dev) for a in host)
    plan = Plan([spec.params()], [spec.n], "f32", tape_depth=1, device=dev)
    ones = torch.ones(spec.n, dtype=torch.float32, device=dev)

    def fwd():
        x, v, r = x0.clone(), v0.clone(), r0.clone()
        plan.step(x, v, r, 1)
        k0 = plan.retained_lists()
        _, _, rs = plan.rhs(x, v, r, rho_sum=True)
        return x, v, r, rs, (k0, plan.retained_lists())

    def bwd(x1, v1, r1, kept):
        xb = plan.density_adjoint(x1, v1, r1, ones, retained=kept[1] if kept else None)
        vb, rb = torch.zeros_like(v0), torch.zeros_like(r0)
        plan.step_adjoint(x0, v0, r0, xb, vb, rb, retained=kept[0] if kept else None)
        return xb

    out = {"workload": "density_backward_tgv2d_64k_f32", "particles": spec.n, "paper_backward_share": 0.32}
    for name, reuse in (("retained", True), ("rebuilt", False)):
        for _ in range(3):
            x1, v1, r1, _, kept = fwd()
            bwd(x1, v1, r1, kept if reuse else None)
        torch.cuda.synchronize()
        t_f, t_b = [], []
        for _ in range(reps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            x1, v1, r1, _, kept = fwd()
            e1.record()
            bwd(x1, v1, r1, kept if reuse else None)
            e2.record()
            torch.cuda.synchronize()
            t_f.append(e0.elapsed_time(e1))
            t_b.append(e1.elapsed_time(e2))
        tf, tb = float(np.median(t_f)), float(np.median(t_b))
        out[name] = {"forward_ms": round(tf, 4), "backward_ms": round(tb, 4), "backward_share": round(tb / (tf + tb), 3)}
    plan.pair_count()
    fwd()
    pairs = plan.pair_count()          # two list builds: the step's state and the state after it
    r = out["retained"]
    out.update({"forward_ms": r["forward_ms"], "backward_ms": r["backward_ms"], "backward_share": r["backward_share"],
                "pair_interactions_per_s": round(2 * pairs / ((r["forward_ms"] + r["backward_ms"]) * 1e-3), 1),
                "note": "forward = one step + summation density (2 sorts and list builds); backward = density VJP "
                        "+ step VJP, on the forward's retained lists ('retained') or rebuilding both ('rebuilt'); "
                        "median of %d on events around each phase" % reps})
    return out


def bench_rk4(dev, reps=3):
    """Classic RK4 (four right-hand sides per step) on the 2D 256^2 FP32 state: 16 steps with a
    checkpoint every 8 and the checkpointed backward; pair interactions of every stage's RHS
    and VJP per second."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import inputs as I
    from paper_2507_21684_amd.lib import Plan
    from paper_2507_21684_amd.rollout import rollout
    spec = I.SimSpec(2, 256)
    T, K = 16, 8
    x0, v0, r0 = (torch.tensor(a.astype(np.float32), device=dev) for a in I.make_state(spec, 0))
    # a skin of 0.05 H lets later stages keep the first stage's lists (the largest stage
    # displacement here is about a quarter of what it allows)
    plan = Plan([spec.params()], [spec.n], "f32", tape_depth=K, device=dev, integrator="rk4", skin=STAGE_SKIN)

    def job():
        v = v0.clone().requires_grad_(True)
        xT, vT, rT = rollout(plan, x0.clone(), v, r0.clone(), T, K)
        (vT ** 2).sum().backward()

    job()
    torch.cuda.synchronize()
    plan.pair_count()
    xs, vs, rs = x0.clone(), v0.clone(), r0.clone()
    plan.step(xs, vs, rs, T)
    pairs = plan.pair_count()          # every stage's right-hand side of the forward pass
    t0 = time.perf_counter()
    for _ in range(reps):
        job()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    assert all(plan.poll() == 0)
    return {"workload": "rk4_tgv2d_64k_f32", "list_skin": STAGE_SKIN, "steps": T, "ckpt_every": K, "ms_per_job": round(t * 1e3, 3),
            "pair_interactions": 2 * pairs, "value": round(2 * pairs / t, 1), "unit": "pair interactions/s",
            "note": "4 right-hand sides per step forward and 4 stage VJPs per step backward are counted"}


def bench_symplectic(dev, reps=3):
    """Symplectic Euler on the 2D 256^2 FP32 state, 16 steps with a checkpoint every 8 and the
    checkpointed backward, without and with re-use of the last substep's rates (two evaluations
    of the update function per step, or one plus a fresh one at each checkpoint); pair
    interactions of every evaluation and of its VJP per second."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import inputs as I
    from paper_2507_21684_amd.lib import Plan
    from paper_2507_21684_amd.rollout import rollout
    spec = I.SimSpec(2, 256)
    T, K = 16, 8
    x0, v0, r0 = (torch.tensor(a.astype(np.float32), device=dev) for a in I.make_state(spec, 0))
    out = {"workload": "symplectic_tgv2d_64k_f32", "steps": T, "ckpt_every": K, "unit": "pair interactions/s"}
    for name in ("symplectic_euler", "symplectic_euler_reuse"):
        plan = Plan([spec.params()], [spec.n], "f32", tape_depth=K, device=dev, integrator=name, skin=STAGE_SKIN)

        def job():
            v = v0.clone().requires_grad_(True)
            xT, vT, rT = rollout(plan, x0.clone(), v, r0.clone(), T, K)
            (vT ** 2).sum().backward()

        job()
        torch.cuda.synchronize()
        plan.pair_count()
        xs, vs, rs = x0.clone(), v0.clone(), r0.clone()
        ck = [plan.empty_state() for _ in range(T // K)]
        plan.step(xs, vs, rs, T, ck, K)     # the job's evaluation schedule (fresh at checkpoints)
        pairs = plan.pair_count()
        t0 = time.perf_counter()
        for _ in range(reps):
            job()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        assert all(plan.poll() == 0)
        out[name] = {"ms_per_job": round(t * 1e3, 3), "pair_interactions": 2 * pairs,
                     "value": round(2 * pairs / t, 1)}
        del plan
    out["reuse_speedup"] = round(out["symplectic_euler"]["ms_per_job"] / out["symplectic_euler_reuse"]["ms_per_job"], 3)
    return out


def bench_renorm(dev, wl, x0, v0, r0, skin, R, lanes, ms_plain, pairs, reps=3):
    """The default job with the renormalised delta-diffusion (one extra list pass per right-hand
    side, two per adjoint step) on the same list settings and lanes as the plain job."""
    import torch
    from paper_2507_21684_amd.lib import Plan
    plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype, tape_depth=wl.ckpt_every,
                device=dev, skin=skin, rebuild_every=R, renormalised_diffusion=True, speed_skins=R > 1)
    plan.set_tuning(*lanes)
    run_job(plan, x0, v0, r0, wl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run_job(plan, x0, v0, r0, wl)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    assert all(plan.poll() == 0)
    return {"workload": wl.name + "_renormalised_diffusion", "ms_per_job": round(t * 1e3, 3),
            "value": round(pairs / t, 1), "unit": "pair interactions/s",
            "cost_vs_plain_diffusion": round(t * 1e3 / ms_plain, 3)}


def bench_shift(dev, wl, x0, v0, r0, lanes, pairs_per_state, reps=20, beta=0.02):
    """Particle shifting of the default initial state and its VJP, beside one plain step of the
    same state.  Each call sorts the state, builds its exact lists and runs the shift sweep (and
    the VJP its adjoint sweep); the step is a one-step call, which also sorts and builds.  Every
    call starts from a fresh copy of the initial state (copied outside the timed region); beta =
    0.02 is CFL 0.2 times the Mach number 0.1 of the Taylor-Green flow.  Median over `reps`
    calls, events on the stream the library launches on."""
    import numpy as np
    import torch
    from paper_2507_21684_amd.lib import Plan
    plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype, tape_depth=1, device=dev)
    plan.set_tuning(*lanes)

    def fresh():
        return (x0.clone(), v0.clone(), r0.clone(), torch.ones_like(x0), torch.ones_like(v0), torch.ones_like(r0))

    calls = {"shift": lambda a: plan.shift(a[0], a[1], a[2], beta),
             "shift_adjoint": lambda a: plan.shift_adjoint(a[0], a[1], a[2], a[3], a[4], a[5], beta),
             "step": lambda a: plan.step(a[0], a[1], a[2], 1)}
    out = {}
    for name, fn in calls.items():
        fn(fresh())
        times = []
        for _ in range(reps):
            args = fresh()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn(args)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        out[name] = float(np.median(times))
        status = plan.poll()
        assert all(status == 0), "%s: device status %s" % (name, status)
    return {"workload": wl.name + "_shift", "beta": beta, "shift_ms": round(out["shift"], 4),
            "shift_adjoint_ms": round(out["shift_adjoint"], 4), "step_ms": round(out["step"], 4),
            "pair_interactions_per_call": int(pairs_per_state),
            "shift_value": round(pairs_per_state / (out["shift"] * 1e-3), 1),
            "shift_adjoint_value": round(pairs_per_state / (out["shift_adjoint"] * 1e-3), 1),
            "unit": "pair interactions/s",
            "note": "each call sorts and builds exact lists of its state; step = one sph_step call of 1 step; "
                    "pairs per call = the job's mean pairs per state"}


def bench_export(dev, wl, x0, v0, r0, reps=20):
    """The neighbour export (sph_neighbors) of the default initial state: a sort, an exact list
    build and the CSR export over original indices (offsets int64[N+1], entries int32), one
    synchronous call (it returns the entry count to the host).  Median wall time over `reps`
    calls after a warm-up call; the bytes are the CSR written."""
    import numpy as np
    import torch
    from paper_2507_21684_amd.lib import Plan
    plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype, tape_depth=1, device=dev)
    off, nbr = plan.neighbors(x0, v0, r0)
    total = int(nbr.numel())
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.neighbors(x0, v0, r0)
        times.append(time.perf_counter() - t0)
    assert all(plan.poll() == 0)
    t = float(np.median(times))
    n = int(sum(s.n for s in wl.sims))
    nbytes = 8 * (n + 1) + 4 * total
    return {"workload": wl.name + "_neighbor_export", "entries": total, "pairs": total - n,
            "ms_per_call": round(t * 1e3, 4), "csr_bytes": nbytes, "csr_gbs": round(nbytes / t / 1e9, 1),
            "note": "one synchronous sph_neighbors call: sort, exact list build, CSR export; wall time"}


def bench_graphs(dev, name, skins, R, lanes, reps=5):
    """One workload's job with every library call issued directly and as cached executable HIP
    graphs (sph_set_graphs): fixed state, checkpoint and cotangent buffers, so the graphs are
    captured once; the same plan settings as the timed job.  Wall time per job, median of reps
    after a warm-up job."""
    import numpy as np
    import torch
    from paper_2507_21684_amd.lib import Plan
    wl = workloads()[name]()
    _, (x0, v0, r0) = packed_inputs(wl, dev)
    plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype,
                tape_depth=max(wl.ckpt_every, wl.tape), device=dev, skin=skins, rebuild_every=R, speed_skins=R > 1)
    plan.set_tuning(*lanes)
    T, K = wl.steps, wl.ckpt_every
    x, v, r = plan.empty_state()
    ck = [plan.empty_state() for _ in range((T + K - 1) // K)]
    gx, gv, gr = torch.empty_like(x), torch.empty_like(v), torch.empty_like(r)
    masses = plan_masses(plan, wl, v0) if wl.loss == "ke" else None

    def job():
        x.copy_(x0)
        v.copy_(v0)
        r.copy_(r0)
        plan.step(x, v, r, T, ck, K)
        gx.zero_()
        gv.copy_(masses * v if masses is not None else 2.0 * v)
        gr.zero_()
        plan.rollout_backward(ck, T, K, gx, gv, gr)

    out = {"workload": name}
    for mode in ("direct", "graphs"):
        plan.set_graphs(mode == "graphs")
        job()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            job()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        out[mode + "_ms"] = round(float(np.median(times)) * 1e3, 3)
        assert all(plan.poll() == 0)
    plan.set_graphs(False)
    out["speedup"] = round(out["direct_ms"] / out["graphs_ms"], 3)
    out["note"] = "wall time per job, median of %d; the direct and graph paths give bitwise the same results" % reps
    return out


def log(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def bench_serving(dev, count, warmup, load=0.75, budget_gib=96):
    """Poisson arrivals of uneven 2D/3D solve-plus-gradient requests: continuous batching vs plain FIFO.

    The request mix is fixed by the trace seed; the arrival rate is `load` times the plain path's
    saturation throughput (1 / mean plain service time, measured on the same requests), so the
    same trace is offered to both servers.  Latency percentiles skip the first `warmup` requests.
    Below saturation both servers keep up with the arrivals, so their throughputs are equal; the
    saturation leg queues the same requests at once and compares the time to serve them all."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import serving as S
    from paper_2507_21684_amd.inputs import Request, serving_trace
    base = serving_trace(seed=2026, count=count, rate=1.0)
    # warm the allocator, the kernels and the plan tables on a few requests of each dimension
    for r in [r for r in base if r.spec.dim == 2][:2] + [r for r in base if r.spec.dim == 3][:1]:
        S.plain_request(Request(r.rid, 0.0, r.spec, r.seed, 16), "f32", 8, dev)
    service = []
    t_last = time.perf_counter()
    for k, r in enumerate(base):
        service.append(S.plain_request(r, "f32", 8, dev)[0])
        if time.perf_counter() - t_last > 10:
            t_last = time.perf_counter()
            log("serving, plain path: %d of %d requests, %.1f s of service" % (k + 1, count, sum(service)))
    service = np.array(service)
    log("serving, plain path done: mean service %.1f ms" % (service.mean() * 1e3))
    # where the plain path's time goes: requests by dimension and by size; batching can only
    # remove the per-launch cost of the requests too small to fill the GPU alone
    dims = np.array([r.spec.dim for r in base])
    sizes = np.array([r.spec.n for r in base])
    split = {"2d_s": round(float(service[dims == 2].sum()), 3), "3d_s": round(float(service[dims == 3].sum()), 3),
             "ge_256k_particles_s": round(float(service[sizes >= 1 << 18].sum()), 3),
             "requests_ge_256k_particles": int((sizes >= 1 << 18).sum())}
    rate = load / service.mean()
    trace = [Request(r.rid, r.arrival / rate, r.spec, r.seed, r.steps) for r in base]
    arrivals = np.array([r.arrival for r in trace])
    lat_plain = S.fifo_latencies(arrivals, service)
    makespan_plain = float(np.max(arrivals + lat_plain) - arrivals[0])
    torch.cuda.empty_cache()
    sch, eng, done = S.serve(trace, "f32", 8, int(budget_gib * (1 << 30)), dev, progress=log)
    log("serving, batched path done: %d ticks, %.1f s creating plans" % (sch.ticks, eng.plan_seconds))
    lat_served = np.array([j.finished - j.req.arrival for j in sorted(done, key=lambda j: j.req.rid)])
    makespan_served = float(max(j.finished for j in done) - arrivals[0])
    work = 2 * eng.pairs
    keep = slice(warmup, None)
    pp, ps = S.percentiles(lat_plain[keep]), S.percentiles(lat_served[keep])
    # saturation: the same requests all queued at t = 0, so that throughput is set by the server
    # and not by the arrivals (the plain path then takes the sum of its service times)
    served_info = {"peak_admitted_gib": round(sch.peak_used / (1 << 30), 2),
                   "failed_requests": int(sum(1 for j in done if j.error)),
                   "mean_batch": round(float(np.mean(sch.batch_sizes)), 2), "ticks": sch.ticks,
                   "plan_creation_s": round(eng.plan_seconds, 3)}
    del sch, eng, done
    torch.cuda.empty_cache()
    burst = [Request(r.rid, 0.0, r.spec, r.seed, r.steps) for r in base]
    sch_b, eng_b, done_b = S.serve(burst, "f32", 8, int(budget_gib * (1 << 30)), dev, progress=log)
    makespan_burst = float(max(j.finished for j in done_b))
    work_b = 2 * eng_b.pairs
    log("serving, saturation: %.2f s served vs %.2f s plain" % (makespan_burst, float(service.sum())))
    saturation = {"served": round(work_b / makespan_burst, 1), "plain": round(work_b / float(service.sum()), 1),
                  "speedup": round(float(service.sum()) / makespan_burst, 3),
                  "makespan_s": round(makespan_burst, 3), "mean_batch": round(float(np.mean(sch_b.batch_sizes)), 2),
                  "peak_admitted_gib": round(sch_b.peak_used / (1 << 30), 2),
                  "failed_requests": int(sum(1 for j in done_b if j.error))}
    return {"workload": "poisson_%d_mixed_2d3d_f32" % count, "requests": count, "warmup_requests": warmup,
            "rate_per_s": round(rate, 3), "load_vs_plain_saturation": load,
            "mean_plain_service_ms": round(float(service.mean() * 1e3), 3), "plain_service_split": split,
            "pair_interactions": work,
            "hbm_budget_gib": budget_gib, **served_info,
            "served": {"value": round(work / makespan_served, 1), "p50_ms": round(ps["p50_ms"], 3),
                       "p99_ms": round(ps["p99_ms"], 3), "makespan_s": round(makespan_served, 3)},
            "plain": {"value": round(work / makespan_plain, 1), "p50_ms": round(pp["p50_ms"], 3),
                      "p99_ms": round(pp["p99_ms"], 3), "makespan_s": round(makespan_plain, 3)},
            "saturation": saturation,
            "unit": "pair interactions/s"}


def measure_workload(name, dev, reps, warmup):
    """One workload end to end: its tuned plan (lanes, list skin, rebuild interval), `warmup`
    untimed jobs, exact pair counts of its trajectory, an untimed pass with every kernel class
    timed (breakdown and dominant kernel), then `reps` timed jobs in which only the dominant
    kernel's launches carry HIP events, and that kernel's roofline."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import autotune
    from paper_2507_21684_amd.lib import Plan
    wl = workloads()[name]()
    host, (x0, v0, r0) = packed_inputs(wl, dev)
    if wl.adjoint:
        plan = autotune.tune_plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype,
                                  wl.ckpt_every, x0, v0, r0, dev, tape_depth=wl.tape or None)
    else:
        plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype, tape_depth=0, device=dev)
    lanes = plan.get_tuning()
    R = plan.rebuild_every
    for _ in range(warmup):
        run_job(plan, x0, v0, r0, wl)
    torch.cuda.synchronize()
    per_state = count_pairs(plan, x0, v0, r0, wl)
    K = wl.ckpt_every
    # pairs of the timed trajectory itself: calls of one rebuild interval each follow the job's
    # build schedule; single steps give the per-state split (equal to within a few pairs)
    p_fwd = count_pairs_schedule(plan, x0, v0, r0, wl)
    scale = p_fwd / max(sum(per_state), 1)
    per_state = [c * scale for c in per_state]
    p_adj = p_fwd if wl.adjoint else 0          # adjoint step n runs on forward state n
    taped = wl.adjoint and plan.tape_depth >= wl.steps
    recompute_swept = [] if taped else [n for n in range(wl.steps) if wl.adjoint and (n + 1) % K != 0
                                        and n != wl.steps - 1]
    p_rec = int(round(sum(per_state[n] for n in recompute_swept)))
    plan.poll()
    n_part = int(sum(s.n for s in wl.sims))
    log("workload %s: %d simulation(s), %d particles, pairs per job %d" % (wl.name, len(wl.sims), n_part,
                                                                            p_fwd + p_adj))
    _, prof_all = timed_jobs(plan, x0, v0, r0, wl, 1)
    breakdown = {k: round(v[0], 3) for k, v in prof_all.items()}
    dom = max(("build", "sweep", "adjoint") if wl.adjoint else ("build", "sweep"), key=lambda k: prof_all[k][0])
    elapsed, prof = timed_jobs(plan, x0, v0, r0, wl, reps, [dom])
    status = plan.poll()
    assert np.all(status == 0), "device reported non-finite values or neighbour overflow: %s" % status
    dim = wl.sims[0].dim
    roof = roofline(prof, dom, wl, per_state, reps, dim, n_part, tuple(lanes) + (R,), taped, plan.speed_skins)
    ms = 1e3 * elapsed / reps
    log("%s: timed %d jobs, %.3f ms per job" % (wl.name, reps, ms))
    config = {"workload": wl.name, "dim": dim, "simulations": len(wl.sims), "particles": n_part,
              "sim_steps": wl.steps, "ckpt_every": wl.ckpt_every, "adjoint": wl.adjoint, "loss": wl.loss,
              "pairs_fwd": p_fwd, "pairs_adj": p_adj, "pairs_recompute": p_rec,
              "lanes_per_particle": list(lanes), "list_rebuild_every": R, "tape_depth": plan.tape_depth,
              "backward": "on the forward's tape" if plan.tape_depth >= wl.steps else
                          "recomputes each checkpoint segment"}
    if len(wl.sims) > 1:
        config["list_skin_range"] = [round(min(plan.skins), 4), round(max(plan.skins), 4)]
    else:
        config["list_skin"] = round(plan.skin, 4)
    config["half_skins"] = "speed-scaled" if plan.speed_skins else "uniform"
    res = {"workload": wl.name, "value": round((p_fwd + p_adj) * reps / elapsed, 1), "unit": "pair interactions/s",
           "ms_per_job": round(ms, 3), "timed_jobs": reps, "dtype": wl.dtype, "config": config, "roofline": roof,
           "kernel_ms_per_job": breakdown}
    return res, wl, plan, host, (x0, v0, r0)


def unpack(wl, host):
    """Per-simulation (x, v, rho) host arrays of a packed workload state."""
    import numpy as np
    offs = np.concatenate([[0], np.cumsum([s.n for s in wl.sims])])
    return [tuple(np.ascontiguousarray(a[..., offs[k]:offs[k + 1]]) for a in host) for k in range(len(wl.sims))]


# Bounded oracle samples per workload: (simulations, steps) with every thread, and with one
# thread; about 10-30 s of host time in all.
def cpu_samples(wl):
    n = len(wl.sims)
    if n > 1:
        pick = [int((k + 0.5) * n / 20) for k in range(20)]       # 20 simulations spread over the batch
        return pick, wl.steps, pick, wl.steps
    if wl.name == "tgv3d_262k_f32":
        return [0], 2, None, None                                  # two steps of the full box
    if wl.name == "tgv2d_64k_f32":
        return [0], wl.steps, [0], 8
    return [0], wl.steps, [0], wl.steps


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed passes of the whole job")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched_512_tgv2d_f32", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="only the headline workload and its plain path")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain path of a batched workload (kernel traces of the batch alone)")
    ap.add_argument("--serving", type=int, default=1000, help="requests of the served workload (0 skips it)")
    ap.add_argument("--serving-warmup", type=int, default=50, help="requests left out of the latency percentiles")
    ap.add_argument("--counter-pass", action="store_true",
                    help="for hardware-counter runs: warm-up and one job of the workload, then a plain "
                         "device copy of 256 MiB (the calibration kernel for byte counters); prints nothing")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; runs on more than one GPU are not supported "
              "(independent simulations would be assigned whole to GPUs, with no exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_21684_amd import autotune
    from paper_2507_21684_amd.lib import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.counter_pass:
        wl = workloads()[args.workload]()
        host, (x0, v0, r0) = packed_inputs(wl, dev)
        if wl.adjoint:
            plan = autotune.tune_plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype,
                                      wl.ckpt_every, x0, v0, r0, dev, tape_depth=wl.tape or None)
        else:
            plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype, tape_depth=0, device=dev)
        for _ in range(args.warmup + 1):
            run_job(plan, x0, v0, r0, wl)
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        return

    head, wl, plan, host, (x0, v0, r0) = measure_workload(args.workload, dev, args.steps, args.warmup)
    parts = unpack(wl, host)
    skins, R = list(plan.skins), plan.rebuild_every
    del plan
    torch.cuda.empty_cache()

    latency = None
    if len(wl.sims) > 1 and not args.no_plain:
        log("plain path: one plan per simulation, run in turn")
        t_plain, lat_plain = plain_path(dev, wl, x0, v0, r0, skins, R)
        work = head["config"]["pairs_fwd"] + head["config"]["pairs_adj"]
        t_b = head["ms_per_job"]
        latency = {"batched": {"p50_ms": t_b, "p99_ms": t_b,
                               "note": "every simulation of the batch completes with the batch's job"},
                   "plain": {"value": round(work / t_plain, 1), "ms_per_job": round(t_plain * 1e3, 3),
                             "p50_ms": round(float(np.percentile(lat_plain, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat_plain, 99)), 3)},
                   "speedup": round(t_plain * 1e3 / t_b, 2)}
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline of %s" % wl.name)
        cpu = cpu_baseline(dev, wl, parts, *cpu_samples(wl))

    legs = {}
    if not args.no_legs:
        for name in ("tgv3d_262k_f32", "tgv2d_64k_f32", "tgv2d_1k_f64"):
            if name == args.workload:
                continue
            res, lwl, lplan, lhost, _ = measure_workload(name, dev, max(1, min(args.steps, 10)), args.warmup)
            del lplan
            torch.cuda.empty_cache()
            if not args.no_cpu_baseline:
                log("CPU oracle baseline of %s" % name)
                res["cpu_baseline"] = cpu_baseline(dev, lwl, unpack(lwl, lhost), *cpu_samples(lwl))
            legs[name] = res

    extra = {}
    if not args.no_legs:
        from paper_2507_21684_amd.inputs import tgv2d_64k_f32
        w2 = tgv2d_64k_f32()
        h2, (a0, b0, c0) = packed_inputs(w2, dev)
        c2 = legs.get("tgv2d_64k_f32", head if wl.name == w2.name else None)
        lanes2 = tuple(c2["config"]["lanes_per_particle"]) if c2 else (4, 4)
        skin2 = c2["config"].get("list_skin", 0.26) if c2 else 0.26
        R2 = c2["config"]["list_rebuild_every"] if c2 else 8
        pairs2 = c2["config"]["pairs_fwd"] if c2 else None
        log("density backward benchmark")
        extra["density_backward"] = bench_density_backward(dev)
        if c2:
            log("renormalised diffusion job")
            extra["renormalised_diffusion"] = bench_renorm(dev, w2, a0, b0, c0, skin2, R2, lanes2, c2["ms_per_job"],
                                                           2 * pairs2)
            log("particle shifting")
            extra["shift"] = bench_shift(dev, w2, a0, b0, c0, lanes2, pairs2 / w2.steps)
        log("neighbour export")
        extra["neighbor_export"] = bench_export(dev, w2, a0, b0, c0)
        log("RK4 job")
        extra["rk4"] = bench_rk4(dev)
        log("symplectic Euler jobs")
        extra["symplectic"] = bench_symplectic(dev)
        log("graph mode")
        graphs = [bench_graphs(dev, wl.name, skins, R, tuple(head["config"]["lanes_per_particle"]))]
        if c2 and wl.name != w2.name:
            graphs.append(bench_graphs(dev, w2.name, skin2, R2, lanes2))
        extra["graph_mode"] = graphs

    served = None
    if args.serving > 0:
        torch.cuda.empty_cache()
        log("served workload")
        served = bench_serving(dev, args.serving, min(args.serving_warmup, args.serving // 2))

    out = {"metric": METRIC, "value": head["value"], "unit": "pair interactions/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_job"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl.dtype,
           "data": "synthetic", "config": head["config"], "latency": latency,
           "roofline": head["roofline"], "kernel_ms_per_job": head["kernel_ms_per_job"], "cpu_baseline": cpu,
           "legs": legs, "serving": served, **extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
