#!/usr/bin/env python3
"""Benchmark of the differentiable WCSPH hot path on one MI355X.

Metric: pair interactions per second, forward + adjoint.  A pair interaction is one
directed neighbour pair (i, j), j != i, in one right-hand-side evaluation of the forward
pass or in one adjoint step; recomputation during the backward pass is done but not
counted as work.  One benchmark "step" is one pass of the whole job: the forward rollout
with checkpoints, the loss seed and the checkpointed backward rollout.

Default workload (tgv2d_64k_f32): 2D periodic Taylor-Green, 256^2 = 65536 particles,
FP32, 64 steps of dt = 0.25 H / c0, checkpoint every 8, loss sum |v_T|^2, gradient with
respect to the initial state.  Inputs are synthetic (seeded jittered lattice).

The JSON line also carries the roofline of the dominant pair kernel (device time from HIP
events the library records on its launch stream during the timed region), the CPU oracle
on the host's cores, and the batched workload (512 uneven 2D simulations in one plan)
against the plain path (one plan per simulation, run one after the other), with the
per-simulation completion latency p50/p99 of both.
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
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


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
    xT, vT, rT = rollout(plan, x, v, r, wl.steps, wl.ckpt_every)
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


def cpu_baseline(wl, host):
    """The oracle as it stands, on this host's cores, over the same job."""
    from oracle import oracle as O
    spec = wl.sims[0]
    p = O.Params(**spec.params())
    threads = O.num_threads()
    xd, vd, rd = [a.astype("float64") for a in host]
    t0 = time.perf_counter()
    O.rollout(p, xd, vd, rd, wl.steps, 1 if wl.loss == "ke" else 0)
    return time.perf_counter() - t0, threads


def timed_jobs(plan, x0, v0, r0, wl, reps):
    """Wall time of `reps` jobs with library-side kernel timing; returns (seconds, profile)."""
    import torch
    plan.profile_read()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run_job(plan, x0, v0, r0, wl)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    return t1 - t0, plan.profile_read()


def roofline(prof, wl, per_state, reps, dim):
    """Roofline of the dominant pair kernel: algorithmic flops per launch / mean launch time."""
    K = wl.ckpt_every
    recompute_swept = [n for n in range(wl.steps) if wl.adjoint and (n + 1) % K != 0 and n != wl.steps - 1]
    p_fwd = sum(per_state)
    cand = ("sweep", "adjoint") if wl.adjoint else ("sweep",)
    dom = max(cand, key=lambda k: prof[k][0])
    ms_dom, n_dom = prof[dom]
    if dom == "sweep":
        pairs = (p_fwd + sum(per_state[n] for n in recompute_swept)) * reps
    else:
        pairs = p_fwd * reps
    flops_per_launch = FLOPS_PER_PAIR[(dom, dim)] * pairs / n_dom
    mean_launch_s = ms_dom / n_dom * 1e-3
    achieved = flops_per_launch / mean_launch_s / 1e12
    peak = PEAK_TFLOPS[wl.dtype]
    return {"bound": "alu", "kernel": {"sweep": "k_sweep", "adjoint": "k_adj_sweep"}[dom],
            "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": None, "mean_launch_us": round(mean_launch_s * 1e6, 2),
            "pairs_per_launch": int(pairs / n_dom)}


def bench_batched(dev, reps):
    """512 uneven 2D simulations: one batched plan vs one plan per simulation run in turn."""
    import numpy as np
    import torch
    from paper_2507_21684_amd import autotune
    from paper_2507_21684_amd.inputs import batched_512_f32, Workload
    from paper_2507_21684_amd.lib import Plan
    wl = batched_512_f32()
    host, (x0, v0, r0) = packed_inputs(wl, dev)
    plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype, tape_depth=wl.ckpt_every,
                device=dev)
    autotune.tune(plan, x0, v0, r0)
    run_job(plan, x0, v0, r0, wl)
    per_state = count_pairs(plan, x0, v0, r0, wl)
    work = 2 * sum(per_state)
    t_batched, _ = timed_jobs(plan, x0, v0, r0, wl, reps)
    t_batched /= reps
    assert np.all(plan.poll() == 0)
    del plan
    # plain path: one plan per simulation, run one after the other (FIFO)
    offs = np.concatenate([[0], np.cumsum([s.n for s in wl.sims])])
    plains = []
    for k, s in enumerate(wl.sims):
        sub = Workload("one", [s], [wl.seeds[k]], wl.dtype, wl.steps, wl.ckpt_every, True, wl.loss)
        st = (x0[:, offs[k]:offs[k + 1]].contiguous(), v0[:, offs[k]:offs[k + 1]].contiguous(),
              r0[offs[k]:offs[k + 1]].contiguous())
        p = Plan([s.params()], [s.n], wl.dtype, tape_depth=wl.ckpt_every, device=dev)
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
    lat_plain = np.array([ev0.elapsed_time(e) for e in evs])
    lat_batched = np.full(len(wl.sims), t_batched * 1e3)
    return {"workload": wl.name, "simulations": len(wl.sims), "particles": int(offs[-1]), "sim_steps": wl.steps,
            "pair_interactions": work, "unit": "pair interactions/s",
            "batched": {"value": round(work / t_batched, 1), "ms_per_job": round(t_batched * 1e3, 3),
                        "p50_ms": round(float(np.percentile(lat_batched, 50)), 3),
                        "p99_ms": round(float(np.percentile(lat_batched, 99)), 3)},
            "plain": {"value": round(work / t_plain, 1), "ms_per_job": round(t_plain * 1e3, 3),
                      "p50_ms": round(float(np.percentile(lat_plain, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat_plain, 99)), 3)},
            "speedup": round(t_plain / t_batched, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed passes of the whole job")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tgv2d_64k_f32", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
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
    wl = workloads()[args.workload]()
    host, (x0, v0, r0) = packed_inputs(wl, dev)
    plan = Plan([s.params() for s in wl.sims], [s.n for s in wl.sims], wl.dtype,
                tape_depth=wl.ckpt_every if wl.adjoint else 0, device=dev)
    lanes = autotune.tune(plan, x0, v0, r0) if wl.adjoint else plan.get_tuning()

    for _ in range(args.warmup):
        run_job(plan, x0, v0, r0, wl)
    torch.cuda.synchronize()
    per_state = count_pairs(plan, x0, v0, r0, wl)
    K = wl.ckpt_every
    p_fwd = sum(per_state)
    p_adj = p_fwd if wl.adjoint else 0          # adjoint step n runs on forward state n
    recompute_swept = [n for n in range(wl.steps) if wl.adjoint and (n + 1) % K != 0 and n != wl.steps - 1]
    p_rec = sum(per_state[n] for n in recompute_swept)
    plan.poll()

    elapsed, prof = timed_jobs(plan, x0, v0, r0, wl, args.steps)
    status = plan.poll()
    assert np.all(status == 0), "device reported non-finite values or neighbour overflow: %s" % status
    value = (p_fwd + p_adj) * args.steps / elapsed
    dim = wl.sims[0].dim
    roof = roofline(prof, wl, per_state, args.steps, dim)
    breakdown = {k: round(v[0] / args.steps, 3) for k, v in prof.items()}

    cpu = None
    if not args.no_cpu_baseline and len(wl.sims) == 1:
        cdt, threads = cpu_baseline(wl, host)
        cpu = {"value": round((p_fwd + p_adj) / cdt, 1), "unit": "pair interactions/s", "cores": threads,
               "kind": "oracle",
               "sample": "the whole job once: %d forward steps keeping every state + %d adjoint steps, FP64, "
                         "%d OpenMP threads (%.1f s)" % (wl.steps, wl.steps if wl.adjoint else 0, threads, cdt)}

    batched = None
    if not args.no_batched and args.workload != "batched_512_tgv2d_f32":
        del plan
        torch.cuda.empty_cache()
        batched = bench_batched(dev, max(1, min(args.steps, 3)))

    out = {"metric": METRIC, "value": round(value, 1), "unit": "pair interactions/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl.dtype,
           "data": "synthetic",
           "config": {"workload": wl.name, "dim": dim, "simulations": len(wl.sims),
                      "particles": int(sum(s.n for s in wl.sims)), "sim_steps": wl.steps,
                      "ckpt_every": wl.ckpt_every, "adjoint": wl.adjoint, "loss": wl.loss,
                      "pairs_fwd": p_fwd, "pairs_adj": p_adj, "pairs_recompute": p_rec,
                      "lanes_per_particle": list(lanes)},
           "roofline": roof, "kernel_ms_per_step": breakdown, "cpu_baseline": cpu, "batched": batched}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
