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

The JSON line also carries the roofline of the dominant kernel class (device time from
HIP events recorded by the library on its launch stream during the timed region) and the
CPU oracle timed on the host's cores.
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
            "tgv2d_1k_f64": I.tgv2d_1k_f64}


def run_job(plan, x0, v0, rho0, steps, K, loss_kind, mass, adjoint=True):
    import torch
    from paper_2507_21684_amd.rollout import rollout
    x = x0.clone()
    v = v0.clone().requires_grad_(adjoint)
    r = rho0.clone()
    xT, vT, rT = rollout(plan, x, v, r, steps, K)
    if not adjoint:
        return None
    if loss_kind == "ke":
        loss = 0.5 * mass * (vT ** 2).sum()
    else:
        loss = (vT ** 2).sum()
    loss.backward()
    return v.grad


def cpu_baseline(wl, spec, x, v, rho):
    """The oracle as it stands, on this host's cores, over the same job."""
    from oracle import oracle as O
    import numpy as np
    p = O.Params(**spec.params())
    threads = O.num_threads()
    t0 = time.perf_counter()
    O.rollout(p, x, v, rho, wl.steps, 1 if wl.loss == "ke" else 0)
    dt = time.perf_counter() - t0
    return dt, threads


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed passes of the whole job")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tgv2d_64k_f32", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; runs on more than one GPU are not supported "
              "(independent simulations would be assigned whole to GPUs, with no exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_21684_amd.inputs import make_state
    from paper_2507_21684_amd.lib import Plan

    wl = workloads()[args.workload]()
    spec = wl.sims[0]
    npdt = np.float32 if wl.dtype == "f32" else np.float64
    xs, vs, rs = [a.astype(npdt) for a in make_state(spec, wl.seeds[0])]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    x0, v0, r0 = [torch.tensor(a, device=dev).contiguous() for a in (xs, vs, rs)]
    plan = Plan([spec.params()], [spec.n], wl.dtype, device=dev)
    adjoint = wl.adjoint

    for _ in range(args.warmup):
        run_job(plan, x0, v0, r0, wl.steps, wl.ckpt_every, wl.loss, spec.mass, adjoint)
    torch.cuda.synchronize()

    # pair counts (untimed): the directed pairs (j != i) of every forward state n = 0..T-1,
    # from a step-by-step forward pass
    per_state = []
    xs_, vs_, rs_ = x0.clone(), v0.clone(), r0.clone()
    plan.pair_count()
    for _ in range(wl.steps):
        plan.step(xs_, vs_, rs_, 1)
        per_state.append(plan.pair_count())
    torch.cuda.synchronize()
    K = wl.ckpt_every
    p_fwd = sum(per_state)
    p_adj = p_fwd if adjoint else 0          # adjoint step n runs on forward state n
    # the backward recomputes every segment; its sweeps skip the last state of each segment
    recompute_swept = [n for n in range(wl.steps) if adjoint and (n + 1) % K != 0 and n != wl.steps - 1]
    p_rec = sum(per_state[n] for n in recompute_swept)
    plan.profile_read()
    plan.poll()

    # timed region
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_job(plan, x0, v0, r0, wl.steps, wl.ckpt_every, wl.loss, spec.mass, adjoint)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    prof = plan.profile_read()
    status = plan.poll()
    assert np.all(status == 0), "device reported non-finite values or neighbour overflow: %s" % status

    elapsed = t1 - t0
    work = (p_fwd + p_adj) * args.steps
    value = work / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # roofline of the dominant kernel class: algorithmic flops per launch / mean launch time
    dom = max(("sweep", "adjoint"), key=lambda k: prof[k][0])
    ms_dom, n_dom = prof[dom]
    pairs_dom = (p_fwd + p_rec) if dom == "sweep" else p_adj
    launches_per_job = n_dom / args.steps
    assert launches_per_job == (wl.steps + len(recompute_swept) if dom == "sweep" else wl.steps), launches_per_job
    flops_per_launch = FLOPS_PER_PAIR[(dom, spec.dim)] * pairs_dom / launches_per_job
    mean_launch_s = ms_dom / n_dom * 1e-3
    achieved = flops_per_launch / mean_launch_s / 1e12
    peak = PEAK_TFLOPS[wl.dtype]
    roofline = {"bound": "alu", "kernel": {"sweep": "k_sweep", "adjoint": "k_adj_sweep"}[dom],
                "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "mean_launch_us": round(mean_launch_s * 1e6, 2),
                "pairs_per_launch": int(pairs_dom / launches_per_job)}
    breakdown = {k: round(v[0] / args.steps, 3) for k, v in prof.items()}

    cpu = None
    if not args.no_cpu_baseline:
        xd, vd, rd = [a.astype(np.float64) for a in (xs, vs, rs)]
        cdt, threads = cpu_baseline(wl, spec, xd, vd, rd)
        cpu = {"value": round((p_fwd + p_adj) / cdt, 1), "unit": "pair interactions/s", "cores": threads,
               "kind": "oracle",
               "sample": "the whole job once: %d forward steps keeping every state + %d adjoint steps, FP64, "
                         "%d OpenMP threads (%.1f s)" % (wl.steps, wl.steps if adjoint else 0, threads, cdt)}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "pair interactions/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": wl.dtype,
           "data": "synthetic",
           "config": {"workload": wl.name, "dim": spec.dim, "particles": spec.n, "sim_steps": wl.steps,
                      "ckpt_every": wl.ckpt_every, "adjoint": adjoint, "loss": wl.loss,
                      "pairs_fwd": p_fwd, "pairs_adj": p_adj, "pairs_recompute": p_rec},
           "roofline": roofline, "kernel_ms_per_step": breakdown, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
