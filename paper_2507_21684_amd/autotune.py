"""Autotuner for the lanes-per-particle setting of the forward and adjoint sweeps.

The sweeps sum every particle's neighbours as eight canonical partial sums, so the number of
lanes sharing a particle (2, 4 or 8) changes only the speed, never the result.  The tuner
times each setting on the caller's own state with the library's HIP-event profiler (a few
forward steps and one taped backward segment), keeps the fastest setting per sweep, and
caches it in a JSON file keyed by GPU architecture, dimension, dtype and a power-of-two
bucket of the plan's particle count.  The cache path is $SPH_TUNING_CACHE, else
~/.cache/paper_2507_21684_amd/tuning.json.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Tuple

import torch

from .lib import Plan

LANE_CHOICES = (2, 4, 8)


def cache_path() -> str:
    return os.environ.get("SPH_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2507_21684_amd", "tuning.json"))


def _arch() -> str:
    try:
        return str(torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName).split(":")[0]
    except Exception:  # pragma: no cover - property missing on some builds
        return "unknown"


def cache_key(plan: Plan) -> str:
    bucket = 1 << max(0, int(math.ceil(math.log2(max(plan.N, 1)))))
    return "%s:d%d:%s:n%d" % (_arch(), plan.dim, plan.dtype, bucket)


def _load() -> Dict[str, list]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(table: Dict[str, list]) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def measure(plan: Plan, x, v, rho, steps: int = 4, reps: int = 2) -> Dict[int, Tuple[float, float]]:
    """{lanes: (forward-sweep ms per launch, adjoint-sweep ms per launch)} on copies of the state."""
    out = {}
    K = min(steps, max(1, plan.tape_depth))
    for lanes in LANE_CHOICES:
        plan.set_tuning(lanes, lanes)
        best_f, best_a = float("inf"), float("inf")
        for _ in range(reps):
            xs, vs, rs = x.clone(), v.clone(), rho.clone()
            ck = [plan.empty_state()]
            plan.profile_read()
            plan.profile(True, ["sweep", "adjoint"])
            plan.step(xs, vs, rs, K, ck, K)
            gx, gv, gr = torch.zeros_like(x), torch.ones_like(v), torch.zeros_like(rho)
            plan.rollout_backward(ck, K, K, gx, gv, gr)
            torch.cuda.synchronize()
            plan.profile(False)
            prof = plan.profile_read()
            ms_f, n_f = prof["sweep"]
            ms_a, n_a = prof["adjoint"]
            best_f = min(best_f, ms_f / max(n_f, 1))
            best_a = min(best_a, ms_a / max(n_a, 1))
        out[lanes] = (best_f, best_a)
    return out


def tune(plan: Plan, x, v, rho, use_cache: bool = True) -> Tuple[int, int]:
    """Set and return the fastest (lanes_fwd, lanes_adj) for this plan."""
    key = cache_key(plan)
    table = _load() if use_cache else {}
    if key in table:
        lf, la = int(table[key][0]), int(table[key][1])
    else:
        times = measure(plan, x, v, rho)
        lf = min(times, key=lambda k: times[k][0])
        la = min(times, key=lambda k: times[k][1])
        if use_cache:
            table[key] = [lf, la, {str(k): list(t) for k, t in times.items()}]
            _store(table)
    plan.set_tuning(lf, la)
    return lf, la


def apply_cached(plan: Plan) -> Optional[Tuple[int, int]]:
    """Set the cached setting for this plan's bucket if there is one (never measures)."""
    entry = _load().get(cache_key(plan))
    if entry is None:
        return None
    lf, la = int(entry[0]), int(entry[1])
    plan.set_tuning(lf, la)
    return lf, la
