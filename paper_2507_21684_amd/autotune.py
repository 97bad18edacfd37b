"""Autotuner for the plan settings that change speed but not the physics.

* Lanes per particle of the forward and adjoint sweeps (2, 4 or 8).  The sweeps sum every
  particle's neighbours as eight canonical partial sums, so this changes only the speed, never
  the result.  `tune` times each setting on the caller's own state with the library's
  HIP-event profiler (a few forward steps and one taped backward segment) and keeps the
  fastest per sweep.
* Neighbour-list rebuild interval R and skin (the cell size follows the list radius).  Lists
  reused for R steps save R - 1 of every R sorts and builds but hold more entries, which the
  sweeps filter back to r < H.  Half the skin must cover R steps of travel, so each
  simulation's skin is 2 x 1.3 x v_max dt R / H from the largest speed of its state (30 %
  margin), and the plans take speed-scaled half skins (sph_set_skin_mode): each particle's
  list radius follows its own speed, with a floor for acceleration, and the device flags any
  particle that moves farther than its own half skin.  `tune_plan` builds a plan per
  candidate R dividing the checkpoint interval, tunes its lanes, times one checkpoint segment
  forward and backward (with a tape as deep as the segment, so the backward runs on the
  forward's tape), discards candidates whose run raised a device flag, and returns the fastest
  plan, with a tape as deep as the caller asks.

Choices are cached in a JSON file keyed by GPU architecture, dimension, dtype and a
power-of-two bucket of the plan's particle count (the cache path is $SPH_TUNING_CACHE, else
~/.cache/paper_2507_21684_amd/tuning.json).
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional, Sequence, Tuple

import torch

from .lib import Plan

LANE_CHOICES = (2, 4, 8)
REBUILD_CHOICES = (1, 2, 4, 8)
SKIN_MARGIN = 1.3


def rebuild_for(ckpt_every: int, want: int = 8) -> int:
    """Largest rebuild interval not above `want` that divides the checkpoint interval."""
    for R in range(min(want, ckpt_every), 0, -1):
        if ckpt_every % R == 0:
            return R
    return 1


def skin_from_speed(vmax: float, p: dict, R: int) -> float:
    """List skin (fraction of the support) whose half covers R steps at SKIN_MARGIN x vmax."""
    if R <= 1:
        return 0.0
    skin = 2.0 * SKIN_MARGIN * vmax * float(p["dt"]) * R / float(p["H"])
    cap = 0.95 * (float(p["L"]) / (2.0 * float(p["H"])) - 1.0)   # keeps 2 H (1 + skin) < L
    return min(max(skin, 0.05), cap, 1.0)


def skins_for(sims, counts, v, R: int):
    """Per-simulation list skin (fraction of the support) for rebuild interval R: half the skin
    covers R steps at SKIN_MARGIN times the largest speed of the simulation's state."""
    if R <= 1:
        return [0.0] * len(sims)
    speed = torch.sqrt((v.double() ** 2).sum(dim=0)).cpu().numpy()
    out, a = [], 0
    for p, c in zip(sims, counts):
        vmax = float(speed[a:a + c].max()) if c > 0 else 0.0
        a += c
        out.append(skin_from_speed(vmax, p, R))
    return out


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


_TABLE: Dict[str, tuple] = {}   # path -> (modification time, table): the file is read once per change


def _load() -> Dict[str, list]:
    path = cache_path()
    try:
        mtime = os.stat(path).st_mtime_ns
    except OSError:
        return {}
    hit = _TABLE.get(path)
    if hit is not None and hit[0] == mtime:
        return dict(hit[1])
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return {}
    _TABLE[path] = (mtime, table)
    return dict(table)


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
    R = getattr(plan, "rebuild_every", 1)
    K = min(steps, max(1, plan.tape_depth))
    K = R * max(1, K // R)          # checkpoint intervals are multiples of the rebuild interval
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


def _segment_seconds(plan: Plan, x, v, rho, K: int, reps: int = 3) -> Tuple[float, int]:
    """Wall time of K forward steps with a checkpoint plus their taped backward; status bits."""
    ck = [plan.empty_state()]
    best = float("inf")
    plan.poll()
    for _ in range(reps + 1):
        xs, vs, rs = x.clone(), v.clone(), rho.clone()
        gx, gv, gr = torch.zeros_like(x), torch.ones_like(v), torch.zeros_like(rho)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(xs, vs, rs, K, ck, K)
        plan.rollout_backward(ck, K, K, gx, gv, gr)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    status = int(plan.poll().max()) if plan.nsims else 0
    return best, status


def _reuse_plan(sims, counts, dtype, depth: int, device, v, R: int) -> Plan:
    """Plan rebuilding every R steps with skins from the state's speeds (speed-scaled half skins)."""
    return Plan(sims, counts, dtype, tape_depth=depth, device=device, skin=skins_for(sims, counts, v, R),
                rebuild_every=R, speed_skins=R > 1)


def tune_plan(sims: Sequence[dict], counts: Sequence[int], dtype: str, ckpt_every: int, x, v, rho,
              device=None, use_cache: bool = True, choices=REBUILD_CHOICES, tape_depth: Optional[int] = None) -> Plan:
    """Plan with the fastest (rebuild interval, skins, lanes) for one checkpoint segment of this state.
    The returned plan has tape_depth slots (default: the checkpoint interval); with as many slots as a
    rollout has steps, the forward keeps every step and the backward runs without recomputing."""
    K = int(ckpt_every)
    depth = K if tape_depth is None else max(int(tape_depth), K)
    probe = Plan(sims, counts, dtype, tape_depth=K, device=device)
    key = cache_key(probe) + ":K%d:reuse-speed" % K
    del probe
    table = _load() if use_cache else {}
    if key in table:
        R, lf, la = (int(t) for t in table[key][:3])
        plan = _reuse_plan(sims, counts, dtype, depth, device, v, R)
        plan.set_tuning(lf, la)
        return plan
    best, trials = None, {}
    for R in choices:
        if K % R:
            continue
        plan = _reuse_plan(sims, counts, dtype, K, device, v, R)
        lf, la = tune(plan, x, v, rho, use_cache=False)
        secs, status = _segment_seconds(plan, x, v, rho, K)
        trials[str(R)] = [secs, status, lf, la, round(plan.skin, 4)]
        if status == 0 and (best is None or secs < best[0]):
            best = (secs, R, lf, la)
        del plan
    if best is None:
        raise RuntimeError("no list setting ran without device flags: %s" % trials)
    _, R, lf, la = best
    if use_cache:
        table[key] = [R, lf, la, trials]
        _store(table)
    plan = _reuse_plan(sims, counts, dtype, depth, device, v, R)
    plan.set_tuning(lf, la)
    return plan
