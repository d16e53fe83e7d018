"""Refinement ensembles: levels x independent replicates of the manufactured
problem, with the error norms per member, their replicate mean and spread per
level, and the observed orders of the replicate means (Sec. 4.3; the paper
runs one simulation per level, the replicates here are independent Philox
streams, key (seed, replicate)).

Each level runs as ensemble contexts of the C ABI (pic_ensemble_init): all
members of a context advance together, one launch per stage for all of them,
so small meshes are not bound by launch latency, and the steps are replayed
from recorded two-step HIP graphs (pic_use_graphs).  A small autotuner picks
the Poisson solver's workgroup count per member for each (device, level,
members) by timing a few steps per choice, and keeps the result in a JSON
cache.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import pic
from . import workloads as W

# workgroups per member of the Poisson solver tried by the autotuner
CG_GRID_CHOICES = (256, 128, 64, 32, 16, 8, 4, 2, 1)
# workspace bytes of one ensemble context at most (larger levels are split
# into several contexts run one after the other)
MAX_CONTEXT_BYTES = 96 << 30


def _with_env(name, value, fn):
    old = os.environ.get(name)
    if value is not None:
        os.environ[name] = str(value)
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop(name, None)
        else:
            os.environ[name] = old


def _cache_path():
    base = os.environ.get("PIC_TUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "paper_2602_15130_amd", "tune.json")


def _cache_key(prob, disc, precision, members, graphs):
    import torch

    dev = torch.cuda.get_device_name(0)
    nc = "x".join(str(n) for n in disc["nc"])
    return f"{dev}|{nc}|np{disc['np']}|navg{disc['navg']}|{precision}|m{members}|" \
           f"coll{int(bool(prob.get('collisions', True)))}|graphs{int(bool(graphs))}"


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def members_per_context(prob, disc, precision, members):
    """Members one context holds within MAX_CONTEXT_BYTES (at least one)."""
    one = pic.pic_ensemble_workspace_size(prob, disc, precision, 1)
    return max(1, min(members, MAX_CONTEXT_BYTES // max(one, 1)))


def _time_steps(prob, disc, precision, members, blocks, steps=4, seed=1, graphs=True):
    import torch

    def make():
        return pic.Ensemble(prob, disc, seed, 0, members, precision)

    with _with_env("PIC_CG_BLOCKS", blocks, make) as ens:
        if graphs:
            ens.use_graphs(True)
        ens.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ens.stats()
    return 1e3 * dt / steps, st


def autotune(prob, disc, precision, members, choices=CG_GRID_CHOICES, use_cache=True, graphs=True):
    """The solver workgroup count per member that steps an ensemble of
    `members` fastest; returns (blocks, {choice: ms per step}, from_cache)."""
    key = _cache_key(prob, disc, precision, members, graphs)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        rec = cache[key]
        return rec["cg_blocks"], {int(k): v for k, v in rec["ms_per_step"].items()}, True
    timings, seen = {}, set()
    for b in choices:
        ms, st = _time_steps(prob, disc, precision, members, b, graphs=graphs)
        # the library fits the request to the mesh and the GPU; requests that
        # end in the same solver grid are timed once
        if st["cg_blocks"] in seen:
            continue
        seen.add(st["cg_blocks"])
        timings[b] = ms
    best = min(timings, key=timings.get)
    if use_cache:
        cache = _load_cache()
        cache[key] = {"cg_blocks": best, "ms_per_step": {str(k): v for k, v in timings.items()}}
        _store_cache(cache)
    return best, timings, False


def run_level(prob, disc, precision, replicates, seed=1, cg_blocks=None, graphs=True):
    """Every replicate of one level to its final step, members of one context
    at a time (replicates must be consecutive).  Returns the l2 and linf norms
    per replicate ([R, 7] arrays), the stepping wall time (init and norms
    excluded: the state is resident when the clock starts) and solver facts."""
    import torch

    reps = list(replicates)
    assert reps == list(range(reps[0], reps[0] + len(reps))), "consecutive replicates"
    per = members_per_context(prob, disc, precision, len(reps))
    l2 = np.zeros((len(reps), 7))
    linf = np.zeros((len(reps), 7))
    wall = 0.0
    solver = None
    for start in range(0, len(reps), per):
        n = min(per, len(reps) - start)

        def make(first=reps[0] + start, n=n):
            return pic.Ensemble(prob, disc, seed, first, n, precision)

        with _with_env("PIC_CG_BLOCKS", cg_blocks, make) as ens:
            if graphs:
                ens.use_graphs(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ens.step(disc["steps"])
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            e = ens.errors()
            l2[start:start + n], linf[start:start + n] = e["l2"], e["linf"]
            if solver is None:
                st = ens.stats()
                solver = {"cg_blocks": st["cg_blocks"], "cg_brick": st["cg_brick"],
                          "cg_iters_last": st["cg_iters"],
                          "cg_members_per_launch": st["cg_members_per_launch"],
                          "members_per_context": per}
    return l2, linf, wall, solver


def run_ensemble(levels=None, replicates=32, precision="mixed", seed=1, tune=True, n_levels=5,
                 use_cache=True, graphs=True):
    """The refinement ensemble (mesh 8^3 * 2^l, 8 particles per cell, dt halved
    per level to t = 0.01, two-way coupling, hard-sphere NTC with 16 outcomes):
    per level the replicate norms, their mean and standard deviation, and the
    observed orders of the means."""
    levels = levels if levels is not None else W.ensemble_levels(n_levels)
    reps = list(range(replicates))
    out = {"precision": precision, "replicates": replicates, "graphs": bool(graphs), "levels": []}
    total_ps, total_t = 0, 0.0
    for L in levels:
        prob, disc = L["problem"], L["disc"]
        blocks, timings, cached = None, None, None
        if tune:
            members = min(replicates, members_per_context(prob, disc, precision, replicates))
            blocks, timings, cached = autotune(prob, disc, precision, members, use_cache=use_cache,
                                               graphs=graphs)
        l2, linf, wall, solver = run_level(prob, disc, precision, reps, seed, blocks, graphs)
        ps = disc["np"] * disc["steps"] * len(reps)
        total_ps += ps
        total_t += wall
        out["levels"].append({
            "mesh": disc["nc"][0], "particles": disc["np"], "steps": disc["steps"],
            "dt": disc["dt"], "cg_blocks": solver["cg_blocks"], "cg_tuning_ms_per_step": timings,
            "tuning_from_cache": cached, "solver": solver,
            "l2": l2.tolist(), "linf": linf.tolist(),
            "l2_mean": l2.mean(axis=0).tolist(),
            "l2_std": l2.std(axis=0, ddof=1).tolist() if len(reps) > 1 else [0.0] * 7,
            "linf_mean": linf.mean(axis=0).tolist(),
            "wall_s": wall, "particle_steps_per_s": ps / wall,
            "ms_per_step": 1e3 * wall / disc["steps"]})
    means = [lv["l2_mean"] for lv in out["levels"]]
    out["orders_l2_mean"] = W.observed_orders(means)
    out["particle_steps"] = total_ps
    out["wall_s"] = total_t
    out["particle_steps_per_s"] = total_ps / total_t if total_t > 0 else math.nan
    return out
