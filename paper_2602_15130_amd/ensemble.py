"""Refinement ensembles: levels x independent replicates of the manufactured
problem, run through the C ABI (one context per member), with the error norms
gathered per member, their replicate mean and spread per level, and the
observed orders of the replicate means (Sec. 4.3; the paper runs one
simulation per level, replicates are independent Philox streams).

Host orchestration only: members of a level run concurrently on several HIP
streams (small meshes are launch bound, large ones fill the GPU alone), and a
small autotuner picks the Poisson solver's workgroup count per level by timing
a few solves.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np

from . import pic
from . import workloads as W

CG_GRID_CHOICES = (256, 128, 64)


def _with_cg_blocks(blocks, fn):
    old = os.environ.get("PIC_CG_BLOCKS")
    if blocks:
        os.environ["PIC_CG_BLOCKS"] = str(blocks)
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop("PIC_CG_BLOCKS", None)
        else:
            os.environ["PIC_CG_BLOCKS"] = old


def autotune_cg_blocks(prob, disc, precision, choices=CG_GRID_CHOICES, steps=3):
    """Time a few steps of replicate 0 for each solver grid size; return the
    fastest grid and the per-choice milliseconds per step."""
    import torch

    timings = {}
    for blocks in choices:
        sim = _with_cg_blocks(blocks, lambda: pic.Sim(prob, disc, 1, 0, precision))
        sim.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        timings[blocks] = 1e3 * (time.perf_counter() - t0) / steps
        del sim
    best = min(timings, key=timings.get)
    return best, timings


def run_level(prob, disc, precision, replicates, seed=1, streams=4, cg_blocks=None):
    """Run every replicate of one level to its final step; returns the l2 and
    linf norms per replicate (arrays [R, 7]) and the wall time."""
    import torch

    dev = torch.device("cuda:0")
    pool = [torch.cuda.Stream(dev) for _ in range(max(1, streams))]
    l2 = np.zeros((len(replicates), 7))
    linf = np.zeros((len(replicates), 7))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for start in range(0, len(replicates), len(pool)):
        batch = replicates[start:start + len(pool)]
        sims = [_with_cg_blocks(cg_blocks, lambda r=r, s=s: pic.Sim(prob, disc, seed, r, precision,
                                                                   "cuda:0", s))
                for r, s in zip(batch, pool)]
        for sim in sims:
            sim.step(disc["steps"])
        for i, sim in enumerate(sims):
            e = sim.errors()
            l2[start + i], linf[start + i] = e["l2"], e["linf"]
        if start == 0:
            st = sims[0].stats()
            solver = {"cg_blocks": st["cg_blocks"], "cg_brick": st["cg_brick"],
                      "cg_iters_last": st["cg_iters"]}
        del sims
    torch.cuda.synchronize()
    run_level.last_solver = solver
    return l2, linf, time.perf_counter() - t0


def run_ensemble(levels=None, replicates=32, precision="mixed", seed=1, streams=4, autotune=True,
                 n_levels=5):
    """The refinement ensemble (mesh 8^3 * 2^l, 8 particles per cell, dt halved
    per level to t = 0.01, two-way coupling, hard-sphere NTC with 16 outcomes):
    per level the replicate norms, their mean and standard deviation, and the
    observed orders of the means."""
    levels = levels if levels is not None else W.ensemble_levels(n_levels)
    reps = list(range(replicates))
    out = {"precision": precision, "replicates": replicates, "levels": []}
    total_ps, total_t = 0, 0.0
    for L in levels:
        prob, disc = L["problem"], L["disc"]
        blocks, tune = (None, None)
        if autotune and disc["nc"][0] >= 32:
            blocks, tune = autotune_cg_blocks(prob, disc, precision)
        nstreams = streams if disc["np"] <= (1 << 20) else 1
        l2, linf, wall = run_level(prob, disc, precision, reps, seed, nstreams, blocks)
        ps = disc["np"] * disc["steps"] * len(reps)
        total_ps += ps
        total_t += wall
        out["levels"].append({
            "mesh": disc["nc"][0], "particles": disc["np"], "steps": disc["steps"],
            "dt": disc["dt"], "cg_blocks": blocks, "cg_tuning_ms_per_step": tune,
            "solver": run_level.last_solver,
            "l2": l2.tolist(), "linf": linf.tolist(),
            "l2_mean": l2.mean(axis=0).tolist(), "l2_std": l2.std(axis=0, ddof=1).tolist()
            if len(reps) > 1 else [0.0] * 7,
            "linf_mean": linf.mean(axis=0).tolist(),
            "wall_s": wall, "particle_steps_per_s": ps / wall})
    means = [lv["l2_mean"] for lv in out["levels"]]
    out["orders_l2_mean"] = W.observed_orders(means)
    out["particle_steps"] = total_ps
    out["wall_s"] = total_t
    out["particle_steps_per_s"] = total_ps / total_t if total_t > 0 else math.nan
    return out
