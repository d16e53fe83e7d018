"""Throughput of the manufactured-solution PIC/DSMC time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3|cfg2|...]

A step is one pass of the whole path: collision call A, half kick, drift, cell
sort, deposit, Poisson CG, gradient, collision call B, half kick.  Inputs are
resident in HBM before the timed region.  Prints one JSON line with the
whole-job particle-steps/s, the roofline of the dominant kernel (algorithmic
bytes per launch over its mean launch time, from HIP events recorded on the
library's stream during the timed region) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Bytes the method itself must move per particle-step on push + deposit +
# collide, with the uniforms regenerated from Philox rather than stored:
# the particle state read and written once (mixed: cell index 4 + FP32 offsets
# 12 + FP32 velocities 12 = 28 B; FP64: positions 24 + velocities 24 = 48 B)
# and the 4-byte sort key.
METHOD_BYTES = {"mixed": 28 + 28 + 4, "fp64": 48 + 48 + 4}


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def stage_bytes(stage, prob, disc, precision, cg_iters):
    """Bytes this implementation's arrays need per step of a stage (reads +
    writes, mesh arrays counted once): the implementation's own model, larger
    than METHOD_BYTES because it also carries the velocity shape, the sort
    slot and the reordered copy.  Per particle: position
    px (three FP64 coordinates, or three FP32 in-cell offsets with the cell
    index), velocity sv, the manufactured-velocity shape sa (v^M = vbar a, one
    vector per particle), id and cell key 4 bytes each."""
    np_, nn = disc["np"], disc["nc"][0] * disc["nc"][1] * disc["nc"][2]
    coll = bool(prob["collisions"])
    if precision == "fp64":
        px, sv, sa = 24, 24, 24
        sx = px                  # absolute position
    else:
        px, sv, sa = 12, 12, 12
        sx = px + 4              # cell index + in-cell offsets
    if stage == "collide":       # velocities in, averaged velocity change out
        return (sv + sv) * np_ + 4 * nn
    if stage == "kick":          # x, v, <dv> and cell key in; v out; E and cell starts
        return (sx + sv + (sv + 4 if coll else 0) + sv) * np_ + 28 * nn
    if stage == "drift":         # x, v, a in; x, key, slot out
        return (sx + sv + sa + sx + 4 + 4) * np_ + 4 * nn
    if stage == "sort":          # scatter slots (key, slot -> index, key); the
        # ordered move reads the indices and gathers/scatters x, v, a, id; key
        # out; in the fused step it also writes the cell moments (64 B a cell)
        return (16 + 8 + 2 * (px + sv + sa + 4) + 4) * np_ + 12 * nn + 64 * nn
    if stage == "deposit":       # cell moments in; node charge and right-hand
        # side out, the right-hand side's mean removed
        return 64 * nn + 16 * nn + 16 * nn
    if stage == "cg":            # per iteration: stencil on p and r, update x, r
        return max(cg_iters, 1) * 80 * nn
    if stage == "gradient":
        return 32 * nn
    if stage == "particle":      # fused pass: x, v, a, key in; x, v, key, slot out
        return (2 * (px + sv) + sa + 4 + 4 + 4) * np_ + 28 * nn
    return 0


# Every source that goes into the library: a change to any of them voids the
# committed counter record.
DEVICE_SOURCES = ("pic.hip", "pic_device.hpp", "pic_kernels.hpp", "pic_particle.hpp", "pic_mixed.hpp",
                  "pic_cg_brick.hpp", "pic_lowmode.hpp", "pic_angles.hpp", "pic_collide_heavy.hpp",
                  "pic_order.hpp", "pic_host.hpp")


def measured_traffic(stage, workload):
    """HBM bytes per step of a stage from the committed hardware-counter record
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when the record is for another
    workload or the device sources have changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_15130_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["device_sources_sha256_16"] or rec["workload"] != workload:
        return None
    m = rec["per_step_MiB"].get(stage)
    if m is None:
        return None
    f = rec["copy_factor"]
    return int((m["FETCH_SIZE"] * f["FETCH_SIZE"] + m["WRITE_SIZE"] * f["WRITE_SIZE"]) * 2**20)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cells_by_id(cell_start, ids):
    """Cell of every particle, indexed by particle id, from a cell-sorted order."""
    import numpy as np
    cells = np.repeat(np.arange(len(cell_start) - 1), np.diff(cell_start))
    out = np.empty_like(cells)
    out[ids] = cells
    return out


def _compare_with_oracle(pic, g, o, prob, disc):
    """Per-quantity differences of a GPU simulation from the FP64 oracle at the
    same step, by particle identity: largest position difference (minimum
    image) in cells and velocity difference in vbar over the particles whose
    cell agrees, the number whose cell differs, phi and rho relative to their
    largest value, and the relative differences of the error norms."""
    import numpy as np
    ig, io = g.get(pic.STATE_ID), o.get(o.ID)
    xg, xo = np.empty((3, disc["np"])), np.empty((3, disc["np"]))
    vg, vo = np.empty_like(xg), np.empty_like(xo)
    xg[:, ig], xo[:, io] = g.get(pic.STATE_X), o.get(o.X)
    vg[:, ig], vo[:, io] = g.get(pic.STATE_V), o.get(o.V)
    same = _cells_by_id(g.get(pic.STATE_CELL_START), ig) == _cells_by_id(o.get(o.CELL_START), io)
    L = np.array(prob["L"])[:, None]
    h = prob["L"][0] / disc["nc"][0]
    dx = np.abs(xg - xo)
    dx = np.minimum(dx, L - dx).max(axis=0)
    dv = np.abs(vg - vo).max(axis=0)
    pg, po = g.get(pic.STATE_PHI), o.get(o.PHI)
    rg, ro = g.get(pic.STATE_RHO), o.get(o.RHO)
    eg, eo = g.errors(), o.errors()
    return {"step": int(o.step_index),
            "max_dx_over_h": float(dx[same].max() / h),
            "max_dv_over_vbar": float(dv[same].max() / prob["vbar"]),
            "cell_flips": int((~same).sum()),
            "phi_rel": float(np.abs(pg - po).max() / np.abs(po).max()),
            "rho_rel": float(np.abs(rg - ro).max() / np.abs(ro).max()),
            "l2_rel": [float("%.3g" % v) for v in np.abs(eg["l2"] / eo["l2"] - 1)],
            "accepted": {"gpu": int(g.stats()["n_accepted"]), "oracle": int(o.accepted)}}


def oracle_leg(pic, prob, disc, seed, precision):
    """The oracle on the host cores, on a bounded sample of the workload: init
    (untimed, all threads), one time step on all threads, one on a single
    thread (particle-steps/s each).  The same two oracle steps also give the
    per-quantity differences of the GPU form from the FP64 oracle at full size
    (a GPU simulation from the same initial state, compared after each step)."""
    import oracle as O

    nthreads = O.max_threads()
    progress(f"oracle init ({disc['np']} particles, {nthreads} threads)")
    o = O.Sim(prob, disc, seed, 0)
    o.init()
    g = pic.Sim(prob, disc, seed, 0, precision)
    rates, parity = {}, []
    try:
        for threads in (nthreads, 1):
            O.set_threads(threads)
            progress(f"oracle step on {threads} thread(s)")
            t0 = time.perf_counter()
            o.step(1)
            rates[threads] = (disc["np"] / (time.perf_counter() - t0), time.perf_counter() - t0)
            g.step(1)
            parity.append(_compare_with_oracle(pic, g, o, prob, disc))
    finally:
        O.set_threads(nthreads)
        g.close()
    base = {"value": rates[nthreads][0], "unit": "particle-steps/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"one time step of the full workload ({disc['np']} particles, "
                      f"{disc['nc'][0]}^3 mesh) after init, FP64 C with OpenMP over the "
                      f"independent per-particle and per-cell loops, {nthreads} threads, "
                      f"{rates[nthreads][1]:.1f} s",
            "single_core": {"value": rates[1][0], "cores": 1,
                            "sample": f"the next time step on one thread, {rates[1][1]:.1f} s"},
            "nproc": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model()}
    return base, {"reference": "FP64 oracle", "form": precision, "steps": parity}


def convergence_report(pic, W, levels=(0, 1, 2, 3)):
    """Observed orders of the FP64 and mixed forms on the refinement ladder
    (one-way, collisionless: second order in h and dt), from the l2 norms of
    x, y, z, u, v, w and phi at t = 0.01."""
    ladder = W.order_ladder(levels)
    rep = {"ladder": "mesh 8^3 * 2^l, 8 particles per cell, dt 1e-3 / 2^l, t = 0.01, "
                     "one-way, collisionless", "levels": [L["disc"]["nc"][0] for L in ladder]}
    orders = {}
    for precision in ("fp64", "mixed"):
        norms = []
        for L in ladder:
            g = pic.Sim(L["problem"], L["disc"], 1, 0, precision)
            g.step(L["disc"]["steps"])
            norms.append(list(g.errors()["l2"]))
            g.close()
        orders[precision] = W.observed_orders(norms)
        rep[precision] = {"l2": [[float("%.6g" % v) for v in n] for n in norms],
                          "orders": [[round(v, 4) for v in o] for o in orders[precision]]}
    gap = max(abs(a - b) for oa, ob in zip(orders["fp64"], orders["mixed"]) for a, b in zip(oa, ob))
    rep["max_order_gap"] = round(gap, 5)
    return rep


def paper_ladder_report(pic, W, levels=(1, 2, 3), cases=("coupled", "isolated")):
    """The paper's refinement ladder (Table 1, Sec. 5.4; the Sec. 5.2
    manufactured functions in SI units) in both forms: l2 norms of x, y, z, u,
    v, w and phi at t = T per level, observed orders between levels, and the
    largest gap between the two forms' orders (the mixed form must match)."""
    import math
    kw = {"coupled": dict(collisions=True),
          "isolated": dict(collisions=True, field_to_particles=False, particles_to_field=False,
                           isolate=True)}
    n = [W.TABLE1_NCELL[lv - 1] for lv in levels]
    rep = {"ladder": "Table 1 levels %s (%s cells per axis), s = 7, r = 5"
                     % (",".join(map(str, levels)), ",".join(map(str, n)))}
    for case in cases:
        prob = W.paper_problem(**kw[case])
        orders, out = {}, {}
        for precision in ("fp64", "mixed"):
            norms = []
            for lv in levels:
                progress(f"paper ladder {case} {precision} level {lv}")
                disc = W.paper_level(lv)
                with pic.Sim(prob, disc, 1, 0, precision) as g:
                    g.step(disc["steps"])
                    norms.append(list(g.errors()["l2"]))
            orders[precision] = [[math.log(a / b) / math.log(n[i + 1] / n[i])
                                  for a, b in zip(norms[i], norms[i + 1])]
                                 for i in range(len(levels) - 1)]
            out[precision] = {"l2": [[float("%.6g" % v) for v in x] for x in norms],
                              "orders": [[round(v, 4) for v in o] for o in orders[precision]]}
        out["max_order_gap"] = round(max(abs(a - b) for oa, ob in zip(orders["fp64"], orders["mixed"])
                                         for a, b in zip(oa, ob)), 5)
        rep[case] = out
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--beside", default="cfg2",
                    help="second workload timed beside the first (the FP64 form); 'none' to skip")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-convergence", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads' records (cfg1, cfg3 without collisions, 128^3, paper family at 64^3)")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the refinement-ensemble (cfg4) block of the default line")
    ap.add_argument("--levels", default="1,2,3", help="Table 1 levels for --workload table1")
    ap.add_argument("--cases", default="isolated,coupled,collisionless",
                    help="Table 1 cases for --workload table1")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes five times (reference for "
                         "hardware byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the path is built and measured on a single "
              "MI355X (the multi-GPU sharding is a design, not a measured run)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_15130_amd import pic, workloads as W

    if args.workload == "cfg4":
        print(json.dumps(run_ensemble_bench()), flush=True)
        return
    if args.workload == "table1":
        print(json.dumps(run_table1(args.levels, args.cases)), flush=True)
        return
    progress(f"timing {args.workload}")
    out = run_workload(pic, W, torch, args.workload, args.steps, args.warmup)
    if args.beside and args.beside != "none":
        progress(f"timing {args.beside}")
        b = run_workload(pic, W, torch, args.beside, args.steps, args.warmup)
        out["beside"] = {k: b[k] for k in ("value", "ms_per_step", "dtype", "config", "roofline",
                                           "roofline_particle_path", "stages", "cg_iters_last")}
    if not args.no_convergence:
        progress("convergence ladder")
        out["convergence"] = convergence_report(pic, W)
        out["convergence"]["paper_ladder"] = paper_ladder_report(pic, W)
    if not args.no_extra:
        # the other single-GPU workloads, each as a compact record (20 timed
        # steps): the 32^3 two-way collisionless FP64 case, the headline
        # case without collisions, the 128^3 single-simulation point and the
        # paper's own functions at 64^3
        out["more_workloads"] = {}
        for w in ("cfg1", "cfg3_collisionless", "cfg3_128", "cfg3_paper", "cfg2_paper"):
            progress(f"timing {w}")
            r = run_workload(pic, W, torch, w, min(args.steps, 20), 2)
            out["more_workloads"][w] = {
                "value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"],
                "dtype": r["dtype"], "config": r["config"], "stages": r["stages"],
                "roofline": {k: r["roofline"][k] for k in ("kernel", "achieved", "frac",
                                                           "us_per_step")}}
    if not args.no_ensemble:
        progress("refinement ensemble (cfg4)")
        e = run_ensemble_bench()
        out["ensemble"] = {k: e[k] for k in ("value", "unit", "config", "particle_steps", "wall_s",
                                             "levels", "level_rate_vs_best")}
    if not args.no_cpu_baseline:
        c = W.get(args.workload)
        out["cpu_baseline"], out["parity_vs_oracle"] = oracle_leg(
            pic, c["problem"], c["disc"], c["seed"], c["precision"])
    print(json.dumps(out), flush=True)


def run_ensemble_bench(replicates=32):
    """The batched refinement ensemble: 5 levels (8^3 .. 128^3, 8 particles per
    cell, dt halved per level to t = 0.01) x 32 replicates, mixed form, two-way,
    hard-sphere NTC with 16 outcomes.  Each level runs as one ensemble context
    (all replicates advance together, one launch per stage); the solver grid is
    autotuned per level.  Throughput over all members, stepping only (the
    state is resident when each level's clock starts)."""
    from paper_2602_15130_amd import ensemble

    out = ensemble.run_ensemble(replicates=replicates, precision="mixed")
    lv = [{k: x[k] for k in ("mesh", "particles", "steps", "solver", "wall_s", "ms_per_step",
                             "particle_steps_per_s", "cg_tuning_ms_per_step", "l2_mean", "l2_std")}
          for x in out["levels"]]
    top = max(x["particle_steps_per_s"] for x in out["levels"])
    return {"metric": "particle-steps/s", "value": out["particle_steps_per_s"],
            "unit": "particle-steps/s", "n_gpus": 1, "steps": None, "warmup": 0,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic (manufactured solution, Philox seed 1)",
            "config": {"workload": "cfg4", "levels": [x["mesh"] for x in out["levels"]],
                       "replicates": replicates, "precision": "mixed"},
            "particle_steps": out["particle_steps"], "wall_s": out["wall_s"], "levels": lv,
            "level_rate_vs_best": [x["particle_steps_per_s"] / top for x in out["levels"]],
            "orders_l2_mean": out["orders_l2_mean"]}


def run_table1(levels, cases_arg="isolated,coupled,collisionless"):
    """The paper's Table 1 ladder, FP64 form: isolated collisions, fully coupled
    collisional and fully coupled collisionless; l2 / linf norms per level and
    observed orders (progress to stderr, one line per step)."""
    import math

    import torch
    from paper_2602_15130_amd import pic, workloads as W

    levels = [int(x) for x in levels.split(",")]
    cases = {"isolated": dict(collisions=True, field_to_particles=False, particles_to_field=False,
                              isolate=True),
             "coupled": dict(collisions=True), "collisionless": dict(collisions=False)}
    out = {"workload": "table1", "levels": levels, "cases": {}}
    wanted = cases_arg.split(",")
    for name, kw in cases.items():
        if name not in wanted:
            continue
        prob = W.paper_problem(**kw)
        rows = []
        for lv in levels:
            disc = W.paper_level(lv, collisions=kw.get("collisions", True))
            g = pic.Sim(prob, disc, 1, 0, "fp64")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(disc["steps"]):
                g.step(1)
                torch.cuda.synchronize()
                print(f"{name} level {lv} step {s + 1}/{disc['steps']} {time.perf_counter() - t0:.1f}s",
                      file=sys.stderr, flush=True)
            wall = time.perf_counter() - t0
            e = g.errors()
            rows.append({"level": lv, "ncell": disc["nc"][0], "particles": disc["np"],
                         "n_avg": disc["navg"], "steps": disc["steps"], "wall_s": round(wall, 2),
                         "accepted": g.stats()["n_accepted"], "l2": [float(x) for x in e["l2"]],
                         "linf": [float(x) for x in e["linf"]]})
            g.close()
        orders = []
        for a, b in zip(rows, rows[1:]):
            r = math.log(b["ncell"] / a["ncell"])
            orders.append({"levels": [a["level"], b["level"]],
                           "l2": [round(math.log(x / y) / r, 3) for x, y in zip(a["l2"], b["l2"])],
                           "linf": [round(math.log(x / y) / r, 3) for x, y in zip(a["linf"], b["linf"])]})
        out["cases"][name] = {"runs": rows, "orders": orders}
    return out


def run_workload(pic, W, torch, workload, steps, warmup):
    c = W.get(workload)
    prob, disc, precision, seed = c["problem"], c["disc"], c["precision"], c["seed"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sim = pic.Sim(prob, disc, seed, 0, precision, "cuda:0", stream)
    if warmup:
        sim.step(warmup)
    # Stage breakdown: a few steps with every stage bracketed by HIP events on
    # the library's stream.  Every stage runs once per step (the fused particle
    # pass runs as step-straddling launches: the B half of one step with the A
    # half of the next), so rates are per step: algorithmic bytes of one step's
    # worth of the stage over its time per step.
    nbreak = max(1, min(steps, 10))
    torch.cuda.synchronize()
    sim.timing(True)
    sim.step(nbreak)
    stages = sim.timing_read()
    st = sim.stats()
    per_stage = {}
    for name, (ms, n) in stages.items():
        if n == 0:
            continue
        b = stage_bytes(name, prob, disc, precision, st["cg_iters"])
        per_stage[name] = {"ms_total": round(ms, 3), "launches": n,
                           "us_per_step": round(1e3 * ms / nbreak, 2),
                           "GBs": round(b / (ms / nbreak * 1e-3) / 1e9, 1)}
    dom = max(per_stage, key=lambda k: per_stage[k]["ms_total"])
    # The timed region: events only around the dominant stage, whose average
    # time per step over these K steps gives the roofline's achieved rate.
    sim.timing_stages([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms, dom_n = sim.timing_read()[dom]
    sim.timing(False)
    st = sim.stats()
    elapsed = t1 - t0
    value = disc["np"] * steps / elapsed

    impl_bytes = stage_bytes(dom, prob, disc, precision, st["cg_iters"])
    dom_s = dom_ms / steps * 1e-3
    # the fused particle pass is push + collide; its roofline uses the method's
    # minimum bytes, the implementation's own model is reported beside it
    dom_bytes = METHOD_BYTES[precision] * disc["np"] if dom == "particle" else impl_bytes
    ach = dom_bytes / dom_s / 1e9
    kernel_names = {"particle": "k_particles_" + ("f64" if precision == "fp64" else "mixed"),
                    "cg": "k_cg_brick / k_cg (+ low-mode pre-solve)", "sort": "k_order_tiles",
                    "deposit": "k_deposit_tiles"}
    roof = {"bound": "hbm", "kernel": kernel_names.get(dom, dom), "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, workload), "algorithmic_bytes_per_step": dom_bytes,
            "bytes_basis": ("method minimum, %d B per particle-step" % METHOD_BYTES[precision]
                            if dom == "particle" else "implementation model"),
            "implementation_bytes_per_step": impl_bytes,
            "implementation_GBs": round(impl_bytes / dom_s / 1e9, 1),
            "per": "time step", "us_per_step": round(1e3 * dom_ms / steps, 2), "launches": dom_n}
    # push + deposit + collide: the fused pass, the sort (which deposits) and
    # the node charge, at the method's minimum bytes per particle-step
    part_names = [k for k in ("particle", "collide", "kick", "drift", "sort", "deposit") if k in per_stage]
    pb = METHOD_BYTES[precision] * disc["np"]
    pms = sum(per_stage[k]["ms_total"] for k in part_names) / nbreak
    pach = pb / (pms * 1e-3) / 1e9
    impl_pb = sum(stage_bytes(k, prob, disc, precision, st["cg_iters"]) for k in part_names)
    roof_part = {"bound": "hbm", "kernels": part_names, "achieved": round(pach, 1),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(pach / HBM_PEAK_GBS, 4),
                 "ms_per_step": round(pms, 3),
                 "method_bytes_per_particle_step": METHOD_BYTES[precision],
                 "implementation_bytes_per_particle_step": round(impl_pb / disc["np"], 1)}
    out = {
        "metric": "particle-steps/s", "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic (manufactured solution, Philox seed %d)" % seed,
        "config": {"workload": workload, "family": prob["family"], "mesh": list(disc["nc"]),
                   "particles": disc["np"],
                   "n_avg": disc["navg"], "dt": disc["dt"], "precision": precision,
                   "collisions": bool(prob["collisions"]), "two_way": bool(prob["particles_to_field"])},
        "roofline": roof,
        "roofline_particle_path": roof_part,
        "stages": per_stage,
        "stages_steps": nbreak,
        "cg_iters_last": st["cg_iters"],
        "cg_solver": {"blocks": st["cg_blocks"], "brick": st["cg_brick"]},
        "accepted_collisions": st["n_accepted"],
    }
    sim.close()
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    main()
