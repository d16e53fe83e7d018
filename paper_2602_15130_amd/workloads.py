"""Workload descriptions: plain parameter dicts for the problems that are run.

Holds no arithmetic of the method — only problem constants and sizes, so that
the GPU library and the CPU oracle can be fed the same inputs.  Two families of
manufactured solutions are described:

* ``paper``: the functions and SI constants of the paper's numerical examples
  (Sec. 5.2) and the five discretizations of its Table 1.
* ``cfg``: the synthetic configurations used for throughput measurement: unit
  cube, number density proportional to 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z),
  Gaussian velocities with unit variance, the paper's manufactured potential on
  the unit cube, and the paper's dimensionless groups (q/m phibar / vbar^2,
  q N L^2 / (V eps0 phibar), nu_max T) carried over.
"""
from __future__ import annotations

import copy
import math

# ---- SI constants of Sec. 5.2 ------------------------------------------------
E_CHARGE = 1.602176634e-19          # C
M_ELECTRON = 9.1093837015e-31       # kg
EPS0 = 8.8541878128e-12             # F/m
VBAR = 1.0e6                        # m/s
SIGBAR = 1.0e-20                    # 1 Angstrom^2 in m^2
L_PAPER = 1.5                       # m
N_PAPER = 1.0e20
T_PAPER = L_PAPER / (10.0 * VBAR)   # s
PHIBAR_PAPER = 1.0e10               # V
GMAX_PAPER = 10.0 * math.sqrt(3.0) * VBAR

# Fig. 1a's sigma_n values are not in the text.  Any admissible set works if
# sigma(g) > 0 on (0, g_max] and max over [0, g_max] of sigma(g) g equals
# 33.2464 sigbar vbar, the value implied by every row of Table 1's 1/P_coll,max.
# This set peaks at g = 10 vbar: sigma g = s0 + s1 g^2 + s2 g^4.
SIGMA_N_PAPER = (28.2464 * SIGBAR * VBAR, 0.1 * SIGBAR / VBAR, -5.0e-4 * SIGBAR / VBAR**3)


def paper_problem(collisions=True, field_to_particles=True, particles_to_field=True,
                  isolate=False, coding_error=0, sigma_n=SIGMA_N_PAPER):
    return {
        "family": "paper", "L": (L_PAPER,) * 3, "nphys": N_PAPER, "q": E_CHARGE,
        "m": 3.0e8 * M_ELECTRON, "eps0": EPS0, "T": T_PAPER, "vbar": VBAR,
        "phibar": PHIBAR_PAPER, "rho_amp": 0.0, "sigma_model": "poly",
        "sigma_n": tuple(sigma_n), "sigma_ref": 0.0, "g_ref": 1.0, "omega": 0.5,
        "g_max": GMAX_PAPER, "field_to_particles": int(field_to_particles),
        "particles_to_field": int(particles_to_field), "collisions": int(collisions),
        "isolate": int(isolate), "coding_error": int(coding_error),
    }


# Table 1: N_cell_i, with T/dt = N_cell_i, k = N_cell_i / 4, N_avg = k^5,
# N_p = 80 k^7 (collisional) or 320 k^5 (collisionless).
TABLE1_NCELL = (8, 12, 16, 20, 24)


def paper_level(level: int, collisions=True, cg_tol=1e-12):
    n = TABLE1_NCELL[level - 1]
    k = n // 4
    np_ = 80 * k**7 if collisions else 320 * k**5
    return {"nc": (n, n, n), "np": np_, "dt": T_PAPER / n, "steps": n,
            "navg": k**5 if collisions else 1, "cg_tol": cg_tol, "cg_max_iter": 20000}


# ---- configuration family ----------------------------------------------------
# Dimensionless groups of the paper's constants, carried to a unit box with
# vbar = 1, phibar = 1, N = 1, eps0 = 1 and T = L / (10 vbar) = 0.1.
Q_OVER_M_CFG = (E_CHARGE / (3.0e8 * M_ELECTRON)) * PHIBAR_PAPER / VBAR**2
Q_CFG = E_CHARGE * N_PAPER * L_PAPER**2 / (L_PAPER**3 * EPS0 * PHIBAR_PAPER)
NU_MAX_T = 33.2464 * SIGBAR * VBAR * N_PAPER * T_PAPER / L_PAPER**3
T_CFG = 0.1
GMAX_CFG = 10.0 * math.sqrt(3.0)
SIGMA_HS_CFG = NU_MAX_T / (GMAX_CFG * T_CFG)   # hard-sphere cross section, same nu_max T


def cfg_problem(two_way=True, collisions=True, field_to_particles=True, sigma="hs",
                collisionality=1.0, isolate=False):
    p = {
        "family": "cfg", "L": (1.0, 1.0, 1.0), "nphys": 1.0, "q": Q_CFG,
        "m": Q_CFG / Q_OVER_M_CFG, "eps0": 1.0, "T": T_CFG, "vbar": 1.0, "phibar": 1.0,
        "rho_amp": 0.5, "sigma_model": "vhs", "sigma_n": (0.0,),
        "sigma_ref": SIGMA_HS_CFG * collisionality, "g_ref": 1.0, "omega": 0.5,
        "g_max": GMAX_CFG, "field_to_particles": int(field_to_particles),
        "particles_to_field": int(two_way), "collisions": int(collisions),
        "isolate": int(isolate), "coding_error": 0,
    }
    if sigma == "maxwell":
        p["omega"] = 1.0
    elif sigma == "poly":
        p["sigma_model"] = "poly"
        s = SIGMA_HS_CFG * collisionality
        p["sigma_n"] = (s * 28.2464 / 33.2464, s * 0.1 / 33.2464, -s * 5.0e-4 / 33.2464)
    return p


def cfg_disc(nc, np_, dt, steps, navg, cg_tol=1e-12, cg_max_iter=20000):
    return {"nc": (nc, nc, nc), "np": int(np_), "dt": float(dt), "steps": int(steps),
            "navg": int(navg), "cg_tol": float(cg_tol), "cg_max_iter": int(cg_max_iter)}


# The five throughput configurations.
CONFIGS = {
    # 8^3, 16,384 particles (32 per cell), one-way: particles feel E, q = 0 in the
    # Poisson source; hard-sphere NTC with 4 averaged outcomes; dt 1e-3, 10 steps.
    "cfg0": {"problem": cfg_problem(two_way=False, collisions=True),
             "disc": cfg_disc(8, 16384, 1e-3, 10, 4), "precision": "fp64", "seed": 1},
    # 32^3, 1,048,576 particles, two-way, no collisions; dt 5e-4, 100 steps.
    "cfg1": {"problem": cfg_problem(two_way=True, collisions=False),
             "disc": cfg_disc(32, 1 << 20, 5e-4, 100, 1), "precision": "fp64", "seed": 1},
    # 64^3, 8,388,608 particles, two-way + hard-sphere NTC, 16 outcomes; 2.5e-4, 100 steps.
    "cfg2": {"problem": cfg_problem(two_way=True, collisions=True),
             "disc": cfg_disc(64, 1 << 23, 2.5e-4, 100, 16), "precision": "fp64", "seed": 1},
    # Mixed-precision form of cfg2.
    "cfg3": {"problem": cfg_problem(two_way=True, collisions=True),
             "disc": cfg_disc(64, 1 << 23, 2.5e-4, 100, 16), "precision": "mixed", "seed": 1},
    # cfg3 without collisions (the collisionless case of the paper's studies):
    # what the particle pass costs without its two collision calls.
    "cfg3_collisionless": {"problem": cfg_problem(two_way=True, collisions=False),
                           "disc": cfg_disc(64, 1 << 23, 2.5e-4, 100, 16), "precision": "mixed",
                           "seed": 1},
    # The single-simulation point at 128^3: 67,108,864 particles (32 per cell),
    # the cfg3 physics with dt halved.
    "cfg3_128": {"problem": cfg_problem(two_way=True, collisions=True),
                 "disc": cfg_disc(128, 1 << 26, 1.25e-4, 100, 16), "precision": "mixed", "seed": 1},
}


def _paper_64(precision):
    """The paper's own functions and SI constants (Sec. 5.2, L = 1.5 m, T =
    L / (10 vbar)) at the throughput size: 64^3 cells, 8,388,608 particles,
    fully coupled and collisional, dt = T / 64 (Table 1's T / dt = N_cell),
    16 averaged outcomes.  Every drift solves the manufactured positions
    (eq. mms_sol) by FP64 roots."""
    n = 64
    return {"problem": paper_problem(collisions=True),
            "disc": {"nc": (n, n, n), "np": 1 << 23, "dt": T_PAPER / n, "steps": n, "navg": 16,
                     "cg_tol": 1e-12, "cg_max_iter": 20000},
            "precision": precision, "seed": 1}


CONFIGS["cfg2_paper"] = _paper_64("fp64")
CONFIGS["cfg3_paper"] = _paper_64("mixed")


def ensemble_levels(n_levels=5):
    """Refinement ensemble: mesh 8^3 .. 128^3, 8 particles per cell, dt halved
    per level at a fixed end time 0.01, two-way + hard-sphere NTC, 16 outcomes."""
    out = []
    for lvl in range(n_levels):
        nc = 8 << lvl
        out.append({"problem": cfg_problem(two_way=True, collisions=True),
                    "disc": cfg_disc(nc, 8 * nc**3, 1e-3 / 2**lvl, 10 * 2**lvl, 16)})
    return out


def order_ladder(levels=(0, 1, 2, 3), two_way=False, collisions=False, navg=1):
    """Refinement ladder for observed orders: the ensemble sizing (mesh 8^3 * 2^l,
    8 particles per cell, dt 1e-3 / 2^l, 10 * 2^l steps to t = 0.01).  One-way
    and collisionless by default, where every error source is O(h^2) and
    O(dt^2) and the particle count adds no noise (the field solve sees only
    the manufactured source)."""
    out = []
    for lvl in levels:
        nc = 8 << lvl
        out.append({"level": lvl,
                    "problem": cfg_problem(two_way=two_way, collisions=collisions),
                    "disc": cfg_disc(nc, 8 * nc**3, 1e-3 / 2**lvl, 10 * 2**lvl, navg)})
    return out


def observed_orders(norms):
    """log2 ratios of successive error norms (h halves per level)."""
    import math
    return [[math.log2(a / b) if a > 0 and b > 0 else float("nan") for a, b in zip(n0, n1)]
            for n0, n1 in zip(norms, norms[1:])]


def get(name: str) -> dict:
    return copy.deepcopy(CONFIGS[name])
