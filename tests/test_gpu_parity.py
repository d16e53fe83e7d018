"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work (cell sort, particle order, cell starts, candidate pairs, accept
decisions) must match bit for bit.  FP64 floating point must agree to 1e-12
relative to the natural scale of each quantity (L for positions, the largest
|v| for velocities, max |phi| for the potential), except where the Poisson CG
bounds the agreement: two CG runs stopped at relative residual tol differ by at
most about kappa * tol in phi, kappa = 3 / sin^2(pi / n) for the periodic
7-point operator, so those cases use tol 1e-13 and state the bound.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pic():
    from paper_2602_15130_amd import pic
    return pic


def _pair(prob, disc, seed=1, rep=0, precision="fp64"):
    P = _pic()
    g = P.Sim(prob, disc, seed, rep, precision)
    o = O.Sim(prob, disc, seed, rep)
    assert o.init() == 0
    return P, g, o


def _rel(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / scale


def _kappa(nc):
    return 3.0 / math.sin(math.pi / max(nc)) ** 2


def _compare_state(P, g, o, prob, disc, phi_tol=1e-12, xv_tol=1e-12, tag=""):
    L = max(prob["L"])
    np.testing.assert_array_equal(g.get(P.STATE_ID), o.get(o.ID), err_msg=f"particle order {tag}")
    np.testing.assert_array_equal(g.get(P.STATE_CELL_START), o.get(o.CELL_START),
                                  err_msg=f"cell starts {tag}")
    xg, xo = g.get(P.STATE_X), o.get(o.X)
    vg, vo = g.get(P.STATE_V), o.get(o.V)
    vs = max(np.abs(vo).max(), prob["vbar"])
    assert _rel(xg, xo, L) < xv_tol, f"x {tag}: {_rel(xg, xo, L)}"
    assert _rel(vg, vo, vs) < xv_tol, f"v {tag}: {_rel(vg, vo, vs)}"
    rg, ro = g.get(P.STATE_RHO), o.get(o.RHO)
    assert _rel(rg, ro, np.abs(ro).max()) < 1e-12, f"rho {tag}"
    pg, po = g.get(P.STATE_PHI), o.get(o.PHI)
    assert _rel(pg, po, np.abs(po).max()) < phi_tol, f"phi {tag}: {_rel(pg, po, np.abs(po).max())}"
    eg, eo = g.get(P.STATE_E), o.get(o.E)
    assert _rel(eg, eo, np.abs(eo).max()) < phi_tol * 10, f"E {tag}"


def _small(nc, np_, dt, navg, two_way=True, collisions=True, tol=1e-13, **kw):
    prob = W.cfg_problem(two_way=two_way, collisions=collisions, **kw)
    disc = W.cfg_disc(nc, np_, dt, 1, navg, cg_tol=tol)
    return prob, disc


# ----------------------------------------------------------------------------- init
def test_init_parity_cfg0():
    c = W.get("cfg0")
    P, g, o = _pair(c["problem"], c["disc"])
    _compare_state(P, g, o, c["problem"], c["disc"], tag="init")
    e = g.errors()
    assert np.all(e["l2"][:6] == 0) and np.all(e["linf"][:6] == 0)
    eo = o.errors()
    np.testing.assert_allclose(e["l2"][6], eo["l2"][6], rtol=1e-12)


@pytest.mark.parametrize("np_", [1, 2, 255, 257, 5000])
def test_init_parity_ragged_and_sparse(np_):
    # ragged particle counts, many empty cells and single-particle cells
    prob, disc = _small(8, np_, 1e-3, 2)
    P, g, o = _pair(prob, disc, seed=7)
    _compare_state(P, g, o, prob, disc, phi_tol=_kappa(disc["nc"]) * 1e-13, tag=f"np={np_}")


def test_init_parity_non_cubic_mesh():
    prob = W.cfg_problem()
    prob["L"] = (1.0, 0.75, 1.25)
    disc = {"nc": (5, 7, 9), "np": 3000, "dt": 1e-3, "navg": 3, "cg_tol": 1e-13,
            "cg_max_iter": 5000, "steps": 1}
    P, g, o = _pair(prob, disc, seed=3)
    _compare_state(P, g, o, prob, disc, phi_tol=_kappa(disc["nc"]) * 1e-13, tag="non-cubic")


# ----------------------------------------------------------------------------- steps
def test_steps_parity_cfg0_full_run():
    """cfg0 (8^3, 16,384 particles, one-way, hard-sphere NTC, N_avg = 4), all 10 steps."""
    c = W.get("cfg0")
    P, g, o = _pair(c["problem"], c["disc"])
    for s in range(c["disc"]["steps"]):
        g.step(1)
        assert o.step(1) == 0
        _compare_state(P, g, o, c["problem"], c["disc"], tag=f"step {s + 1}")
    sg, eo = g.stats(), o.errors()
    assert sg["n_accepted"] == o.accepted and sg["n_gmax"] == o.gmax_events
    e = g.errors()
    np.testing.assert_allclose(e["l2"], eo["l2"], rtol=1e-9)
    np.testing.assert_allclose(e["linf"], eo["linf"], rtol=1e-9)


def test_steps_parity_two_way_collisional():
    prob, disc = _small(8, 12000, 2e-3, 6, two_way=True, collisions=True, collisionality=20.0)
    P, g, o = _pair(prob, disc, seed=11)
    tol = _kappa(disc["nc"]) * 1e-13
    for s in range(4):
        g.step(1)
        o.step(1)
        _compare_state(P, g, o, prob, disc, phi_tol=tol, xv_tol=1e-11, tag=f"step {s + 1}")
    assert g.stats()["n_accepted"] == o.accepted > 0


def test_steps_parity_paper_family_collisional():
    """Sec. 5.2 functions, polynomial cross section, Table 1 level-1 mesh and
    time step with a reduced particle count."""
    prob = W.paper_problem(collisions=True)
    disc = dict(W.paper_level(1, cg_tol=1e-13))
    disc["np"] = 6000
    disc["navg"] = 8
    P, g, o = _pair(prob, disc, seed=2)
    tol = _kappa(disc["nc"]) * 1e-13
    for s in range(3):
        g.step(1)
        o.step(1)
        _compare_state(P, g, o, prob, disc, phi_tol=tol, xv_tol=1e-11, tag=f"paper step {s + 1}")
    eg, eo = g.errors(), o.errors()
    np.testing.assert_allclose(eg["l2"], eo["l2"], rtol=1e-7)


def test_isolation_mode_gpu_matches_manufactured_trajectory():
    prob = W.paper_problem(collisions=False, field_to_particles=False, particles_to_field=False,
                           isolate=True)
    disc = dict(W.paper_level(1, collisions=False))
    disc["np"] = 3000
    P = _pic()
    g = P.Sim(prob, disc, 5, 0)
    g.step(4)
    e = g.errors()
    assert e["linf"][:3].max() < 5e-15 * W.L_PAPER
    assert e["linf"][3:6].max() < 5e-14 * W.VBAR


# ----------------------------------------------------------------------------- collisions
def _pairs_sorted(arr):
    a = np.asarray(arr, dtype=np.int64).reshape(-1, 7)
    order = np.lexsort((a[:, 3], a[:, 2], a[:, 1], a[:, 0]))
    return a[order]


@pytest.mark.parametrize("call", [0, 1])
def test_collide_parity_and_pair_list(call):
    prob, disc = _small(8, 16384, 1e-3, 4, collisionality=30.0)
    P, g, o = _pair(prob, disc, seed=4)
    cap = 400000
    dg, sg, pg, ng = g.collide(call, 0.0, pairlog_cap=cap)
    do, so, po, no, st = o.collide(call, 0.0, log_cap=cap)
    assert ng == no and ng > 1000
    np.testing.assert_array_equal(_pairs_sorted(pg), _pairs_sorted(po))
    scale = np.abs(o.get(o.V)).max()
    assert _rel(dg, do, scale) < 1e-12
    assert _rel(sg, so, np.abs(so).max()) < 1e-12


def test_collide_momentum_conserved_per_cell():
    prob, disc = _small(8, 16384, 1e-3, 4, collisionality=30.0)
    P = _pic()
    g = P.Sim(prob, disc, 9, 0)
    dv, _, _, _ = g.collide(0, 0.0)
    cs = g.get(P.STATE_CELL_START)
    sums = np.add.reduceat(dv, cs[:-1], axis=1)[:, np.diff(cs) > 0]
    assert np.abs(sums).max() < 1e-13


def test_deterministic_rerun():
    prob, disc = _small(8, 9000, 2e-3, 4, collisionality=20.0)
    P = _pic()
    a = P.Sim(prob, disc, 21, 3)
    b = P.Sim(prob, disc, 21, 3)
    a.step(3)
    b.step(3)
    for item in (P.STATE_X, P.STATE_V, P.STATE_ID, P.STATE_PHI):
        np.testing.assert_array_equal(a.get(item), b.get(item))


# ----------------------------------------------------------------------------- errors
def test_error_norms_parity_after_steps():
    prob, disc = _small(8, 8000, 2e-3, 3, collisionality=10.0)
    P, g, o = _pair(prob, disc, seed=13)
    g.step(3)
    o.step(3)
    eg, eo = g.errors(), o.errors()
    np.testing.assert_allclose(eg["l2"], eo["l2"], rtol=1e-9)
    np.testing.assert_allclose(eg["linf"], eo["linf"], rtol=1e-9)


def test_cg_nonconvergence_reported():
    prob, disc = _small(8, 4000, 1e-3, 1, collisions=False)
    disc["cg_max_iter"] = 1
    P = _pic()
    with pytest.raises(P.PicError) as ei:
        g = P.Sim(prob, disc, 1, 0)
        g.stats()
    assert ei.value.code == P.PIC_ENOCONV


# ----------------------------------------------------------------------------- full size
def test_full_size_cfg2_properties_and_samples():
    """cfg2 at full size (64^3, 8,388,608 particles, N_avg = 16): properties that
    hold at any size, and sampled particles/cells against the oracle."""
    c = W.get("cfg2")
    prob, disc = c["problem"], c["disc"]
    P = _pic()
    g = P.Sim(prob, disc, c["seed"], 0)
    g.step(1)
    cs = g.get(P.STATE_CELL_START)
    ids = g.get(P.STATE_ID)
    x = g.get(P.STATE_X)
    v = g.get(P.STATE_V)
    assert cs[0] == 0 and cs[-1] == disc["np"] and np.all(np.diff(cs) >= 0)
    assert np.array_equal(np.sort(ids), np.arange(disc["np"]))
    keys = O.cell_keys(prob, disc, x)
    assert np.all(np.diff(keys) >= 0)
    np.testing.assert_array_equal(cs, np.concatenate([[0], np.cumsum(np.bincount(keys, minlength=64**3))]))
    rho = g.get(P.STATE_RHO)
    assert rho.sum() * (1 / 64) ** 3 == pytest.approx(prob["q"] * prob["nphys"], rel=1e-12)
    # sampled cells: the oracle's Algorithm 1 on the same cell velocities
    dv, src, _, _ = g.collide(0, g.stats()["step"] * disc["dt"])
    rng = np.random.default_rng(0)
    for cell in rng.choice(64**3, size=24, replace=False):
        s, e = cs[cell], cs[cell + 1]
        do, _, _, _ = O.collide_cell(prob, disc, c["seed"], 0, 1, 0, int(cell), v[:, s:e])
        assert _rel(dv[:, s:e], do, max(1.0, np.abs(v[:, s:e]).max())) < 1e-12
    # sampled particles: manufactured velocity from the particle identity
    for i in rng.choice(disc["np"], size=32, replace=False):
        xi = O.init_uniforms(c["seed"], 0, int(ids[i]))
        vm = O.vM(prob, xi[3:], 0.0)
        # one step moved v by field, collisions and source only: stays near v^M
        assert np.abs(v[:, i] - vm).max() < 1.0


# ----------------------------------------------------------------------------- fused pass
def _run_path(prob, disc, unfused, steps, seed=5):
    import os
    P = _pic()
    old = os.environ.get("PIC_UNFUSED")
    os.environ["PIC_UNFUSED"] = "1" if unfused else "0"
    try:
        g = P.Sim(prob, disc, seed, 1)
    finally:
        if old is None:
            os.environ.pop("PIC_UNFUSED")
        else:
            os.environ["PIC_UNFUSED"] = old
    for n in steps:
        g.step(n)
    return P, g


@pytest.mark.parametrize("case", ["cfg0", "dense", "paper"])
def test_fused_pass_is_bitwise_equal_to_unfused(case):
    """The fused particle pass (call B, kick 2, call A, kick 1, drift per
    cell-aligned tile) performs the same operations in the same order as the
    separate kernels, so the two paths agree bit for bit, including when
    pic_step is called with different step counts."""
    if case == "cfg0":
        c = W.get("cfg0")
        prob, disc = c["problem"], c["disc"]
    elif case == "dense":  # most (cell, outcome) lanes have pairs: the event list overflows
        prob, disc = _small(8, 16384, 2e-3, 128, collisionality=5.0)
    else:
        prob = W.paper_problem(collisions=True)
        disc = dict(W.paper_level(1, cg_tol=1e-13))
        disc["np"] = 6000
        disc["navg"] = 8
    P, a = _run_path(prob, disc, False, [1, 3, 2])
    _, b = _run_path(prob, disc, True, [1, 3, 2])
    for item in (P.STATE_X, P.STATE_V, P.STATE_ID, P.STATE_CELL_START, P.STATE_PHI):
        np.testing.assert_array_equal(a.get(item), b.get(item))
    assert a.stats()["n_accepted"] == b.stats()["n_accepted"]


def test_fused_pass_large_cells_use_global_scratch():
    """Cells larger than the LDS tile (here ~700 particles per cell) take the
    global-memory path of the same kernel; parity with the oracle holds."""
    prob, disc = _small(3, 19000, 1e-3, 3, collisionality=2.0)
    P, g, o = _pair(prob, disc, seed=8)
    for s in range(2):
        g.step(1)
        o.step(1)
        _compare_state(P, g, o, prob, disc, phi_tol=_kappa(disc["nc"]) * 1e-13, xv_tol=1e-11,
                       tag=f"large cells step {s + 1}")


# ----------------------------------------------------------------------------- Poisson solvers
def _with_env(name, value, fn):
    import os
    old = os.environ.get(name)
    os.environ[name] = value
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop(name)
        else:
            os.environ[name] = old


@pytest.mark.parametrize("n,blocks", [(16, 0), (32, 0), (32, 16), (64, 0), (128, 0)])
def test_brick_solver_matches_global_solver_and_oracle(n, blocks):
    """The on-chip brick CG and the global-memory CG run the same recurrence
    and differ only in the order of the block partial sums; both stop at
    ||r|| <= tol ||b||, so phi agrees within kappa * tol, and with the oracle.
    Covers few bricks (16^3), bricks of 2048 nodes (blocks=16) and the
    512- or 1024-thread instances (128^3).  (A brick's xy face holds one
    workgroup's threads, so meshes below 16 x 16 use the global solver.)"""
    prob = W.cfg_problem(two_way=True, collisions=False)
    disc = W.cfg_disc(n, 32 * n**3 if n <= 32 else 2 * n**3, 5e-4, 1, 1, cg_tol=1e-13)
    P = _pic()
    mk = lambda: P.Sim(prob, disc, 3, 0)  # noqa: E731
    g = _with_env("PIC_CG_BLOCKS", str(blocks), mk) if blocks else mk()
    st = g.stats()
    assert st["cg_brick"][0] > 0, f"brick solver not selected for {n}^3: {st}"
    h = _with_env("PIC_CG_GLOBAL", "1", mk)
    assert h.stats()["cg_brick"] == [0, 0, 0]
    pg, ph = g.get(P.STATE_PHI), h.get(P.STATE_PHI)
    kap = _kappa(disc["nc"])
    assert _rel(pg, ph, np.abs(ph).max()) < kap * 1e-13
    assert abs(st["cg_iters"] - h.stats()["cg_iters"]) <= 1
    g.step(2)
    h.step(2)
    pg, ph = g.get(P.STATE_PHI), h.get(P.STATE_PHI)
    assert _rel(pg, ph, np.abs(ph).max()) < kap * 1e-13
    if n <= 16:
        o = O.Sim(prob, disc, 3, 0)
        assert o.init() == 0
        o.step(2)
        po = o.get(o.PHI)
        assert _rel(pg, po, np.abs(po).max()) < kap * 1e-13


@pytest.mark.parametrize("nc", [(16, 16, 16), (12, 10, 14), (64, 64, 64)])
def test_lowmode_presolve_matches_plain_cg(nc):
    """The exact low-Fourier-mode solve before the CG changes only the initial
    guess: both runs stop at ||r|| <= tol ||b||, so phi agrees within kappa * tol,
    and the pre-solve needs fewer iterations."""
    prob = W.cfg_problem(two_way=True, collisions=False)
    disc = W.cfg_disc(nc[0], 8 * nc[0] * nc[1] * nc[2], 5e-4, 1, 1, cg_tol=1e-13)
    disc["nc"] = nc
    P = _pic()
    mk = lambda: P.Sim(prob, disc, 5, 0)  # noqa: E731
    g = mk()
    h = _with_env("PIC_CG_LOWMODES", "0", mk)
    kap = _kappa(nc)
    for _ in range(2):
        pg, ph = g.get(P.STATE_PHI), h.get(P.STATE_PHI)
        assert _rel(pg, ph, np.abs(ph).max()) < kap * 1e-13
        assert g.stats()["cg_iters"] < h.stats()["cg_iters"]
        g.step(1)
        h.step(1)
    if nc[0] <= 16:
        o = O.Sim(prob, disc, 5, 0)
        assert o.init() == 0
        o.step(2)
        po = o.get(o.PHI)
        assert _rel(g.get(P.STATE_PHI), po, np.abs(po).max()) < kap * 1e-13


# ----------------------------------------------------------------------------- trilinear elements
@pytest.mark.parametrize("nc", [(16, 16, 16), (12, 10, 14)])
def test_q1_field_discretization_matches_oracle(nc):
    """poisson_op = 1 (trilinear elements, Sec. 4.2): the FP64 state after
    initialisation and two coupled steps (positions, velocities, rho, phi, E)
    matches the oracle's Q1 run; phi differs from the 7-point run by the
    discretization (O(h^2)), and the low-mode pre-solve with the Q1 eigenvalues
    only changes the initial guess."""
    prob = W.cfg_problem(two_way=True, collisions=True)
    disc = W.cfg_disc(nc[0], 8 * nc[0] * nc[1] * nc[2], 5e-4, 2, 4, cg_tol=1e-13)
    disc["nc"] = nc
    disc["poisson_op"] = 1
    P = _pic()
    g = P.Sim(prob, disc, 5, 0)
    o = O.Sim(prob, disc, 5, 0)
    assert o.init() == 0
    kap = _kappa(nc)
    _compare_state(P, g, o, prob, disc, phi_tol=kap * 1e-13, tag="q1 init")
    h = _with_env("PIC_CG_LOWMODES", "0", lambda: P.Sim(prob, disc, 5, 0))
    pg, ph = g.get(P.STATE_PHI), h.get(P.STATE_PHI)
    assert _rel(pg, ph, np.abs(ph).max()) < kap * 1e-13
    assert g.stats()["cg_iters"] < h.stats()["cg_iters"]
    d7 = dict(disc)
    d7["poisson_op"] = 0
    p7 = P.Sim(prob, d7, 5, 0).get(P.STATE_PHI)
    dphi = _rel(pg, p7, np.abs(p7).max())
    assert 1e-6 < dphi < 0.2, dphi
    g.step(2)
    o.step(2)
    _compare_state(P, g, o, prob, disc, phi_tol=kap * 1e-13, xv_tol=1e-11, tag="q1 step 2")
    m = P.Sim(prob, disc, 5, 0, "mixed")
    m.step(2)
    pm = m.get(P.STATE_PHI)
    assert _rel(pm, g.get(P.STATE_PHI), np.abs(pm).max()) < 1e-4


# ----------------------------------------------------------------------------- collision-heavy regime
def test_heavy_collision_kernel_matches_serial_and_oracle():
    """Table 1 level 2 (101 particles per cell, N_avg = 243, ~6 candidate pairs
    per outcome) runs its collision calls in k_collide_heavy: its pair list is
    identical to the serial kernel's, its <dv> agrees to the fixed-point
    quantum (far below FP64 state rounding), and sampled cells agree with the
    oracle's Algorithm 1."""
    prob = W.paper_problem(collisions=True)
    disc = dict(W.paper_level(2))
    P = _pic()
    g = P.Sim(prob, disc, 1, 0)
    h = _with_env("PIC_HEAVY", "0", lambda: P.Sim(prob, disc, 1, 0))
    cap = 4_000_000
    dg, sg, lg, ng = g.collide(0, 0.0, pairlog_cap=cap)
    dh, sh, lh, nh = h.collide(0, 0.0, pairlog_cap=cap)
    assert ng == nh and 0 < ng <= cap

    def srt(a):
        a = np.asarray(a, dtype=np.int64).reshape(-1, 7)
        return a[np.lexsort((a[:, 3], a[:, 2], a[:, 1], a[:, 0]))]

    np.testing.assert_array_equal(srt(lg), srt(lh))
    scale = np.abs(g.get(P.STATE_V)).max()
    assert _rel(dg, dh, scale) < 1e-13
    np.testing.assert_array_equal(sg, sh)
    v = g.get(P.STATE_V)
    cs = g.get(P.STATE_CELL_START)
    for cell in np.random.default_rng(3).choice(12**3, size=6, replace=False):
        s, e = cs[cell], cs[cell + 1]
        do, _, _, _ = O.collide_cell(prob, disc, 1, 0, 0, 0, int(cell), v[:, s:e])
        assert _rel(dg[:, s:e], do, scale) < 1e-12
    g.step(2)
    h.step(2)
    assert _rel(g.get(P.STATE_V), h.get(P.STATE_V), scale) < 1e-11


def test_heavy_mode_big_cells_run_by_the_per_cell_kernel():
    """With a 15x time step at Table 1 level 2 (32 outcomes) the mean outcome has ~90
    candidate pairs: the paper's non-uniform density puts the dense cells past
    the workgroup kernel's capacity (192 pairs per outcome), so they run in
    k_collide_big while the rest stay in k_collide_heavy.  The combined pair
    list equals the serial kernel's, <dv> agrees (big cells bit for bit), the
    capacity flag stays down, and the densest cell and a sparse one agree with
    the oracle's Algorithm 1."""
    prob = W.paper_problem(collisions=True)
    disc = dict(W.paper_level(2))
    disc["dt"] = disc["dt"] * 15.0
    disc["navg"] = 32  # keeps the pair logs at ~5M records
    P = _pic()
    g = P.Sim(prob, disc, 1, 0)
    h = _with_env("PIC_HEAVY", "0", lambda: P.Sim(prob, disc, 1, 0))
    cap = 8_000_000
    dg, sg, lg, ng = g.collide(0, 0.0, pairlog_cap=cap)
    dh, sh, lh, nh = h.collide(0, 0.0, pairlog_cap=cap)
    assert ng == nh and 0 < ng <= cap

    def srt(a):
        a = np.asarray(a, dtype=np.int64).reshape(-1, 7)
        return a[np.lexsort((a[:, 3], a[:, 2], a[:, 1], a[:, 0]))]

    np.testing.assert_array_equal(srt(lg), srt(lh))
    cs = g.get(P.STATE_CELL_START)
    counts = np.diff(cs)
    L = W.L_PAPER
    # Algorithm 1: P_max = (sigma g)_max w dt / V_cell, w = N / N_p physical particles each
    pmax = (33.2464 * W.SIGBAR * W.VBAR) * (W.N_PAPER / disc["np"]) * disc["dt"] / (L**3 / 12**3)
    # pair bound per cell; 30 % margins keep the check off the threshold
    bound = counts * (counts - 1.0) * pmax / 2.0 + 1.0
    big, small = bound >= 1.3 * 193.0, bound <= 193.0 / 1.3
    assert big.any() and small.any()
    scale = np.abs(g.get(P.STATE_V)).max()
    assert _rel(dg, dh, scale) < 1e-13
    for cell in np.flatnonzero(big)[:3]:
        s, e = cs[cell], cs[cell + 1]
        np.testing.assert_array_equal(dg[:, s:e], dh[:, s:e])
    v = g.get(P.STATE_V)
    for cell in (int(np.argmax(counts)), int(np.argmin(np.where(counts > 1, counts, 10**9)))):
        s, e = cs[cell], cs[cell + 1]
        do, _, _, _ = O.collide_cell(prob, disc, 1, 0, 0, 0, cell, v[:, s:e])
        assert _rel(dg[:, s:e], do, scale) < 1e-12
    g.step(1)
    h.step(1)
    assert _rel(g.get(P.STATE_V), h.get(P.STATE_V), scale) < 1e-11


# ----------------------------------------------------------------------------- checkpoint
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_resume_is_bitwise(precision):
    """A context restored from a checkpoint continues exactly as the original;
    a checkpoint of another seed is refused."""
    prob, disc = _small(16, 60000, 1e-3, 4, collisionality=3.0)
    P = _pic()
    g = P.Sim(prob, disc, 4, 0, precision)
    g.step(3)
    data = g.checkpoint()
    h = P.Sim(prob, disc, 4, 0, precision)
    h.restore(data)
    g.step(2)
    h.step(2)
    for item in (P.STATE_X, P.STATE_V, P.STATE_ID, P.STATE_CELL_START, P.STATE_PHI, P.STATE_RHO):
        np.testing.assert_array_equal(g.get(item), h.get(item))
    assert g.stats()["n_accepted"] == h.stats()["n_accepted"] and h.stats()["step"] == 5
    other = P.Sim(prob, disc, 5, 0, precision)
    with pytest.raises(P.PicError) as ei:
        other.restore(data)
    assert ei.value.code == P.PIC_EINVAL


# ----------------------------------------------------------------------------- stage timing
def test_stage_timing_covers_the_chosen_stages_only():
    """pic_timing_enable times every stage of the fused step; pic_timing_stages
    times only the chosen ones (the others stay at zero launches); timing
    never changes the result."""
    prob, disc = _small(16, 60000, 1e-3, 4)
    P = _pic()
    g = P.Sim(prob, disc, 3, 0, "mixed")
    h = P.Sim(prob, disc, 3, 0, "mixed")
    g.timing(True)
    g.step(3)
    h.step(3)
    st = g.timing_read()
    for name in ("particle", "sort", "deposit", "cg", "gradient"):
        ms, n = st[name]
        assert n >= 3 and ms > 0.0, (name, st[name])
    g.timing_stages(["particle"])
    g.step(2)
    h.step(2)
    st = g.timing_read()
    assert st["particle"][1] >= 2 and st["particle"][0] > 0.0
    assert all(n == 0 for k, (ms, n) in st.items() if k != "particle"), st
    g.timing(False)
    np.testing.assert_array_equal(g.get(P.STATE_V), h.get(P.STATE_V))
