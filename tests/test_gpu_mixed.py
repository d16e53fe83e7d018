"""Mixed-precision form (FP32 particle stages, FP64 roots / CG / norms) against
the FP64 oracle.

Bars, per quantity (the FP32 error model behind them is in the design notes:
the rounding of a step moves a velocity by at most ~5e-7 vbar and an offset by
~1e-7 h, so 1e-5 holds for the 10 or fewer steps these tests take):
  * candidate pair lists (cell, call, outcome, pair, p, q) and cell starts at a
    common state: bit-exact (N_pairs is FP64 and index selection is integer);
  * accept decisions: equal, except that the first differing decision of an
    outcome must be a near-tie |U - sigma g / (sigma g)_max| <= 2^-22 (the
    FP32 ratio's rounding and the 24-bit uniform);
  * positions within 1e-5 h and velocities within 1e-5 vbar for every particle
    not touched by a cell flip; a flipped particle must lie within 1e-5 h of a
    face of its oracle cell, and the particles of the cells a flip touches (and,
    step by step, of the cells those share with them) are excluded and counted;
  * phi and rho: 1e-6 relative; error norms: 1e-3 relative.
Comparisons are by particle identity because a cell flip changes the order.
"""
import numpy as np
import pytest

import oracle as O
from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from mixed_compare import TOL, Tracker, by_id as _by_id  # noqa: E402
from mixed_compare import first_flips_are_near_ties as _first_flips_are_near_ties  # noqa: E402
from mixed_compare import sorted_pairs as _sorted_pairs  # noqa: E402


def _pic():
    from paper_2602_15130_amd import pic
    return pic


def _pair(prob, disc, seed=1, rep=0):
    P = _pic()
    g = P.Sim(prob, disc, seed, rep, "mixed")
    o = O.Sim(prob, disc, seed, rep)
    assert o.init() == 0
    return P, g, o


def test_mixed_init_matches_fp64_oracle():
    c = W.get("cfg0")
    P, g, o = _pair(c["problem"], c["disc"])
    np.testing.assert_array_equal(g.get(P.STATE_ID), o.get(o.ID))
    np.testing.assert_array_equal(g.get(P.STATE_CELL_START), o.get(o.CELL_START))
    h = 1 / 8
    assert np.abs(g.get(P.STATE_X) - o.get(o.X)).max() < 1e-7 * h
    assert np.abs(g.get(P.STATE_V) - o.get(o.V)).max() < 1e-6
    rg, ro = g.get(P.STATE_RHO), o.get(o.RHO)
    assert np.abs(rg - ro).max() < 1e-6 * np.abs(ro).max()
    pg, po = g.get(P.STATE_PHI), o.get(o.PHI)
    assert np.abs(pg - po).max() < 1e-6 * np.abs(po).max()


@pytest.mark.parametrize("call", [0, 1])
def test_mixed_pair_lists_bit_exact(call):
    prob = W.cfg_problem(collisionality=30.0)
    disc = W.cfg_disc(8, 16384, 1e-3, 1, 4, cg_tol=1e-13)
    P, g, o = _pair(prob, disc, seed=4)
    cap = 400000
    dg, sg, pg, ng = g.collide(call, 0.0, pairlog_cap=cap)
    do, so, po, no, st = o.collide(call, 0.0, log_cap=cap)
    assert ng == no and ng > 1000
    a, _ = _sorted_pairs(pg)
    b, ties = _sorted_pairs(po, o.last_accept_test)
    np.testing.assert_array_equal(a[:, :6], b[:, :6])
    flips = _first_flips_are_near_ties(a, b, ties)
    # <dv> per particle within the bar, except the cells of flipped outcomes
    cs = o.get(o.CELL_START)
    flipped_cells = np.unique(b[a[:, 6] != b[:, 6], 0])
    keep = np.ones(disc["np"], dtype=bool)
    for c in flipped_cells:
        keep[cs[c]:cs[c + 1]] = False
    assert np.abs(dg - do)[:, keep].max() <= TOL * prob["vbar"]
    assert flips <= 2
    assert np.abs(sg - so).max() < 1e-5 * np.abs(so).max()


def test_mixed_steps_cfg0():
    c = W.get("cfg0")
    P, g, o = _pair(c["problem"], c["disc"])
    tr = Tracker(c["problem"], c["disc"])
    for s in range(1, 11):
        g.step(1)
        o.step(1)
        tr.check(P, g, o, tag=f"step {s}")
    eg, eo = g.errors(), o.errors()
    np.testing.assert_allclose(eg["l2"], eo["l2"], rtol=1e-3)
    pg, po = g.get(P.STATE_PHI), o.get(o.PHI)
    assert np.abs(pg - po).max() < 1e-6 * np.abs(po).max()


def test_mixed_steps_two_way_collisional():
    prob = W.cfg_problem(two_way=True, collisionality=20.0)
    disc = W.cfg_disc(8, 12000, 2e-3, 1, 6, cg_tol=1e-13)
    P, g, o = _pair(prob, disc, seed=11)
    tr = Tracker(prob, disc)
    for s in range(1, 5):
        g.step(1)
        o.step(1)
        tr.check(P, g, o, tag=f"two-way step {s}")
    rg, ro = g.get(P.STATE_RHO), o.get(o.RHO)
    assert np.abs(rg - ro).max() < 1e-5 * np.abs(ro).max()
    eg, eo = g.errors(), o.errors()
    np.testing.assert_allclose(eg["l2"], eo["l2"], rtol=1e-3)


@pytest.mark.parametrize("nc,np_", [(8, 12000), (3, 19000)])
def test_mixed_step_chunks_are_bitwise_equal(nc, np_):
    """One pic_step(6) runs passes that hold call B of a step and call A of the
    next, kick A reusing kick B's field acceleration (same time, same
    position); six pic_step(1) calls run every half as a pass of its own and
    compute it afresh.  The states agree bit for bit (3^3: tiles larger than
    their LDS slots, where nothing is kept)."""
    prob = W.cfg_problem(two_way=True, collisionality=20.0)
    disc = W.cfg_disc(nc, np_, 2e-3, 1, 6, cg_tol=1e-13)
    P = _pic()
    a = P.Sim(prob, disc, 11, 0, "mixed")
    b = P.Sim(prob, disc, 11, 0, "mixed")
    a.step(6)
    for _ in range(6):
        b.step(1)
    for item in (P.STATE_X, P.STATE_V, P.STATE_ID, P.STATE_CELL_START, P.STATE_PHI):
        np.testing.assert_array_equal(a.get(item), b.get(item))
    assert a.stats()["n_accepted"] == b.stats()["n_accepted"] > 0


def test_mixed_large_cells_global_path():
    prob = W.cfg_problem(collisionality=2.0)
    disc = W.cfg_disc(3, 19000, 1e-3, 1, 3, cg_tol=1e-13)
    P, g, o = _pair(prob, disc, seed=8)
    tr = Tracker(prob, disc)
    for s in (1, 2):
        g.step(1)
        o.step(1)
        tr.check(P, g, o, tag=f"large cells step {s}")


def test_mixed_full_size_cfg3_properties():
    c = W.get("cfg3")
    prob, disc = c["problem"], c["disc"]
    P = _pic()
    g = P.Sim(prob, disc, c["seed"], 0, "mixed")
    g.step(2)
    cs = g.get(P.STATE_CELL_START)
    ids = g.get(P.STATE_ID)
    assert cs[0] == 0 and cs[-1] == disc["np"] and np.all(np.diff(cs) >= 0)
    assert np.array_equal(np.sort(ids), np.arange(disc["np"]))
    x = g.get(P.STATE_X)
    keys = O.cell_keys(prob, disc, x)
    # positions rebuilt in FP64 from cell + offset land in their own cell
    assert np.all(np.diff(keys) >= 0)
    rho = g.get(P.STATE_RHO)
    assert rho.sum() * (1 / 64) ** 3 == pytest.approx(prob["q"] * prob["nphys"], rel=1e-6)
    e = g.errors()
    assert np.all(np.isfinite(e["l2"])) and e["l2"][0] < 1e-3


def test_mixed_full_size_cfg3_against_oracle():
    """The headline configuration (64^3, 8,388,608 particles, two-way, hard
    spheres with 16 outcomes) against the FP64 oracle at full size: the
    initial state, one collision call with its whole pair list (about 240,000
    candidate pairs), and one time step of every particle."""
    c = W.get("cfg3")
    prob, disc = c["problem"], c["disc"]
    P, g, o = _pair(prob, disc, seed=c["seed"])
    np.testing.assert_array_equal(g.get(P.STATE_CELL_START), o.get(o.CELL_START))
    np.testing.assert_array_equal(g.get(P.STATE_ID), o.get(o.ID))
    h = 1 / 64
    assert np.abs(g.get(P.STATE_X) - o.get(o.X)).max() < 2.0**-24 * h * 1.01
    cap = 1 << 20
    dg, sg, pg, ng = g.collide(0, 0.0, pairlog_cap=cap)
    do, so, po, no, st = o.collide(0, 0.0, log_cap=cap)
    assert ng == no and 100000 < ng < cap
    a, _ = _sorted_pairs(pg)
    b, ties = _sorted_pairs(po, o.last_accept_test)
    np.testing.assert_array_equal(a[:, :6], b[:, :6])
    flips = _first_flips_are_near_ties(a, b, ties)
    cs = o.get(o.CELL_START)
    keep = np.ones(disc["np"], dtype=bool)
    for cell in np.unique(b[a[:, 6] != b[:, 6], 0]):
        keep[cs[cell]:cs[cell + 1]] = False
    assert np.abs(dg - do)[:, keep].max() <= TOL
    assert np.abs(sg - so).max() <= 1e-5 * np.abs(so).max()
    g.step(1)
    o.step(1)
    Tracker(prob, disc).check(P, g, o, tag="cfg3 step 1")
    pgh, poh = g.get(P.STATE_PHI), o.get(o.PHI)
    assert np.abs(pgh - poh).max() < 1e-6 * np.abs(poh).max()
    print(f"cfg3 full size: {ng} candidate pairs, {flips} accept flips")
