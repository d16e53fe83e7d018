"""Mixed-precision form (FP32 particle stages, FP64 roots / CG / norms) against
the FP64 oracle.

Bars, per quantity:
  * candidate pair lists (cell, call, outcome, pair, p, q) and cell starts at a
    common state: bit-exact (N_pairs is FP64 and index selection is integer);
  * accept decisions: FP32 ratio vs FP64 ratio can flip only on near-ties
    |U - sigma g / (sigma g)_max| < ~1e-6; at most a couple per case;
  * positions: 1e-5 h, velocities: 1e-5 vbar per step taken, for particles not
    touched by a flipped accept or a flipped cell (those are counted and must be
    rare);
  * phi and rho: 1e-6 relative; error norms: 1e-3 relative.
Comparisons are by particle identity because a cell flip changes the order.
"""
import numpy as np
import pytest

import oracle as O
from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pic():
    from paper_2602_15130_amd import pic
    return pic


def _by_id(ids, arr):
    out = np.empty_like(arr)
    out[..., ids] = arr
    return out


def _pair(prob, disc, seed=1, rep=0):
    P = _pic()
    g = P.Sim(prob, disc, seed, rep, "mixed")
    o = O.Sim(prob, disc, seed, rep)
    assert o.init() == 0
    return P, g, o


def _compare(P, g, o, prob, disc, steps, max_outliers=4, tag=""):
    h = prob["L"][0] / disc["nc"][0]
    ig, io = g.get(P.STATE_ID), o.get(o.ID)
    xg, xo = _by_id(ig, g.get(P.STATE_X)), _by_id(io, o.get(o.X))
    vg, vo = _by_id(ig, g.get(P.STATE_V)), _by_id(io, o.get(o.V))
    dx = np.abs(xg - xo)
    dx = np.minimum(dx, prob["L"][0] - dx).max(axis=0)
    dv = np.abs(vg - vo).max(axis=0)
    tol_x, tol_v = 1e-5 * h * max(1, steps), 1e-5 * prob["vbar"] * max(1, steps)
    bad = (dx > tol_x) | (dv > tol_v)
    assert bad.sum() <= max_outliers, f"{tag}: {bad.sum()} particles beyond tolerance " \
        f"(max dx/h {dx.max() / h:.2e}, max dv {dv.max():.2e})"
    good = ~bad
    assert dx[good].max() <= tol_x and dv[good].max() <= tol_v
    return dx.max() / h, dv[good].max()


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

    def srt(a):
        a = np.asarray(a, dtype=np.int64).reshape(-1, 7)
        return a[np.lexsort((a[:, 3], a[:, 2], a[:, 1], a[:, 0]))]

    a, b = srt(pg), srt(po)
    np.testing.assert_array_equal(a[:, :6], b[:, :6])
    flips = int((a[:, 6] != b[:, 6]).sum())
    assert flips <= 2
    if flips == 0:
        assert np.abs(dg - do).max() < 1e-5
    assert np.abs(sg - so).max() < 1e-5 * np.abs(so).max()


def test_mixed_steps_cfg0():
    c = W.get("cfg0")
    P, g, o = _pair(c["problem"], c["disc"])
    for s in range(1, 11):
        g.step(1)
        o.step(1)
        if s in (1, 4, 10):
            _compare(P, g, o, c["problem"], c["disc"], s, tag=f"step {s}")
    eg, eo = g.errors(), o.errors()
    np.testing.assert_allclose(eg["l2"], eo["l2"], rtol=1e-3)
    pg, po = g.get(P.STATE_PHI), o.get(o.PHI)
    assert np.abs(pg - po).max() < 1e-6 * np.abs(po).max()


def test_mixed_steps_two_way_collisional():
    prob = W.cfg_problem(two_way=True, collisionality=20.0)
    disc = W.cfg_disc(8, 12000, 2e-3, 1, 6, cg_tol=1e-13)
    P, g, o = _pair(prob, disc, seed=11)
    g.step(4)
    o.step(4)
    _compare(P, g, o, prob, disc, 4, tag="two-way")
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
    g.step(2)
    o.step(2)
    _compare(P, g, o, prob, disc, 2, tag="large cells")


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
