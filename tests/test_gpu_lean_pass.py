"""The lean fused-pass instance and the general one: with PIC_LEAN_PASS=1 the
library runs the lean instance over all tiles and the general instance over
the tiles it defers (an outcome over the lane-run size, a full record pool, an
overflowing event list, a tile larger than its LDS slots); with
PIC_LEAN_PASS=0 the general instance runs alone.  Both give the same state bit
for bit, in both precision forms, for light, moderate and heavy collision
loads, large cells and ensembles; and the mixed instances that sort long event
lists equal those that scan them."""
import numpy as np
import pytest

from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ITEMS = ("STATE_X", "STATE_V", "STATE_ID", "STATE_CELL_START", "STATE_PHI")


def _pic():
    from paper_2602_15130_amd import pic
    return pic


def _run(monkeypatch, lean, prob, disc, precision, steps, members=None):
    P = _pic()
    monkeypatch.setenv("PIC_LEAN_PASS", "1" if lean else "0")
    if members:
        with P.Ensemble(prob, disc, 5, 0, members, precision) as e:
            e.step(steps)
            return [[e.get(m, getattr(P, n)) for n in ITEMS] for m in range(members)], \
                e.stats()["n_accepted"]
    with P.Sim(prob, disc, 5, 0, precision) as g:
        g.step(steps)
        return [[g.get(getattr(P, n)) for n in ITEMS]], g.stats()["n_accepted"]


CASES = {
    "light": (dict(two_way=True, collisionality=1.0), (8, 16384, 8)),
    "moderate": (dict(two_way=True, collisionality=2.0), (8, 16384, 8)),
    "heavy": (dict(two_way=True, collisionality=30.0), (8, 16384, 8)),
    "large_cells": (dict(two_way=True, collisionality=2.0), (3, 19000, 4)),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(CASES))
def test_lean_and_general_pass_agree(case, precision, monkeypatch):
    pk, (nc, npart, navg) = CASES[case]
    prob = W.cfg_problem(**pk)
    disc = W.cfg_disc(nc, npart, 1e-3, 1, navg, cg_tol=1e-13)
    a, na = _run(monkeypatch, True, prob, disc, precision, 4)
    b, nb = _run(monkeypatch, False, prob, disc, precision, 4)
    assert na == nb > 0
    for n, x, y in zip(ITEMS, a[0], b[0]):
        np.testing.assert_array_equal(x, y, err_msg=f"{case} {precision} {n}")


def test_lean_and_general_pass_agree_in_ensembles(monkeypatch):
    prob = W.cfg_problem(two_way=True, collisionality=2.0)
    disc = W.cfg_disc(8, 16384, 1e-3, 1, 8, cg_tol=1e-13)
    a, na = _run(monkeypatch, True, prob, disc, "mixed", 3, members=3)
    b, nb = _run(monkeypatch, False, prob, disc, "mixed", 3, members=3)
    assert na == nb > 0
    for m in range(3):
        for n, x, y in zip(ITEMS, a[m], b[m]):
            np.testing.assert_array_equal(x, y, err_msg=f"member {m} {n}")


@pytest.mark.parametrize("lean", [True, False])
@pytest.mark.parametrize("case", ["moderate", "heavy", "large_cells"])
def test_sorted_event_lists_change_no_bit(case, lean, monkeypatch):
    """The mixed instances that sort long event lists for the cell threads
    (PIC_SORT_EVENTS=1) and those that scan them (=0) give the same state bit
    for bit: the sort only changes how a cell thread finds its outcomes, not
    their order."""
    pk, (nc, npart, navg) = CASES[case]
    prob = W.cfg_problem(**pk)
    disc = W.cfg_disc(nc, npart, 1e-3, 1, navg, cg_tol=1e-13)
    out = {}
    for srt in ("1", "0"):
        monkeypatch.setenv("PIC_SORT_EVENTS", srt)
        out[srt] = _run(monkeypatch, lean, prob, disc, "mixed", 4)
    (a, na), (b, nb) = out["1"], out["0"]
    assert na == nb > 0
    for n, x, y in zip(ITEMS, a[0], b[0]):
        np.testing.assert_array_equal(x, y, err_msg=f"{case} lean={lean} {n}")
