"""Captured steps (pic_use_graphs): pic_step replays two-step HIP graphs
whose kernels take the step index from a device counter.  Every replay must
equal ordinary stepping bit for bit: both precision forms, the configuration
and paper families (the mixed pass's time-dependent constants computed on the
device), ensembles, both buffer parities, repeated calls with the program's
own work between them, and the graphs dropped when the angle log switches the
pass instance."""
import numpy as np
import pytest

from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ITEMS = ("STATE_X", "STATE_V", "STATE_ID", "STATE_CELL_START", "STATE_PHI", "STATE_RHO")


def _pic():
    from paper_2602_15130_amd import pic
    return pic


def _state(P, g, member=None):
    if member is None:
        return [g.get(getattr(P, n)) for n in ITEMS]
    return [g.get(member, getattr(P, n)) for n in ITEMS]


def _equal(P, a, b, tag, members=None):
    for m in (range(members) if members else [None]):
        for n, x, y in zip(ITEMS, _state(P, a, m), _state(P, b, m)):
            np.testing.assert_array_equal(x, y, err_msg=f"{tag} {n} member {m}")


# (the paper family's manufactured solution is defined up to t = T: its
# cases stay within the level's steps, Table 1 level 1 (8 steps) for FP64,
# whose level 2 runs the collision-heavy separate kernels, level 2 (12) for
# the mixed form)
CASES = {
    "cfg_fp64": (lambda: W.cfg_problem(two_way=True, collisionality=2.0), (8, 16384, 8), "fp64",
                 (7, 5, 2, 6)),
    "cfg_mixed": (lambda: W.cfg_problem(two_way=True, collisionality=2.0), (8, 16384, 8), "mixed",
                  (7, 5, 2, 6)),
    "paper_mixed": (lambda: W.paper_problem(collisions=True), 2, "mixed", (7, 4)),
    "paper_fp64": (lambda: W.paper_problem(collisions=True), 1, "fp64", (4, 3)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_replays_equal_ordinary_steps(case):
    P = _pic()
    mk, sizes, prec, calls = CASES[case]
    prob = mk()
    if isinstance(sizes, tuple):
        disc = W.cfg_disc(sizes[0], sizes[1], 1e-3, 1, sizes[2], cg_tol=1e-13)
    else:
        disc = dict(W.paper_level(sizes, cg_tol=1e-13))
    with P.Sim(prob, disc, 3, 0, prec) as a, P.Sim(prob, disc, 3, 0, prec) as b:
        b.use_graphs(True)
        # 7: three replays; 5: two (the other parity after the odd step
        # count); 2: none; 6: two, reusing both recorded graphs
        for n in calls:
            a.step(n)
            b.step(n)
            torch.cuda.synchronize()
            _equal(P, a, b, f"{case} after {n}")
            assert a.stats()["step"] == b.stats()["step"]
            assert a.stats()["n_accepted"] == b.stats()["n_accepted"]


def test_replays_in_ensembles():
    P = _pic()
    prob = W.cfg_problem(two_way=True, collisionality=2.0)
    disc = W.cfg_disc(8, 16384, 1e-3, 1, 8, cg_tol=1e-13)
    with P.Ensemble(prob, disc, 3, 1, 3, "mixed") as a, P.Ensemble(prob, disc, 3, 1, 3, "mixed") as b:
        b.use_graphs(True)
        for n in (6, 5):
            a.step(n)
            b.step(n)
            _equal(P, a, b, f"ensemble after {n}", members=3)


def test_timing_and_angle_log_with_graphs():
    """Timed steps run ordinarily; switching the angle log on drops the
    recorded graphs (it selects the full pass instance), and the replays that
    follow still equal ordinary steps."""
    P = _pic()
    prob = W.cfg_problem(two_way=True, collisionality=2.0)
    disc = W.cfg_disc(8, 16384, 1e-3, 1, 8, cg_tol=1e-13)
    with P.Sim(prob, disc, 5, 0, "mixed") as a, P.Sim(prob, disc, 5, 0, "mixed") as b:
        b.use_graphs(True)
        a.step(6)
        b.step(6)
        b.timing(True)
        a.step(4)
        b.step(4)
        b.timing(False)
        _equal(P, a, b, "timed")
        a.angle_log(200000)
        b.angle_log(200000)
        a.step(6)
        b.step(6)
        _equal(P, a, b, "angle log")
        ea, na = a.angle_errors()
        eb, nb = b.angle_errors()
        assert na == nb > 0 and np.array_equal(ea, eb)
