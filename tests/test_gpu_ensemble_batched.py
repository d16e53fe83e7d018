"""Ensembles as one context (pic_ensemble_init): the members of a refinement
level run together, one launch per stage for all of them (members along the
grid's z dimension).  Each member must equal, bit for bit, the single
simulation with its replicate (Sec. 4.3 replicates are independent Philox
streams: key (seed, replicate)), in both precision forms, with the Poisson
solver of all members in one launch and with one launch per member."""
import numpy as np
import pytest

from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ITEMS = ("STATE_X", "STATE_V", "STATE_ID", "STATE_CELL_START", "STATE_PHI", "STATE_RHO")


def _pic():
    from paper_2602_15130_amd import pic
    return pic


def _run_and_compare(P, prob, disc, precision, members, first, steps, seed=3):
    with P.Ensemble(prob, disc, seed, first, members, precision) as ens:
        singles = [P.Sim(prob, disc, seed, first + m, precision) for m in range(members)]
        for m in range(members):
            for name in ITEMS:
                item = getattr(P, name)
                np.testing.assert_array_equal(ens.get(m, item), singles[m].get(item),
                                              err_msg=f"init member {m} {name}")
        ens.step(steps)
        for s in singles:
            s.step(steps)
        e = ens.errors()
        acc = 0
        for m, s in enumerate(singles):
            for name in ITEMS:
                item = getattr(P, name)
                np.testing.assert_array_equal(ens.get(m, item), s.get(item),
                                              err_msg=f"{precision} member {m} {name}")
            es = s.errors()
            np.testing.assert_array_equal(e["l2"][m], es["l2"])
            np.testing.assert_array_equal(e["linf"][m], es["linf"])
            acc += s.stats()["n_accepted"]
            s.close()
        st = ens.stats()
        assert st["n_accepted"] == acc > 0 and st["step"] == steps
        assert not np.array_equal(e["l2"][0], e["l2"][1])  # independent replicates
        return st


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_members_equal_single_simulations(level, precision):
    """8^3 and 16^3 levels of the refinement ensemble (8 particles per cell,
    two-way, hard-sphere NTC with 16 outcomes), three members, replicates
    2..4, three steps."""
    P = _pic()
    L = W.ensemble_levels(level + 1)[level]
    st = _run_and_compare(P, L["problem"], L["disc"], precision, 3, 2, 3)
    assert st["cg_members_per_launch"] in (1, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_members_with_one_solver_launch_each(precision, monkeypatch):
    P = _pic()
    monkeypatch.setenv("PIC_CG_MEMBER_LAUNCHES", "1")
    L = W.ensemble_levels(2)[1]
    st = _run_and_compare(P, L["problem"], L["disc"], precision, 2, 5, 2)
    assert st["cg_members_per_launch"] == 1


def test_single_member_and_single_only_calls():
    P = _pic()
    L = W.ensemble_levels(1)[0]
    prob, disc = L["problem"], L["disc"]
    with P.Ensemble(prob, disc, 7, 0, 1, "fp64") as ens, P.Sim(prob, disc, 7, 0, "fp64") as s:
        ens.step(2)
        s.step(2)
        for name in ITEMS:
            item = getattr(P, name)
            np.testing.assert_array_equal(ens.get(0, item), s.get(item))
    with P.Ensemble(prob, disc, 7, 0, 2, "mixed") as ens:
        for call in (lambda: P.pic_errors(ens.ctx), lambda: P.pic_angle_log(ens.ctx, 0, 0)):
            with pytest.raises(P.PicError) as ei:
                call()
            assert ei.value.code == P.PIC_EINVAL
        with pytest.raises(P.PicError) as ei:
            ens.get(2, P.STATE_X)
        assert ei.value.code == P.PIC_EINVAL


@pytest.mark.parametrize("members", [1, 3])
def test_plain_solver_launch_is_bitwise_equal(members, monkeypatch):
    """PIC_CG_PLAIN_LAUNCH=1 launches the solver ordinarily (for profiling
    runs): same results bit for bit, no barrier time-out raised."""
    P = _pic()
    L = W.ensemble_levels(2)[1]
    prob, disc = L["problem"], L["disc"]
    with P.Ensemble(prob, disc, 3, 0, members, "mixed") as a:
        a.step(3)
        ref = [[a.get(m, getattr(P, n)) for n in ITEMS] for m in range(members)]
    monkeypatch.setenv("PIC_CG_PLAIN_LAUNCH", "1")
    with P.Ensemble(prob, disc, 3, 0, members, "mixed") as b:
        b.step(3)
        assert b.stats()["step"] == 3  # pic_stats reads the flags: no barrier time-out
        for m in range(members):
            for n, r in zip(ITEMS, ref[m]):
                np.testing.assert_array_equal(b.get(m, getattr(P, n)), r, err_msg=f"{m} {n}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paper_family_members_equal_single_simulations(precision):
    """The paper's own functions (Sec. 5.2, Table 1 level 1, coupled and
    collisional): each member's drift term comes from the drift-term kernel
    launched for all members at once; members equal the single simulations
    bit for bit."""
    P = _pic()
    prob = W.paper_problem(collisions=True)
    disc = W.paper_level(1)
    _run_and_compare(P, prob, disc, precision, 2, 1, 3)
