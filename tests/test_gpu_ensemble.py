"""The refinement ensemble (levels 8^3 * 2^l, 8 particles per cell, dt halved
per level to t = 0.01, two-way coupling, hard-sphere NTC with 16 outcomes,
independent Philox replicates): every member against the oracle on the small
levels, the mixed form against the FP64 form member by member, the runner's
aggregation and its tuning cache, and the largest level (128^3, 16,777,216 particles) by properties
that hold at any size."""
import numpy as np
import pytest

import oracle as O
from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _levels(n):
    return W.ensemble_levels(n)


def test_members_match_oracle_on_small_levels():
    from paper_2602_15130_amd import ensemble
    for L in _levels(2):
        prob, disc = L["problem"], L["disc"]
        reps = [0, 1, 2] if disc["nc"][0] == 8 else [0, 1]
        l2, linf, _, solver = ensemble.run_level(prob, disc, "fp64", reps)
        assert solver["members_per_context"] == len(reps)
        for i, r in enumerate(reps):
            o = O.Sim(prob, disc, 1, r)
            assert o.init() == 0
            o.step(disc["steps"])
            e = o.errors()
            # the GPU solves the low Fourier modes exactly before its CG, so phi
            # differs from the oracle's by at most kappa * tol; the norms follow
            np.testing.assert_allclose(l2[i], e["l2"], rtol=1e-6, err_msg=f"level {disc['nc']} rep {r}")
            np.testing.assert_allclose(linf[i], e["linf"], rtol=1e-6)
        assert not np.allclose(l2[0], l2[1])  # replicates are independent streams


def test_mixed_members_match_fp64_members():
    from paper_2602_15130_amd import ensemble
    for L in _levels(3):
        prob, disc = L["problem"], L["disc"]
        a = ensemble.run_level(prob, disc, "fp64", [0, 1])[0]
        b = ensemble.run_level(prob, disc, "mixed", [0, 1])[0]
        np.testing.assert_allclose(b, a, rtol=2e-3)


def test_runner_aggregates_and_tunes(tmp_path, monkeypatch):
    from paper_2602_15130_amd import ensemble
    monkeypatch.setenv("PIC_TUNE_CACHE", str(tmp_path / "tune.json"))
    out = ensemble.run_ensemble(levels=_levels(3), replicates=4, precision="mixed")
    assert len(out["levels"]) == 3 and len(out["orders_l2_mean"]) == 2
    lv = out["levels"][2]
    assert lv["mesh"] == 32 and lv["tuning_from_cache"] is False
    tuned = lv["cg_tuning_ms_per_step"]
    assert set(tuned) <= set(ensemble.CG_GRID_CHOICES) and len(tuned) >= 1
    l2 = np.array(lv["l2"])
    assert l2.shape == (4, 7) and np.all(np.isfinite(l2)) and np.all(l2 > 0)
    np.testing.assert_allclose(lv["l2_mean"], l2.mean(axis=0))
    assert out["particle_steps"] == sum(x["particles"] * x["steps"] * 4 for x in out["levels"])
    # the second run takes every level's choice from the cache and gives the same norms
    again = ensemble.run_ensemble(levels=_levels(3), replicates=4, precision="mixed")
    for a, b in zip(out["levels"], again["levels"]):
        assert b["tuning_from_cache"] is True and b["cg_tuning_ms_per_step"] == a["cg_tuning_ms_per_step"]
        np.testing.assert_array_equal(np.array(a["l2"]), np.array(b["l2"]))


def test_largest_level_properties():
    from paper_2602_15130_amd import pic
    L = _levels(5)[4]
    prob, disc = L["problem"], L["disc"]
    assert disc["nc"][0] == 128 and disc["np"] == 16777216
    g = pic.Sim(prob, disc, 1, 0, "mixed")
    g.step(2)
    cs = g.get(pic.STATE_CELL_START)
    ids = g.get(pic.STATE_ID)
    assert cs[0] == 0 and cs[-1] == disc["np"] and np.all(np.diff(cs) >= 0)
    assert np.array_equal(np.sort(ids), np.arange(disc["np"]))
    rho = g.get(pic.STATE_RHO)
    assert rho.sum() * (1 / 128) ** 3 == pytest.approx(prob["q"] * prob["nphys"], rel=1e-6)
    e = g.errors()
    assert np.all(np.isfinite(e["l2"])) and e["l2"][0] < 1e-3
