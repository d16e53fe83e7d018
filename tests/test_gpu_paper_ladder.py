"""The paper's own refinement ladder (Table 1, paper family, SI constants) on
the GPU, FP64 form: levels 1-3 for the isolated-collision case (q/m = 0, the
exact-difference substitution of Sec. 5.4.1), the fully coupled collisional
case and the fully coupled collisionless case.  Level 1 against the oracle;
observed orders of the l2 norms on the finer pair near the paper's second
order (the isolated-collision l2 norm between 2 and 2.5, Sec. 5.4.1)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "isolated": dict(collisions=True, field_to_particles=False, particles_to_field=False,
                     isolate=True),
    "coupled": dict(collisions=True),
    "collisionless": dict(collisions=False),
}


@pytest.mark.parametrize("case", list(CASES))
def test_table1_ladder_levels_1_to_3(case):
    from paper_2602_15130_amd import pic
    prob = W.paper_problem(**CASES[case])
    coll = CASES[case].get("collisions", True)
    norms = []
    for lv in (1, 2, 3):
        disc = W.paper_level(lv, collisions=coll)
        g = pic.Sim(prob, disc, 1, 0, "fp64")
        g.step(disc["steps"])
        norms.append(np.array(g.errors()["l2"]))
        if lv == 1:
            o = O.Sim(prob, disc, 1, 0)
            assert o.init() == 0
            o.step(disc["steps"])
            np.testing.assert_allclose(norms[0], o.errors()["l2"], rtol=1e-6)
        del g
    r = math.log(W.TABLE1_NCELL[2] / W.TABLE1_NCELL[1])
    orders = np.log(norms[1] / norms[2]) / r
    lo, hi = (1.8, 2.8) if case != "collisionless" else (1.8, 2.5)
    assert np.all((orders > lo) & (orders < hi)), orders
