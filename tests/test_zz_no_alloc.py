"""pic_errors_noalloc (error norms with the partial sums in the library's
static scratch) against pic_errors (partial sums in the context's
workspace): both run the same kernels on the same grid, so the norms agree
bit for bit, on two calls in a row with a smaller problem second, and again
on the first problem after the scratch held the second's partials."""
import numpy as np
import pytest

from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _sims(precision):
    from paper_2602_15130_amd import pic as P
    prob = W.cfg_problem(two_way=True, collisionality=10.0)
    big = P.Sim(prob, W.cfg_disc(16, 300000, 1e-3, 1, 4, cg_tol=1e-12), 3, 0, precision)
    small = P.Sim(prob, W.cfg_disc(5, 700, 1e-3, 1, 4, cg_tol=1e-12), 7, 0, precision)
    big.step(2)
    small.step(3)
    return P, big, small


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_errors_noalloc_equals_errors(precision):
    P, big, small = _sims(precision)
    for s in (big, small, big):
        a = P.pic_errors(s.ctx)
        b = P.pic_errors_noalloc(s.ctx)
        assert b["status"] == a["status"] == P.PIC_OK
        assert b["t"] == a["t"]
        np.testing.assert_array_equal(b["l2"], a["l2"])
        np.testing.assert_array_equal(b["linf"], a["linf"])
        assert np.all(a["l2"] > 0)
