"""Scattering-angle recovery on the GPU (eq. angle_recovery and the
empirical-CDF errors after it): the recorded (chi, eps) set equals the
oracle's, the GPU metric equals the oracle's metric on the same records, the
mixed form agrees, the metric behaves as O(N^-1/2) at full size, and an
undersized log is reported."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2602_15130_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _paper_isolated():
    prob = W.paper_problem(collisions=True, field_to_particles=False, particles_to_field=False,
                           isolate=True)
    disc = dict(W.paper_level(1))
    disc["navg"] = 8
    return prob, disc


def test_angle_records_and_metric_match_oracle():
    from paper_2602_15130_amd import pic
    prob, disc = _paper_isolated()
    g = pic.Sim(prob, disc, 1, 0, "fp64")
    g.angle_log(200000)
    g.step(2)
    eg, n = g.angle_errors()
    rg = g.angle_records(n)
    o = O.Sim(prob, disc, 1, 0)
    assert o.init() == 0
    with O.AngleRecorder() as rec:
        o.step(2)
    assert n == rec.total and n > 5000
    for col in (0, 1):
        np.testing.assert_allclose(np.sort(rg[:, col]), np.sort(rec.records[:, col]), rtol=0, atol=1e-9)
    np.testing.assert_allclose(eg, O.angle_errors(rg), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(eg, O.angle_errors(rec.records), rtol=0, atol=2.0 / n)


def test_mixed_form_angles():
    from paper_2602_15130_amd import pic
    prob = W.cfg_problem(two_way=False, collisionality=30.0)
    disc = W.cfg_disc(8, 16384, 1e-3, 1, 8)
    out = {}
    for prec in ("fp64", "mixed"):
        g = pic.Sim(prob, disc, 2, 0, prec)
        g.angle_log(400000)
        g.step(2)
        out[prec] = g.angle_errors()
    (ef, nf), (em, nm) = out["fp64"], out["mixed"]
    assert abs(nf - nm) <= 2 and nf > 10000
    np.testing.assert_allclose(em, ef, rtol=0, atol=5e-4)
    assert np.all(np.array(ef)[[1, 3]] * math.sqrt(nf) < 2.0)


def test_full_size_angles_and_capacity():
    from paper_2602_15130_amd import pic
    c = W.get("cfg3")
    g = pic.Sim(c["problem"], c["disc"], 1, 0, "mixed")
    g.angle_log(1 << 20)
    g.step(2)
    e, n = g.angle_errors()
    assert n > 50000
    assert np.all(np.array(e)[[1, 3]] * math.sqrt(n) < 2.0), (e, n)
    g.angle_log(10)
    g.step(1)
    with pytest.raises(pic.PicError) as ei:
        g.angle_errors()
    assert ei.value.code == pic.PIC_ESPACE


@pytest.mark.parametrize("chi_model,chi_alpha", [(1, 1.0), (2, 2.0), (2, 1.5)])
def test_anisotropic_samplers_match_oracle(chi_model, chi_alpha):
    """The manufactured anisotropy (eq. pchi_ms / eq. fpiv_ms) and VSS
    (eq. vss): the FP64 form's recorded (chi, eps) set equals the oracle's, its
    metric against the model's own CDF equals the oracle's and is O(N^-1/2),
    while the isotropic CDF is rejected; the mixed form's metric agrees; a
    collision call agrees with the oracle's Algorithm 1 cell by cell."""
    from paper_2602_15130_amd import pic
    prob, disc = _paper_isolated()
    prob["chi_model"], prob["chi_alpha"] = chi_model, chi_alpha
    g = pic.Sim(prob, disc, 1, 0, "fp64")
    g.angle_log(200000)
    g.step(2)
    eg, n = g.angle_errors()
    rg = g.angle_records(n)
    o = O.Sim(prob, disc, 1, 0)
    assert o.init() == 0
    with O.AngleRecorder() as rec:
        o.step(2)
    assert n == rec.total and n > 5000
    for col in (0, 1):
        np.testing.assert_allclose(np.sort(rg[:, col]), np.sort(rec.records[:, col]), rtol=0, atol=1e-9)
    np.testing.assert_allclose(eg, O.angle_errors(rg, chi_model, chi_alpha), rtol=1e-12, atol=1e-15)
    assert np.all(np.array(eg)[[1, 3]] * math.sqrt(n) < 2.0), np.array(eg) * math.sqrt(n)

    # mixed form on the configuration family: the same law
    cp = W.cfg_problem(two_way=False, collisionality=30.0)
    cp["chi_model"], cp["chi_alpha"] = chi_model, chi_alpha
    cd = W.cfg_disc(8, 16384, 1e-3, 1, 8)
    m = pic.Sim(cp, cd, 2, 0, "mixed")
    m.angle_log(400000)
    m.step(4)
    em, nm = m.angle_errors()
    assert nm > 25000 and np.all(np.array(em)[[1, 3]] * math.sqrt(nm) < 2.0), (em, nm)
    # the isotropic law differs from these by at least 0.034 in sup norm
    assert O.angle_errors(m.angle_records(nm), 0, 1.0)[1] * math.sqrt(nm) > 4.0

    # one collision call, cell by cell against the oracle
    h = pic.Sim(prob, disc, 3, 0, "fp64")
    dg, _, _, _ = h.collide(0, 0.0)
    v = h.get(pic.STATE_V)
    cs = h.get(pic.STATE_CELL_START)
    scale = np.abs(v).max()
    for cell in np.random.default_rng(5).choice(len(cs) - 1, size=6, replace=False):
        s, e = cs[cell], cs[cell + 1]
        do, _, _, _ = O.collide_cell(prob, disc, 3, 0, 0, 0, int(cell), v[:, s:e])
        assert np.abs(dg[:, s:e] - do).max() <= 1e-12 * scale
