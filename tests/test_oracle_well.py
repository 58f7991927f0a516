"""Pins of the oracle's well-shaped bond of the 1-bead DNA model (section 3, in
the reading U = U_min [(r - r_w)^2 / (r_z - r_w)^2 - 1] below r_cut, 0 beyond):
the special values the reading fixes (the minimum -U_min at the well, zero at
r_z and, by symmetry, at 2 r_w - r_z), the cutoff, finite differences of the
energy, and directional halves (each bead feels the type it stores)."""
import numpy as np
import pytest

import oracle
import synth

BACKBONE = (10.0, 0.3, 0.6, float("inf"))   # U_min, r_l, r_0, no cutoff
HYB = (1.0, 0.6, 1.0, 1.0)                  # U_min, r_h, r_c, cut at r_c


def _pair(r, t_ij, t_ji, wells, bonds=None, L=20.0):
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    s = synth.System(L=L, x=x, v=np.zeros((2, 3)), type=np.array([1, 2], dtype=np.int32),
                     reactive=np.ones(2, dtype=np.uint8), bonds=np.array([[0, 1, t_ij, t_ji]], dtype=np.int32))
    ff = synth.ForceField(eps=0.0, gamma=0.0)
    ff.wells = dict(wells)
    ff.bonds = dict(bonds or {})
    return oracle.Oracle.from_system(s, ff, synth.RuleSet(every=0), seed=1)


@pytest.mark.parametrize("well", [BACKBONE, HYB])
def test_special_values(well):
    umin, rw, rz, _ = well
    o = _pair(rw, 1, 1, {1: well})
    assert o.energy()[2] == pytest.approx(-umin, abs=1e-14)
    assert np.abs(o.forces()).max() < 1e-12
    # zero just inside r_z, attractive there: bead 0 pulled towards +x by 2 U_min / (r_z - r_w)
    o = _pair(rz - 1e-12, 1, 1, {1: well})
    assert o.energy()[2] == pytest.approx(0.0, abs=1e-9)
    assert o.forces()[0, 0] == pytest.approx(2.0 * umin / (rz - rw), rel=1e-9)
    # the mirror zero below the well, repulsive there
    r = 2 * rw - rz
    if r > 0:
        o = _pair(r, 1, 1, {1: well})
        assert o.energy()[2] == pytest.approx(0.0, abs=1e-12)
        assert o.forces()[0, 0] == pytest.approx(-2.0 * umin / (rz - rw), rel=1e-12)


def test_backbone_well_is_zero_at_contact():
    """With the paper's backbone numbers the zero below the well falls at r = 0."""
    o = _pair(1e-9, 1, 1, {1: BACKBONE})
    assert o.energy()[2] == pytest.approx(0.0, abs=1e-7)


def test_cutoff_removes_force_and_energy():
    o = _pair(1.05, 1, 1, {1: HYB})
    assert o.energy()[2] == 0.0 and np.abs(o.forces()).max() == 0.0
    o = _pair(0.999, 1, 1, {1: HYB})
    assert o.energy()[2] < 0.0 and o.forces()[0, 0] > 0.0


def test_directional_halves():
    """Bead 0 stores the backbone well, bead 1 the hybridization well: each feels
    its own force, and the energy is the mean of the two."""
    r = 0.7
    o = _pair(r, 2, 1, {2: BACKBONE, 1: HYB})
    f = o.forces()
    u_b = BACKBONE[0] * ((r - 0.3) ** 2 / 0.09 - 1.0)
    u_h = HYB[0] * ((r - 0.6) ** 2 / 0.16 - 1.0)
    assert o.energy()[2] == pytest.approx(0.5 * (u_b + u_h), rel=1e-13)
    assert f[0, 0] == pytest.approx(2.0 * 10.0 * (r - 0.3) / 0.09, rel=1e-13)
    assert f[1, 0] == pytest.approx(-2.0 * 1.0 * (r - 0.6) / 0.16, rel=1e-13)


def test_matches_a_harmonic_bond_up_to_the_offset():
    """Below the cutoff the well is a harmonic bond K (r - r_w)^2 with
    K = U_min / (r_z - r_w)^2, shifted by -U_min."""
    for r in (0.2, 0.45, 0.9):
        ow = _pair(r, 1, 1, {1: BACKBONE})
        oh = _pair(r, 1, 1, {}, bonds={1: (10.0 / 0.09, 0.3)})
        assert np.allclose(ow.forces(), oh.forces(), rtol=1e-13, atol=0)
        assert ow.energy()[2] == pytest.approx(oh.energy()[2] - 10.0, rel=1e-13, abs=1e-13)


def test_finite_differences_on_a_ladder():
    lad = synth.ladder_1bead(8, hyb_dist=0.62, bb_dist=0.33)
    rng = np.random.default_rng(4)
    lad.x = synth.wrap(lad.x + rng.normal(0, 0.04, size=lad.x.shape), lad.L)
    ff = synth.ForceField(eps=0.0, gamma=0.0)
    ff.wells = {1: HYB, 2: BACKBONE, 3: BACKBONE}
    o = oracle.Oracle.from_system(lad, ff, synth.RuleSet(every=0), seed=1, generate=False)
    f = o.forces()
    h, worst = 1e-6, 0.0
    for i in (0, 3, 8, 12):
        for k in range(3):
            xp = lad.x.copy(); xp[i, k] += h
            xm = lad.x.copy(); xm[i, k] -= h
            o.set_state(xp, lad.v, lad.type)
            up = o.energy()[2]
            o.set_state(xm, lad.v, lad.type)
            um = o.energy()[2]
            worst = max(worst, abs(-(up - um) / (2 * h) - f[i, k]) / (1.0 + abs(f[i, k])))
    assert worst < 1e-6
