"""Pins of the oracle's forces and energies against what the mathematics fixes:
finite differences of the energy, Newton's third law, closed-form special values
and special cases (potential minima, the straight angle at theta0 = pi, the
cis/trans dihedral)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _two_body_system(positions, types, bonds, L=20.0):
    x = np.array(positions, dtype=np.float64)
    n = x.shape[0]
    return synth.System(L=L, x=synth.wrap(x, L), v=np.zeros((n, 3)), type=np.array(types, dtype=np.int32),
                        reactive=np.ones(n, dtype=np.uint8), bonds=np.array(bonds, dtype=np.int32).reshape(-1, 4))


def _ff(eps=1.0, bonds=None, angles=None, dihedrals=None, depth=1):
    ff = synth.ForceField(eps=eps, exclude_depth=depth, gamma=0.0)
    ff.bonds = bonds or {}
    ff.angles = angles or {}
    ff.dihedrals = dihedrals or {}
    return ff


def _energy(o):
    e = o.energy()
    return e[1] + e[2] + e[3] + e[4]


def _fd_check(o, sysm, idx, h=1e-6):
    f = o.forces()
    worst = 0.0
    for i in idx:
        for k in range(3):
            xp = sysm.x.copy(); xp[i, k] += h
            xm = sysm.x.copy(); xm[i, k] -= h
            o.set_state(synth.wrap(xp, sysm.L), sysm.v, sysm.type)
            up = _energy(o)
            o.set_state(synth.wrap(xm, sysm.L), sysm.v, sysm.type)
            um = _energy(o)
            fd = -(up - um) / (2 * h)
            worst = max(worst, abs(fd - f[i, k]) / (1.0 + abs(f[i, k])))
    o.set_state(sysm.x, sysm.v, sysm.type)
    return worst


@pytest.fixture(scope="module")
def perturbed_duplexes():
    s = synth.small_duplexes(n_duplex=3, n_bp=6, rho=0.05)
    rng = np.random.default_rng(0)
    s.x = synth.wrap(s.x + rng.normal(0, 0.08, size=s.x.shape), s.L)
    return s


@pytest.mark.parametrize("term", ["pair", "bond", "angle", "angle_pi", "dihedral", "dihedral_phase"])
def test_finite_difference_each_term(perturbed_duplexes, term):
    s = perturbed_duplexes
    base = synth.ff_t2()
    zero_b = {t: (0.0, 1.0) for t in base.bonds}
    if term == "pair":
        ff = _ff(eps=1.0, bonds=zero_b, angles={1: (0.0, 1.0)}, dihedrals={1: (0.0, 0.0)})
    elif term == "bond":
        ff = _ff(eps=0.0, bonds=base.bonds, angles={1: (0.0, 1.0)}, dihedrals={1: (0.0, 0.0)})
    elif term == "angle":
        ff = _ff(eps=0.0, bonds=zero_b, angles={1: (10.0, 2.0)}, dihedrals={1: (0.0, 0.0)})
    elif term == "angle_pi":
        ff = _ff(eps=0.0, bonds=zero_b, angles={1: (10.0, math.pi)}, dihedrals={1: (0.0, 0.0)})
    elif term == "dihedral":
        ff = _ff(eps=0.0, bonds=zero_b, angles={1: (0.0, 1.0)}, dihedrals={1: (5.0, 0.0)})
    else:
        ff = _ff(eps=0.0, bonds=zero_b, angles={1: (0.0, 1.0)}, dihedrals={1: (5.0, 0.7)})
    o = oracle.Oracle.from_system(s, ff, synth.rules_t2(), seed=1)
    assert _fd_check(o, s, range(s.n)) < 2e-6


def test_finite_difference_total_and_newton3(perturbed_duplexes):
    s = perturbed_duplexes
    o = oracle.Oracle.from_system(s, synth.ff_t2(), synth.rules_t2(), seed=1)
    f = o.forces()
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * np.abs(f).sum()
    assert _fd_check(o, s, range(0, s.n, 3)) < 2e-6


def test_wca_closed_form_values():
    rc = 2.0 ** (1.0 / 6.0)
    # U(sigma) = eps ; U(rc) = 0 with zero force ; force at sigma = 24 eps / sigma
    for r, u_exp, f_exp in [(1.0, 1.0, 24.0), (rc * (1 - 1e-12), 0.0, 0.0)]:
        s = _two_body_system([[5, 5, 5], [5 + r, 5, 5]], [1, 1], [])
        o = oracle.Oracle.from_system(s, _ff(), None)
        e = o.energy()
        f = o.forces()
        assert e[1] == pytest.approx(u_exp, abs=1e-12)
        assert f[1, 0] == pytest.approx(f_exp, abs=1e-9)
        assert f[0, 0] == pytest.approx(-f_exp, abs=1e-9)
    # beyond the cutoff: nothing
    s = _two_body_system([[5, 5, 5], [6.2, 5, 5]], [1, 1], [])
    o = oracle.Oracle.from_system(s, _ff(), None)
    assert o.energy()[1] == 0.0 and np.all(o.forces() == 0.0)


def test_wca_minimum_image_across_boundary():
    s = _two_body_system([[0.2, 5, 5], [19.2, 5, 5]], [1, 1], [])
    o = oracle.Oracle.from_system(s, _ff(), None)
    f = o.forces()
    assert o.energy()[1] == pytest.approx(1.0, abs=1e-12)   # separation 1.0 through the boundary
    assert f[0, 0] == pytest.approx(24.0, abs=1e-9)          # pushed towards +x, away from its image


def test_bonded_pairs_excluded_from_wca():
    s = _two_body_system([[5, 5, 5], [6.0, 5, 5]], [1, 2], [(0, 1, 4, 4)])
    o = oracle.Oracle.from_system(s, _ff(bonds={4: (100.0, 1.0)}), None)
    e = o.energy()
    assert e[1] == 0.0
    assert e[2] == 0.0
    assert np.all(np.abs(o.forces()) < 1e-12)


def test_harmonic_bond_values_and_directional_types():
    # U = K (r - r0)^2 per direction; the bond energy is the mean of the two stored types
    s = _two_body_system([[5, 5, 5], [6.5, 5, 5]], [1, 2], [(0, 1, 2, 3)])
    o = oracle.Oracle.from_system(s, _ff(bonds={2: (100.0, 1.0), 3: (50.0, 1.2)}, eps=0.0), None)
    e = o.energy()
    assert e[2] == pytest.approx(0.5 * (100 * 0.25 + 50 * 0.09), abs=1e-12)
    f = o.forces()
    assert f[0, 0] == pytest.approx(2 * 100 * 0.5, abs=1e-9)     # bead 0 pulled by its own type 2
    assert f[1, 0] == pytest.approx(-2 * 50 * 0.3, abs=1e-9)     # bead 1 pulled by its own type 3


@pytest.mark.parametrize("theta", [math.pi, 0.5 * math.pi, 2.0])
def test_angle_closed_form(theta):
    a = [5 + math.cos(theta), 5 + math.sin(theta), 5]
    s = _two_body_system([a, [5, 5, 5], [6, 5, 5]], [5, 5, 5], [(1, 0, 2, 3), (1, 2, 3, 2)])
    s.angles = np.array([[1, 0, 1, 2]], dtype=np.int32)
    o = oracle.Oracle.from_system(s, _ff(eps=0.0, bonds={2: (0.0, 1.0), 3: (0.0, 1.0)}, angles={1: (10.0, math.pi)}),
                                  None)
    e = o.energy()
    f = o.forces()
    assert e[3] == pytest.approx(10.0 * (theta - math.pi) ** 2, abs=1e-12)
    assert np.all(np.isfinite(f))
    if theta == math.pi:
        assert np.abs(f).max() < 1e-9
    assert np.abs(f.sum(axis=0)).max() < 1e-12


def _dihedral_system(phi):
    # b at origin-ish, c along +x, a in the xy plane, d rotated by phi about b->c
    b = np.array([5.0, 5.0, 5.0]); c = b + [1.0, 0, 0]
    a = b + [0.0, 1.0, 0]
    d = c + [0.0, math.cos(phi), math.sin(phi)]
    s = _two_body_system([a, b, c, d], [1, 5, 5, 2], [(0, 1, 4, 4), (1, 2, 2, 3), (2, 3, 4, 4)])
    s.dihedrals = np.array([[1, 0, 1, 2, 3]], dtype=np.int32)
    return s


@pytest.mark.parametrize("phi", [0.0, math.pi, 0.5 * math.pi, -0.5 * math.pi, 1.0])
def test_dihedral_closed_form(phi):
    s = _dihedral_system(phi)
    ff = _ff(eps=0.0, bonds={2: (0.0, 1.0), 3: (0.0, 1.0), 4: (0.0, 1.0)}, dihedrals={1: (5.0, 0.0)})
    o = oracle.Oracle.from_system(s, ff, None)
    # cis = 0: U = K (1 - cos phi)
    assert o.energy()[4] == pytest.approx(5.0 * (1 - math.cos(phi)), abs=1e-12)
    if phi == 0.0:
        assert np.abs(o.forces()).max() < 1e-12


def test_dihedral_sign_convention():
    # IUPAC: viewed along b->c, a positive dihedral turns the near bond a clockwise onto the far bond d.
    # With a along +y and d = (0, cos, sin): phi = +90 deg puts d along +z.  A phase phi0 = +pi/2
    # must then give zero energy, and phi0 = -pi/2 the maximum 2K.
    s = _dihedral_system(0.5 * math.pi)
    for p0, u_exp in [(0.5 * math.pi, 0.0), (-0.5 * math.pi, 10.0)]:
        ff = _ff(eps=0.0, bonds={2: (0.0, 1.0), 3: (0.0, 1.0), 4: (0.0, 1.0)}, dihedrals={1: (5.0, p0)})
        o = oracle.Oracle.from_system(s, ff, None)
        # b1 = b - a = -y, b2 = +x, b3 = +z: sign(b1 . (b2 x b3)) = sign(-y . -y) > 0
        assert o.energy()[4] == pytest.approx(u_exp, abs=1e-12)


def test_degenerate_dihedral_is_skipped_not_nan():
    b = np.array([5.0, 5.0, 5.0])
    s = _two_body_system([b - [1, 0, 0], b, b + [1, 0, 0], b + [2, 0, 0]], [1, 5, 5, 2],
                         [(0, 1, 4, 4), (1, 2, 2, 3), (2, 3, 4, 4)])
    s.dihedrals = np.array([[1, 0, 1, 2, 3]], dtype=np.int32)
    ff = _ff(eps=0.0, bonds={2: (0.0, 1.0), 3: (0.0, 1.0), 4: (0.0, 1.0)}, dihedrals={1: (5.0, 0.0)})
    o = oracle.Oracle.from_system(s, ff, None)
    assert np.all(np.isfinite(o.forces()))
    assert o.energy()[4] == 0.0


def test_virial_of_a_pair():
    # virial = sum over pairs of r_ij . F_ij = r * |F| for a single repulsive pair
    s = _two_body_system([[5, 5, 5], [6.0, 5, 5]], [1, 1], [])
    o = oracle.Oracle.from_system(s, _ff(), None)
    assert o.energy()[5] == pytest.approx(24.0, abs=1e-9)
