"""Pins of the oracle's virial, term by term.

For forces that are sums of internal interactions (pair, bond, angle and
dihedral terms all depend on separations only, so they sum to zero and are
unchanged by translation), the virial W = sum over interactions of r . F equals
sum_i x_i . F_i evaluated with coordinates in which no interaction crosses the
periodic boundary (Clausius; e.g. Allen and Tildesley, Computer Simulation of
Liquids, section 2.4).  Each case below switches one potential on, places a
perturbed 2-bead duplex cluster in the middle of a large box and compares the
virial the oracle reports with sum_i x_i . F_i of the forces it reports.  A
dropped factor or a wrong sign in a pair or bond virial makes the two differ.
Angle and dihedral energies depend on angles only, so they do not change when
all coordinates are scaled about any origin; by Euler's theorem on homogeneous
functions their sum_i x_i . F_i is zero, and the pin asserts that the oracle's
virial of those terms vanishes with it.
"""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def cluster():
    rng = np.random.default_rng(41)
    b = synth._Builder()
    synth.add_duplex(b, synth.random_sequence(rng, 7), origin=[14.0, 14.0, 15.0])
    synth.add_duplex(b, synth.random_sequence(rng, 6), origin=[14.5, 14.3, 15.95], flip_x=True)
    s = synth._finish(b, 30.0, rng, 1.0)
    s.x = s.x + rng.normal(0.0, 0.09, size=s.x.shape)
    assert s.x.min() > 5.0 and s.x.max() < 25.0   # no interaction crosses the boundary
    return s


def _ff(kind):
    ff = synth.ForceField(eps=0.0, gamma=0.0, exclude_depth=1)
    zero_b = {t: (0.0, 1.0) for t in (1, 2, 3, 4)}
    ff.bonds, ff.angles, ff.dihedrals = dict(zero_b), {1: (0.0, 1.0)}, {1: (0.0, 0.0)}
    if kind == "wca":
        ff.eps = 1.0
    elif kind == "bond":
        ff.bonds = {1: (50.0, 1.2), 2: (100.0, 1.0), 3: (100.0, 1.0), 4: (100.0, 1.0)}
    elif kind == "well":
        ff.bonds = {}
        ff.wells = {1: (1.0, 0.9, 1.6, 1.5), 2: (10.0, 0.8, 1.3, math.inf), 3: (10.0, 0.8, 1.3, math.inf),
                    4: (5.0, 0.95, 1.4, math.inf)}
    elif kind == "angle":
        ff.angles = {1: (10.0, 2.0)}
    elif kind == "angle_pi":
        ff.angles = {1: (10.0, math.pi)}
    elif kind == "dihedral":
        ff.dihedrals = {1: (5.0, 0.7)}
    elif kind == "dpd":
        ff.pair, ff.dpd_a, ff.dpd_gamma, ff.rc = "dpd", 25.0, 0.0, 1.0
    return ff


@pytest.mark.parametrize("kind", ["wca", "bond", "well", "angle", "angle_pi", "dihedral", "dpd"])
def test_virial_equals_sum_of_x_dot_f(cluster, kind):
    o = oracle.Oracle.from_system(cluster, _ff(kind), synth.rules_t2(), seed=3)
    f = o.forces()
    e = o.energy()
    w = float(np.sum(cluster.x * f))
    assert np.abs(f).max() > 1e-3, "the term under test exerts no force"
    assert e[5] == pytest.approx(w, rel=1e-10, abs=1e-10 * np.abs(cluster.x * f).sum())


def test_virial_of_all_terms_is_the_sum_of_each(cluster):
    ff = synth.ff_t2(gamma=0.0)
    o = oracle.Oracle.from_system(cluster, ff, synth.rules_t2(), seed=3)
    f = o.forces()
    assert o.energy()[5] == pytest.approx(float(np.sum(cluster.x * f)), rel=1e-10)
