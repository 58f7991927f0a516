"""Pins of the oracle's DPD force field (section 3: soft conservative force
a w(r), dissipative force -gamma w^2 (e . v_ij), random force sigma w xi / sqrt(dt)
with sigma^2 = 2 T gamma): closed forms of the conservative part, finite
differences of its energy, exclusions, momentum conservation of the full pair
force, and the fluctuation-dissipation balance (the thermostat holds the
temperature it is given, independently of dt)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _dpd_ff(a=25.0, gamma=4.5, T=1.0, dt=0.01, depth=1, rc=1.0):
    ff = synth.ForceField(pair="dpd", dpd_a=a, dpd_gamma=gamma, rc=rc, exclude_depth=depth, gamma=0.0, dt=dt,
                          T0=T, T1=T)
    return ff


def _sys(x, L, v=None, bonds=()):
    x = np.array(x, dtype=np.float64)
    n = x.shape[0]
    return synth.System(L=L, x=synth.wrap(x, L), v=np.zeros((n, 3)) if v is None else np.array(v, dtype=np.float64),
                        type=np.ones(n, dtype=np.int32), reactive=np.zeros(n, dtype=np.uint8),
                        bonds=np.array(bonds, dtype=np.int32).reshape(-1, 4))


@pytest.mark.parametrize("r", [0.05, 0.3, 0.7, 0.99])
def test_conservative_pair_closed_form(r):
    a, rc = 25.0, 1.0
    s = _sys([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]], 10.0)
    o = oracle.Oracle.from_system(s, _dpd_ff(a=a, gamma=0.0), synth.RuleSet(every=0), seed=1)
    f = o.forces()
    w = 1.0 - r / rc
    # r_ij = x_i - x_j points from j to i: bead 0 is pushed to -x, bead 1 to +x
    assert f[0] == pytest.approx([-a * w, 0.0, 0.0], abs=1e-12)
    assert f[1] == pytest.approx([a * w, 0.0, 0.0], abs=1e-12)
    assert o.energy()[1] == pytest.approx(0.5 * a * rc * w * w, rel=1e-13)


def test_conservative_vanishes_at_and_beyond_cutoff():
    for r in (1.0, 1.2):
        s = _sys([[5.0, 5.0, 5.0], [5.0, 5.0 + r, 5.0]], 10.0)
        o = oracle.Oracle.from_system(s, _dpd_ff(gamma=0.0), synth.RuleSet(every=0), seed=1)
        assert np.abs(o.forces()).max() == 0.0 and o.energy()[1] == 0.0


def test_bonded_pair_is_excluded():
    s = _sys([[5.0, 5.0, 5.0], [5.6, 5.0, 5.0]], 10.0, bonds=[(0, 1, 1, 1)])
    o = oracle.Oracle.from_system(s, _dpd_ff(gamma=0.0), synth.RuleSet(every=0), seed=1)
    assert np.abs(o.forces()).max() == 0.0


def test_conservative_forces_are_minus_the_energy_gradient():
    rng = np.random.default_rng(3)
    L = 4.0
    x = rng.uniform(0, L, size=(150, 3))
    s = _sys(x, L)
    ff = _dpd_ff(gamma=0.0)
    o = oracle.Oracle.from_system(s, ff, synth.RuleSet(every=0), seed=1)
    f = o.forces()
    h = 1e-6
    worst = 0.0
    for i in (0, 17, 64, 149):
        for k in range(3):
            xp = x.copy(); xp[i, k] += h
            xm = x.copy(); xm[i, k] -= h
            up = oracle.Oracle.from_system(_sys(xp, L), ff, synth.RuleSet(every=0), seed=1).energy()[1]
            um = oracle.Oracle.from_system(_sys(xm, L), ff, synth.RuleSet(every=0), seed=1).energy()[1]
            worst = max(worst, abs(-(up - um) / (2 * h) - f[i, k]))
    assert worst < 1e-6


def _fluid(n_side=6, rho=3.0, seed=5, T=1.0):
    n = int(rho * n_side ** 3)
    L = float(n_side)
    rng = np.random.default_rng(seed)
    return _sys(rng.uniform(0, L, size=(n, 3)), L, v=rng.normal(0.0, math.sqrt(T), size=(n, 3)))


def test_full_pair_force_conserves_momentum():
    s = _fluid()
    s.v -= s.v.mean(axis=0)
    o = oracle.Oracle.from_system(s, _dpd_ff(), synth.RuleSet(every=0), seed=7)
    o.step(20)
    _, v = o.state()
    assert np.abs(v.sum(axis=0)).max() < 1e-9


@pytest.mark.parametrize("gamma,dt", [(4.5, 0.01), (4.5, 0.005), (100.0, 0.01)])
def test_thermostat_holds_the_temperature(gamma, dt):
    """Fluctuation-dissipation: starting hot (T = 3), the fluid relaxes to the set
    T = 1; the mean kinetic energy per bead is 3T/2 within 3 % (dt = 0.01 is the
    paper's step; halving it must not move the temperature; friction 100 is the
    paper's stated value)."""
    s = _fluid(T=3.0)
    o = oracle.Oracle.from_system(s, _dpd_ff(gamma=gamma, dt=dt), synth.RuleSet(every=0), seed=11)
    o.step(int(round(8.0 / dt)))
    ke = []
    for _ in range(40):
        o.step(int(round(0.25 / dt)))
        ke.append(o.energy()[0] / s.n)
    assert np.mean(ke) == pytest.approx(1.5, rel=0.03)
