"""Pins of the oracle's time stepping: velocity Verlet conserves energy with a
drift/fluctuation scaling as dt^2 (gamma = 0, sweep off); the Langevin thermostat
reaches equipartition <KE> = 3/2 N T; a run restarted from a saved snapshot follows the original one."""
import numpy as np
import pytest

import oracle
import synth


def _nve_system():
    s = synth.small_duplexes(n_duplex=4, n_bp=6, rho=0.05, seed_d=3, T=0.5)
    return s


def _energy_error(dt, t_total=2.0):
    s = _nve_system()
    ff = synth.ff_t2(gamma=0.0, dt=dt)
    rules = synth.rules_t2(every=0)
    o = oracle.Oracle.from_system(s, ff, rules, seed=1)
    e0 = None
    worst = 0.0
    nsteps = int(round(t_total / dt))
    chunk = max(1, nsteps // 50)
    for _ in range(nsteps // chunk):
        o.step(chunk)
        e = o.energy()
        tot = e[0] + e[1] + e[2] + e[3] + e[4]
        if e0 is None:
            e0 = tot
        worst = max(worst, abs(tot - e0))
    return worst


def test_nve_energy_error_scales_as_dt_squared():
    e1 = _energy_error(0.004)
    e2 = _energy_error(0.002)
    ratio = e1 / e2
    assert 2.5 < ratio < 6.0, (e1, e2)
    assert e2 < 0.05


def test_langevin_equipartition():
    s = synth.random_gas(300, 12.0, seed=4, min_dist=0.9)
    ff = synth.ForceField(gamma=2.0, dt=0.005, T0=1.3, T1=1.3)
    o = oracle.Oracle.from_system(s, ff, synth.RuleSet(every=0), seed=5)
    o.step(400)
    ke = []
    for _ in range(60):
        o.step(20)
        ke.append(o.energy()[0])
    ratio = np.mean(ke) / (1.5 * s.n * 1.3)
    assert abs(ratio - 1.0) < 0.05


def test_temperature_ramp_is_linear():
    s = synth.random_gas(400, 14.0, seed=6, min_dist=0.9)
    ff = synth.ForceField(gamma=5.0, dt=0.005, T0=0.5, T1=1.5, ramp_steps=4000)
    o = oracle.Oracle.from_system(s, ff, synth.RuleSet(every=0), seed=7)
    o.step(3000)
    ke = []
    for _ in range(25):
        o.step(40)
        ke.append(o.energy()[0] / (1.5 * s.n))
    # the thermostat lags the ramp slightly; the ramp ends at 1.5 after 4000 steps
    assert 1.3 < np.mean(ke) < 1.6


def test_restart_reproduces_the_run():
    s = synth.small_duplexes(n_duplex=3, n_bp=6, rho=0.05)
    ff = synth.ff_t2()
    rules = synth.rules_t2(p=0.5, every=10)
    a = oracle.Oracle.from_system(s, ff, rules, seed=3)
    a.step(60)
    x1, v1 = a.state()
    b = oracle.Oracle.from_system(s, ff, rules, seed=3)
    b.step(30)
    x, v = b.state()
    c = oracle.Oracle(s.n, s.L, 3)
    c.set_state(x, v, s.type)
    c.set_reactive(s.reactive)
    c.set_bonds(b.bonds())
    c.set_angles(b.angles())
    c.set_dihedrals(b.dihedrals())
    c.set_forcefield(ff)
    c.set_rules(rules)
    c.set_step(30)
    c.step(30)
    x2, v2 = c.state()
    # the restarted oracle holds its lists in sorted order, so sums may round differently
    assert np.abs(x1 - x2).max() < 1e-10 and np.abs(v1 - v2).max() < 1e-8
    assert {tuple(r) for r in a.bonds().tolist()} == {tuple(r) for r in c.bonds().tolist()}
