"""Pins of the oracle's constant external forces (the unzipping experiments of
section 3) and of directional bonds with different potentials in the two
directions (the "half bond" remark of section 2): an isolated bead accelerates
uniformly, opposing forces leave the momentum unchanged, a half bond exerts a
net force equal to the one direction's bond force."""
import numpy as np
import pytest

import oracle
import synth


def _sys(x, bonds=(), L=20.0, v=None):
    x = np.array(x, dtype=np.float64)
    n = x.shape[0]
    return synth.System(L=L, x=x, v=np.zeros((n, 3)) if v is None else np.array(v, dtype=np.float64),
                        type=np.ones(n, dtype=np.int32), reactive=np.zeros(n, dtype=np.uint8),
                        bonds=np.array(bonds, dtype=np.int32).reshape(-1, 4))


def _ff(**kw):
    ff = synth.ForceField(eps=0.0, gamma=0.0, dt=0.01)
    for k, v in kw.items():
        setattr(ff, k, v)
    return ff


def test_isolated_bead_accelerates_uniformly():
    """x(t) = x0 + f t^2 / 2 exactly for the velocity-Verlet scheme with a constant force."""
    o = oracle.Oracle.from_system(_sys([[5.0, 5.0, 5.0]]), _ff(), synth.RuleSet(every=0), seed=1)
    f = np.array([0.3, -0.2, 0.1])
    o.set_external_force([0], [f])
    assert np.allclose(o.forces()[0], f, rtol=0, atol=0)
    o.step(100)
    x, v = o.state()
    t = 100 * 0.01
    assert np.allclose(v[0], f * t, rtol=1e-12, atol=1e-14)
    assert np.allclose(x[0], 5.0 + 0.5 * f * t * t + 0.5 * f * t * 0.01, rtol=1e-12)


def test_opposing_forces_keep_momentum_and_clear():
    s = _sys([[5.0, 5.0, 5.0], [5.6, 5.0, 5.0]], bonds=[(0, 1, 1, 1)])
    o = oracle.Oracle.from_system(s, _ff(bonds={1: (1.0, 0.6)}), synth.RuleSet(every=0), seed=1)
    f0 = o.forces()
    o.set_external_force([0, 1], [[0, -28.0, 0], [0, 28.0, 0]])
    f = o.forces()
    assert np.array_equal(f - f0, [[0, -28.0, 0], [0, 28.0, 0]])
    o.set_external_force([], np.zeros((0, 3)))
    assert np.array_equal(o.forces(), f0)
    o.set_external_force([0, 1], [[0, -28.0, 0], [0, 28.0, 0]])
    o.step(50)
    x, v = o.state()
    assert np.abs(v.sum(axis=0)).max() < 1e-12
    assert x[1, 1] - x[0, 1] > 0.1   # pulled apart across the bond


def test_listed_twice_sums_and_bad_ids_rejected():
    o = oracle.Oracle.from_system(_sys([[5.0, 5.0, 5.0]]), _ff(), synth.RuleSet(every=0), seed=1)
    o.set_external_force([0, 0], [[1.0, 0, 0], [2.0, 0, 0]])
    assert o.forces()[0, 0] == 3.0
    with pytest.raises(oracle.OracleError):
        o.set_external_force([1], [[1.0, 0, 0]])


def test_half_bond_gives_a_net_force():
    """Bead 0 stores a bond type with K = 2, bead 1 a type with K = 0: only bead 0
    is pulled, so the pair's total force is bead 0's bond force."""
    r = 1.3
    s = _sys([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]], bonds=[(0, 1, 1, 2)])
    o = oracle.Oracle.from_system(s, _ff(bonds={1: (2.0, 1.0), 2: (0.0, 1.0)}), synth.RuleSet(every=0), seed=1)
    f = o.forces()
    assert f[0, 0] == pytest.approx(2 * 2.0 * (r - 1.0), rel=1e-13)
    assert np.abs(f[1]).max() == 0.0
    assert f.sum(axis=0)[0] == pytest.approx(2 * 2.0 * (r - 1.0), rel=1e-13)
