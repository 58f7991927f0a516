"""Constant external forces (the unzipping experiments of section 3) and
directional bonds with a potential in one direction only (the "half bond" of
section 2) on the HIP path against the FP64 oracle."""
import numpy as np
import pytest

import synth
from gpu_common import both, perturbed, rel_l2, forces_close, same_topology, topo_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_4214_amd  # noqa: F401  (fails loudly without the built library)


def _wrapped_diff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


def _end_pair_pull(s, f):
    """ids and forces pulling the duplex's end pair (smallest x) apart across the strands"""
    x = s.x[:24]
    k = int(np.argmin(x[:12, 0]))
    a, b = k, 12 + k
    dy = np.sign(x[b, 1] - x[a, 1])
    return [a, b], [[0.0, -f * dy, 0.0], [0.0, f * dy, 0.0]]


def test_unzipping_trajectory_fp64():
    """A 12-bp duplex of the 1-bead model in DPD solvent, its end pair pulled apart
    with 100 (the paper's strong pull): forty steps, a sweep every step, topology
    after every five and positions at the end."""
    import paper_1108_4214_amd as pk
    s = synth.dna1_solution(1, 12, 1536, 3.0, 3, 13)
    g, o = both(s, synth.ff_dna1(), synth.rules_fig2(), seed=5)
    ids, f = _end_pair_pull(s, 100.0)
    pk.db_external_force(g.ctx, ids, f)
    o.set_external_force(ids, f)
    for _ in range(8):
        g.step(5)
        o.step(5)
        assert same_topology(g, o), topo_diff(g, o)
    assert np.abs(_wrapped_diff(g.state()[0], o.state()[0], s.L)).max() < 1e-9
    assert o.counts()[0] < len(s.bonds)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_forces_and_energy_with_external_forces(precision, tol):
    import paper_1108_4214_amd as pk
    s = perturbed(synth.dna1_solution(30, 10, 3000, 3.0, 5, 15), 0.05, 1)
    g, o = both(s, synth.ff_dna1(), synth.rules_fig2(), precision=precision)
    rng = np.random.default_rng(3)
    ids = rng.choice(s.n, size=60, replace=False)
    f = rng.normal(0.0, 20.0, size=(60, 3))
    ids[1] = ids[0]                      # listed twice: the forces add
    pk.db_external_force(g.ctx, ids, f)
    o.set_external_force(ids, f)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg
    eg, eo = g.energy(), o.energy()
    assert abs(eg[0] - eo[0]) <= (1e-11 if precision == 0 else 1e-5) * abs(eo[0])
    pk.db_external_force(g.ctx, [], np.zeros((0, 3)))
    o.set_external_force([], np.zeros((0, 3)))
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


def test_half_bonds_propel_a_chain():
    """A chain whose bonds pull only towards the head (the tail-side bead stores a
    type with K = 0): a net force, a growing momentum, and the oracle's trajectory."""
    n = 12
    x = np.array([[5.0 + 1.2 * k, 5.0, 5.0] for k in range(n)])
    s = synth.System(L=20.0, x=x, v=np.zeros((n, 3)), type=np.ones(n, dtype=np.int32),
                     reactive=np.zeros(n, dtype=np.uint8),
                     bonds=np.array([(k, k + 1, 1, 2) for k in range(n - 1)], dtype=np.int32))
    ff = synth.ForceField(eps=1.0, gamma=0.0, dt=0.005, bonds={1: (10.0, 1.0), 2: (0.0, 1.0)})
    g, o = both(s, ff, synth.RuleSet(every=0))
    ok, msg = forces_close(g.forces(), o.forces(), 1e-12)
    assert ok, msg
    assert abs(g.forces().sum(axis=0)[0]) > 1.0
    g.step(50)
    o.step(50)
    xg, vg = g.state()
    xo, vo = o.state()
    assert np.abs(_wrapped_diff(xg, xo, s.L)).max() < 1e-10
    assert np.abs(vg - vo).max() < 1e-9
    assert abs(vg.sum(axis=0)[0]) > 1e-3


def test_external_force_rejects_bad_input_and_batches():
    import paper_1108_4214_amd as pk
    s = synth.dna1_solution(1, 12, 1536, 3.0, 3, 13)
    g = pk.System(s.n, s.L, 1).configure(s, synth.ff_dna1(), synth.rules_fig2())
    for ids, f in (([s.n], [[1.0, 0, 0]]), ([-1], [[1.0, 0, 0]]), ([0], [[np.nan, 0, 0]])):
        with pytest.raises(pk.DynBondError):
            pk.db_external_force(g.ctx, ids, f)
    g2 = pk.System(s.n, s.L, 2).configure(s, synth.ff_dna1(), synth.rules_fig2())
    pk.db_external_force(g2.ctx, [0], [[1.0, 0, 0]])
    with pytest.raises(pk.DynBondError):
        pk.Batch([g, g2])
