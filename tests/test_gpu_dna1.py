"""The paper's 1-bead DNA model end to end on the HIP path (section 3 force field:
well-shaped hybridization and backbone bonds, straight and right angles, cis and
trans stacking dihedrals, DPD solvent at density 3; Fig. 2 rule table with a
sweep every step): forces and energies against the FP64 oracle (relative L2
<= 1e-12 FP64, <= 1e-5 mixed), the hybridization cutoff, FP64 trajectories
with every sweep bit-exact, shadow mode over a longer run, and the full-size
1,000,000-bead solution."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import both, copy_oracle_from_gpu, perturbed, rel_l2, forces_close, same_topology, topo_diff

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_4214_amd  # noqa: F401  (fails loudly without the built library)


def _solution(n_duplex=30, n_bp=10, n_total=3000, seed=5, **kw):
    return synth.dna1_solution(n_duplex, n_bp, n_total, 3.0, seed, seed + 10, **kw)


def _wrapped_diff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_forces_match_oracle(precision, tol):
    s = perturbed(_solution(), 0.06, 1)
    g, o = both(s, synth.ff_dna1(), synth.rules_fig2(), precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_hybridization_cutoff(precision, tol):
    """Strands 0.95 apart with jitter: part of the hybridization bonds are longer
    than the 1.0 cutoff and must feel no force."""
    s = perturbed(_solution(seed=7, hyb=0.95), 0.08, 2)
    ff = synth.ff_dna1()
    g, o = both(s, ff, synth.RuleSet(every=0), precision=precision, generate=False)
    hb = s.bonds[s.bonds[:, 2] == synth.H_BOND]
    d = _wrapped_diff(s.x[hb[:, 0]], s.x[hb[:, 1]], s.L)
    r = np.sqrt((d * d).sum(axis=1))
    assert (r > 1.0).sum() > 10 and (r < 1.0).sum() > 10
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


@pytest.mark.parametrize("precision,tol", [(0, 1e-11), (1, 1e-5)])
def test_energy_matches_oracle(precision, tol):
    """Bond energies carry the wells' offsets (-U_min per bond at the well)."""
    s = perturbed(_solution(seed=8), 0.05, 3)
    g, o = both(s, synth.ff_dna1(), synth.rules_fig2(), precision=precision)
    eg, eo = g.energy(), o.energy()
    for k in range(6):
        assert abs(eg[k] - eo[k]) <= tol * max(abs(eo[k]), 1.0), (k, eg[k], eo[k])


def test_trajectory_fp64_every_step_sweep():
    """Twenty steps, each with a sweep (melting, re-hybridization, angle and
    dihedral generation and purge): positions, velocities, topology."""
    s = perturbed(_solution(seed=9), 0.05, 4)
    g, o = both(s, synth.ff_dna1(), synth.rules_fig2(), seed=13)
    killed = 0
    for _ in range(4):
        g.step(5)
        o.step(5)
        so, _, _ = o.stats()
        killed += so["bonds_killed"]
        assert same_topology(g, o), topo_diff(g, o)
    xg, vg = g.state()
    xo, vo = o.state()
    assert np.abs(_wrapped_diff(xg, xo, s.L)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    assert o.counts()[0] < len(s.bonds)


def test_shadow_mode_ligation_and_rehybridization():
    """Single strands (no hybridization bonds) at T = 1: the GPU runs, and at
    every block the oracle, started from the GPU's state, takes the sweep; both
    sweeps must agree.  Complementary strands hybridize and strand ends ligate."""
    import paper_1108_4214_amd as pk
    s = _solution(n_duplex=40, n_bp=6, n_total=2400, seed=11)
    s.bonds = s.bonds[s.bonds[:, 2] != synth.H_BOND]
    ff, rules = synth.ff_dna1(), synth.rules_fig2()
    g = pk.System(s.n, s.L, 17).configure(s, ff, rules)
    created = 0
    for blk in range(30):
        g.step(3)
        o = copy_oracle_from_gpu(g, s, ff, rules, seed=17, step=g.stats()["steps"])
        o.sweep_now()
        g.sweep_now()
        assert same_topology(g, o), (blk, topo_diff(g, o))
        so, _, _ = o.stats()
        created += so["bonds_created"]
    assert created > 5
    assert g.counts()[0] > len(s.bonds) + 50


def test_well_rejects_bad_arguments():
    import paper_1108_4214_amd as pk
    s = _solution(n_total=3000)
    g = pk.System(s.n, s.L, 1).configure(s, synth.ff_dna1(), synth.rules_fig2())
    for args in ((0, 1.0, 0.6, 1.0, 1.0), (32, 1.0, 0.6, 1.0, 1.0), (1, 1.0, 0.6, 0.6, 1.0), (1, 1.0, 0.6, 1.0, 0.0),
                 (1, float("nan"), 0.6, 1.0, 1.0)):
        with pytest.raises(pk.DynBondError):
            pk.db_bond_well(g.ctx, *args)


# ---- full size: 1,000,000 beads --------------------------------------------------------------

@pytest.fixture(scope="module")
def dna1_workload():
    w = synth.dna1_c3()
    s = perturbed(w.system, 0.03, 6)
    o = oracle.Oracle.from_system(s, w.ff, w.rules, seed=w.seed)
    return w, s, o, o.forces()


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_full_size_forces(precision, tol, dna1_workload):
    import paper_1108_4214_amd as pk
    w, s, _, fo = dna1_workload
    g = pk.System(s.n, s.L, w.seed, precision).configure(s, w.ff, w.rules)
    ok, msg = forces_close(g.forces(), fo, tol)
    assert ok, msg


def test_full_size_three_swept_steps(dna1_workload):
    import paper_1108_4214_amd as pk
    w, s, o, _ = dna1_workload
    g = pk.System(s.n, s.L, w.seed, 0).configure(s, w.ff, w.rules)
    g.step(3)
    o.step(3)
    assert same_topology(g, o), topo_diff(g, o)
    assert np.abs(_wrapped_diff(g.state()[0], o.state()[0], s.L)).max() < 1e-9

