"""Parity of the HIP path with the FP64 oracle on identical seeded inputs:
forces (relative L2 <= 1e-12 in FP64, <= 1e-5 mixed), energies, the initial
pattern enumeration and every sweep (bond / angle / dihedral lists bit-exact,
statistics equal), short trajectories, shadow mode over longer runs, error
paths and determinism."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import (both, copy_oracle_from_gpu, fig2_dynamic_setup, fig2_rules, perturbed, rel_l2, forces_close,
                        same_topology, topo_diff)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_4214_amd  # noqa: F401  (fails loudly without the built library)


def _duplex_system(n_duplex, n_bp, rho, seed, scale=0.05):
    s = synth.duplex_box(n_duplex, n_bp, rho, seed, seed + 10)
    return perturbed(s, scale, seed)


# ---- forces and energies ---------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
@pytest.mark.parametrize("n_duplex,n_bp,rho", [(1, 3, 0.01), (37, 7, 0.3), (150, 12, 0.3)])
def test_forces_match_oracle(precision, tol, n_duplex, n_bp, rho):
    s = _duplex_system(n_duplex, n_bp, rho, seed=n_duplex)
    ff = synth.ff_t2()
    ff.angles = {1: (10.0, 2.6)}   # off the straight angle so every angle term is active
    g, o = both(s, ff, synth.rules_t2(), precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


@pytest.mark.parametrize("precision", [0, 1])
def test_forces_paper_exclusion_depth_two(precision):
    s = _duplex_system(20, 6, 0.2, seed=5)
    ff = synth.ff_t2()
    ff.exclude_depth = 2
    g, o = both(s, ff, synth.rules_t2(), precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), (FP64_TOL if precision == 0 else MIXED_TOL))
    assert ok, msg


def test_forces_fig2_model_dihedral_phases():
    s, ff, rules = fig2_dynamic_setup()
    ff.dihedrals = {1: (1.0, 0.3), 2: (1.0, -1.1), 3: (1.0, math.pi)}
    lad = synth.ladder_1bead(9)
    lad = perturbed(lad, 0.1, 3)
    g, o = both(lad, ff, rules)
    ok, msg = forces_close(g.forces(), o.forces(), FP64_TOL)
    assert ok, msg


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_forces_wide_bonded_neighbourhood(precision, tol):
    """Hubs and arms reach nine distinct beads through their bonded terms, more
    than the per-bead halo holds, so they take the per-entry path while the leaves
    take the halo path; both must match the oracle."""
    s = synth.branched_clusters(27, seed=4)
    ff = synth.ForceField(bonds={1: (30.0, 1.0)}, angles={1: (5.0, 1.9)}, dihedrals={1: (2.0, 0.4)})
    g, o = both(s, ff, synth.RuleSet(), precision=precision, generate=False)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


@pytest.mark.parametrize("precision", [0, 1])
def test_energy_matches_oracle(precision):
    s = _duplex_system(37, 7, 0.3, seed=2)
    ff = synth.ff_t2()
    g, o = both(s, ff, synth.rules_t2(), precision=precision)
    eg, eo = g.energy(), o.energy()
    tol = 1e-11 if precision == 0 else 2e-5
    for k in range(6):
        assert abs(eg[k] - eo[k]) <= tol * max(1.0, abs(eo[k])), (k, eg[k], eo[k])


# ---- topology: initial enumeration -------------------------------------------------------

def test_generation_t2_duplexes():
    s = _duplex_system(30, 9, 0.2, seed=4)
    g, o = both(s, synth.ff_t2(), synth.rules_t2())
    assert same_topology(g, o), topo_diff(g, o)
    nb, na, nd = g.counts()
    assert na == 30 * (2 * 7 + 2 * 9) and nd == 30 * 2 * 8


@pytest.mark.parametrize("n", [2, 3, 8])
def test_generation_fig2_ladder(n):
    lad = synth.ladder_1bead(n)
    g, o = both(lad, synth.ForceField(), fig2_rules())
    assert same_topology(g, o), topo_diff(g, o)


def test_explicit_angle_lists_round_trip():
    s = _duplex_system(3, 5, 0.05, seed=9)
    o = oracle.Oracle.from_system(s, synth.ff_t2(), synth.rules_t2(), seed=1)
    s.angles = o.angles()
    s.dihedrals = o.dihedrals()
    import paper_1108_4214_amd as pk
    g = pk.System(s.n, s.L, 1).configure(s, synth.ff_t2(), synth.rules_t2())
    assert np.array_equal(g.angles(), o.angles()) and np.array_equal(g.dihedrals(), o.dihedrals())


# ---- the sweep on single snapshots -------------------------------------------------------

def _sweep_both(system, ff, rules, seed=11, step=0):
    g, o = both(system, ff, rules, seed=seed)
    g.set_step(step)
    o.set_step(step)
    g.sweep_now()
    o.sweep_now()
    return g, o


def _stats_equal(g, o):
    sg = g.stats()
    so, _, _ = o.stats()
    return all(sg[k] == so[k] for k in so)


@pytest.mark.parametrize("p", [0.1, 0.5, 1.0])
def test_sweep_isolated_pairs(p):
    s = synth.isolated_pairs(3000, 1.0, seed=3)
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, p), ("maxbond", 1, 0, 1)])
    g, o = _sweep_both(s, synth.ForceField(), rules, step=17)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)


@pytest.mark.parametrize("p", [0.1, 0.6])
def test_sweep_averaged_acceptance(p):
    """The appendix's literal acceptance (mean of one uniform per bead) on creations
    and breaks in one sweep: bit-exact against the oracle."""
    s = synth.random_gas(2500, 14.0, seed=7, n_types=4)
    s.bonds = np.array([(2 * k, 2 * k + 1, 1, 1) for k in range(300)], dtype=np.int32)
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, p), ("create", 1, 3, 4, 1.5, p),
                                          ("break", 1, 1.2, p), ("maxbond", 1, 0, 1)], accept="average")
    g, o = _sweep_both(s, synth.ForceField(), rules, seed=3, step=23)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert g.stats()["bonds_created"] > 5 and g.stats()["bonds_broken"] > 0


@pytest.mark.parametrize("L", [1000.0, 4000.0])
def test_sweep_large_box_pairs_at_the_creation_distance(L):
    """Pairs 1e-7 inside and outside the creation distance straddling the faces,
    edges and a corner of a large box, where float copies of the coordinates are
    coarse: every inside pair bonds and no outside pair does, as in the oracle.
    (A prefilter margin that does not grow with the box edge drops inside pairs at
    L = 4000.)"""
    r = 1.5
    s = synth.boundary_pairs(3000, r * (1 - 1e-7), r * (1 + 1e-7), L, seed=int(L))
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, r, 1.0), ("maxbond", 1, 0, 1)])
    g, o = _sweep_both(s, synth.ForceField(), rules, seed=2, step=1)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert g.stats()["bonds_created"] == 1500


@pytest.mark.parametrize("L,n", [(3.0, 30), (4.2, 60)])
def test_sweep_small_grid(L, n):
    """Boxes of one and two cells per edge, where the scan visits every cell once
    (and the creation scan splits the cells over its lanes): a sweep against the
    oracle, with creations, breaks and maxbond."""
    s = synth.random_gas(n, L, seed=5, n_types=2)
    s.bonds = np.array([(0, 1, 1, 1), (2, 3, 1, 1)], dtype=np.int32)
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 0.8), ("break", 1, 1.2, 0.6),
                                          ("maxbond", 1, 0, 2)])
    g, o = _sweep_both(s, synth.ForceField(), rules, step=11)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert o.counts()[0] > 2


@pytest.mark.parametrize("seed", [1, 2])
def test_sweep_dense_gas_with_bonds(seed):
    s = synth.random_gas(2500, 14.0, seed=seed, n_types=4)
    s.bonds = np.array([(2 * k, 2 * k + 1, 1, 1) for k in range(300)], dtype=np.int32)
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 0.7), ("create", 1, 3, 4, 1.5, 0.7),
                                          ("break", 1, 1.2, 0.6), ("maxbond", 1, 0, 1)])
    g, o = _sweep_both(s, synth.ForceField(), rules, seed=seed, step=40)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert g.stats()["bonds_created"] > 50 and g.stats()["bonds_broken"] > 10


@pytest.mark.parametrize("n", [100_000, 200_000, 300_000, 600_000])
def test_sweep_long_creation_list(n):
    """A dense gas whose unbonded beads all nominate: about 1e5, 2e5, 3e5 and 6e5
    listed beads, where the creation scan runs 8, 4, 2 and 1 threads per bead (the
    thread count follows the list's length); nominations, acceptances and
    statistics bit-exact against the oracle."""
    L = 14.0 * (n / 2500.0) ** (1.0 / 3.0)
    s = synth.random_gas(n, L, seed=n // 1000, n_types=4)
    s.bonds = np.array([(2 * k, 2 * k + 1, 1, 1) for k in range(300)], dtype=np.int32)
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 0.7), ("create", 1, 3, 4, 1.5, 0.7),
                                          ("break", 1, 1.2, 0.6), ("maxbond", 1, 0, 1)])
    g, o = _sweep_both(s, synth.ForceField(), rules, seed=4, step=9)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert g.stats()["bonds_created"] > n // 20


def test_topology_energy_ledger():
    """The ledger is the change of the potential energy across a sweep at fixed
    positions: the oracle's energies before and after the same sweep."""
    import paper_1108_4214_amd as pk
    s = synth.random_gas(900, 11.0, seed=3, n_types=4, min_dist=0.85)
    s.bonds = np.array([(2 * k, 2 * k + 1, 1, 1) for k in range(120)], dtype=np.int32)
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 0.7), ("create", 1, 3, 4, 1.5, 0.7),
                                          ("break", 1, 1.2, 0.6), ("maxbond", 1, 0, 1)])
    ff = synth.ForceField(bonds={1: (20.0, 1.0)})
    g, o = both(s, ff, rules, seed=5)
    pk.db_track_topology_energy(g.ctx, 1)
    g.set_step(40)
    o.set_step(40)
    e0 = np.asarray(o.energy())
    g.sweep_now()
    o.sweep_now()
    e1 = np.asarray(o.energy())
    assert same_topology(g, o), topo_diff(g, o)
    du = float(np.sum(e1[1:5] - e0[1:5]))
    st = g.stats()
    assert st["bonds_created"] > 10 and st["bonds_broken"] > 0
    assert abs(du) > 1.0
    assert abs(st["du_topo_last"] - du) <= 1e-9 * max(1.0, float(np.abs(e0[1:5]).sum()))
    assert st["du_topo_cum"] == st["du_topo_last"]


def test_sweep_kill_and_purge_on_stretched_duplexes():
    s = _duplex_system(40, 8, 0.1, seed=6, scale=0.35)
    rules = synth.rules_t2(p=0.5, every=1, r_kill=1.4)
    g, o = _sweep_both(s, synth.ff_t2(), rules, step=3)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert g.stats()["bonds_killed"] > 5 and g.stats()["angles_removed"] > 10


def test_sweep_conversion():
    s = _duplex_system(40, 6, 0.1, seed=8, scale=0.3)
    rules = synth.rules_t2(p=0.9, every=1, convert=True)
    rules.rules.insert(0, ("angle", 2, (5, 0, 0), (synth.mask(4), synth.mask(5))))
    g, o = _sweep_both(s, synth.ff_t2(weak=True), rules, step=5)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)
    assert g.stats()["bonds_converted"] > 5


def test_sweep_fig2_rules_paircheck_and_createdir():
    s, ff, rules = fig2_dynamic_setup(n_strand=60, L=7.0)
    g, o = _sweep_both(s, ff, rules, step=2)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)


def test_sweep_shadowing_and_paircheck13():
    s = synth.random_gas(1500, 11.0, seed=12, n_types=4)
    s.bonds = np.array([(3 * k, 3 * k + 1, 4, 4) for k in range(200)] +
                       [(3 * k + 1, 3 * k + 2, 4, 4) for k in range(200)], dtype=np.int32)
    rules = synth.RuleSet(every=1, paircheck13=1, rules=[("create", 1, 1, 2, 1.5, 1.0), ("create", 2, 1, 2, 1.1, 0.3),
                                                         ("createdir", 2, 3, 3, 4, 1.3, 0.8)])
    g, o = _sweep_both(s, synth.ForceField(), rules, step=9)
    assert same_topology(g, o), topo_diff(g, o)
    assert _stats_equal(g, o)


# ---- trajectories ------------------------------------------------------------------------

def test_short_trajectory_fp64():
    s = synth.single_strands(24, 6, L=11.0, seed_w=3, seed_d=4)
    rules = synth.rules_t2(p=0.7, every=5, r_kill=1.35)
    ff = synth.ff_t2()
    g, o = both(s, ff, rules, seed=9)
    g.step(20)
    o.step(20)
    xg, vg = g.state()
    xo, vo = o.state()
    d = xg - xo
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    assert same_topology(g, o), topo_diff(g, o)


@pytest.mark.parametrize("skin", [0.2, 0.55])
def test_list_kept_across_every_step_sweeps(skin):
    """WCA with a sweep every step: the list is kept while the summed speed bound
    since its full build allows, the changed beads' lists are redone after each
    sweep, and the trajectory still follows the oracle (every position to 1e-9
    after 40 steps; this dilute Langevin system diverges far more slowly than the
    dense DPD solution)."""
    import paper_1108_4214_amd as pk
    s = synth.single_strands(24, 6, L=11.0, seed_w=5, seed_d=6)
    rules = synth.rules_t2(p=0.7, every=1, r_kill=1.35)
    ff = synth.ff_t2()
    g = pk.System(s.n, s.L, 9)
    pk.db_tune(g.ctx, skin, 8)
    g.configure(s, ff, rules)
    o = oracle.Oracle.from_system(s, ff, rules, seed=9)
    for _ in range(8):
        g.step(5)
        o.step(5)
        assert same_topology(g, o), topo_diff(g, o)
    xg, vg = g.state()
    xo, vo = o.state()
    d = xg - xo
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    st = g.stats()
    assert st["list_patches"] > 0 and st["cum_bonds_created"] > 0


@pytest.mark.parametrize("permute_every", [1, 3])
def test_rollback_reruns_the_block(permute_every):
    """A skin far too thin for the speeds forces the scheduler to restore the
    block's input state and re-run it with a fresh list every step (the state is
    kept by the reorder when it runs, else by the block's first step kernel); the
    trajectory must still be the oracle's."""
    import paper_1108_4214_amd as pk
    s = synth.single_strands(24, 6, L=11.0, seed_w=3, seed_d=4, T=2.0)
    rules = synth.rules_t2(p=0.7, every=5, r_kill=1.35)
    ff = synth.ff_t2(T0=2.0, T1=2.0)
    g, o = both(s, ff, rules, seed=9)
    pk.db_tune(g.ctx, 0.02, permute_every)
    g.step(20)
    o.step(20)
    assert g.stats()["rollbacks"] > 0
    xg, vg = g.state()
    xo, vo = o.state()
    d = xg - xo
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    assert same_topology(g, o), topo_diff(g, o)


def test_shadow_mode_dynamic_run():
    s = synth.single_strands(24, 6, L=11.0, seed_w=3, seed_d=4)
    rules = synth.rules_t2(p=0.7, every=2, r_kill=1.35)
    ff = synth.ff_t2()
    import paper_1108_4214_amd as pk
    g = pk.System(s.n, s.L, 9).configure(s, ff, rules)
    events = 0
    for blk in range(60):
        g.step(2)                       # ends just before the next sweep step
        step = g.stats()["steps"]
        o = copy_oracle_from_gpu(g, s, ff, rules, seed=9, step=step)
        o.sweep_now()
        g.sweep_now()
        assert same_topology(g, o), (blk, topo_diff(g, o))
        so, _, _ = o.stats()
        events += so["bonds_created"] + so["bonds_killed"]
    assert events > 20


def test_shadow_mode_fig2_model():
    s, ff, rules = fig2_dynamic_setup()
    rules.every = 3
    import paper_1108_4214_amd as pk
    g = pk.System(s.n, s.L, 21).configure(s, ff, rules)
    events = 0
    for blk in range(40):
        g.step(3)
        step = g.stats()["steps"]
        o = copy_oracle_from_gpu(g, s, ff, rules, seed=21, step=step)
        o.sweep_now()
        g.sweep_now()
        assert same_topology(g, o), (blk, topo_diff(g, o))
        so, _, _ = o.stats()
        events += so["bonds_created"] + so["bonds_killed"] + so["dihedrals_created"]
    assert events > 20


def test_determinism_two_runs_bitwise():
    s = _duplex_system(60, 10, 0.3, seed=13)
    import paper_1108_4214_amd as pk
    out = []
    for _ in range(2):
        g = pk.System(s.n, s.L, 5).configure(s, synth.ff_t2(), synth.rules_t2(p=0.5, every=10))
        g.step(50)
        x, v = g.state()
        out.append((x, v, g.bonds(), g.angles(), g.dihedrals()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_nve_drift_mixed_vs_fp64():
    s = _duplex_system(40, 8, 0.3, seed=14, scale=0.02)
    ff = synth.ff_t2(gamma=0.0, dt=0.002)
    import paper_1108_4214_amd as pk
    drift = []
    for prec in (0, 1):
        g = pk.System(s.n, s.L, 5, prec).configure(s, ff, synth.rules_t2(every=0))
        e0 = g.energy()
        g.step(500)
        e1 = g.energy()
        drift.append(abs(e1[:5].sum() - e0[:5].sum()) / s.n)
    assert drift[0] < 1e-3 and drift[1] < 1e-3, drift


# ---- edge cases and error paths -----------------------------------------------------------

def test_tiny_systems():
    import paper_1108_4214_amd as pk
    for n in (1, 2):
        s = synth.random_gas(n, 5.0, seed=1)
        g, o = both(s, synth.ForceField(), synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0)]))
        assert rel_l2(g.forces() + 1e-300, o.forces() + 1e-300) <= 1e-12 or np.allclose(g.forces(), o.forces())
        g.step(3)
        o.step(3)
        assert np.allclose(g.state()[0], o.state()[0], atol=1e-10)
    g = pk.System(0, 5.0, 1)
    g.configure(synth.random_gas(0, 5.0), synth.ForceField(), None)
    g.step(2)
    assert g.counts() == (0, 0, 0)


def test_bond_capacity_overflow_is_reported():
    import paper_1108_4214_amd as pk
    # bead 0 already holds four bonds; a creation rule without maxbond would add a fifth
    pos = [[5, 5, 5], [6, 5, 5], [4, 5, 5], [5, 6, 5], [5, 4, 5], [5, 5, 6.2]]
    x = np.array(pos, dtype=float)
    s = synth.System(L=12.0, x=x, v=np.zeros_like(x), type=np.array([1, 5, 5, 5, 5, 2], dtype=np.int32),
                     reactive=np.ones(6, dtype=np.uint8),
                     bonds=np.array([(0, k, 4, 4) for k in range(1, 5)], dtype=np.int32))
    g = pk.System(s.n, s.L, 1).configure(s, synth.ForceField(eps=0.0),
                                         synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0)]))
    with pytest.raises(pk.DynBondError) as e:
        g.sweep_now()
    assert e.value.code == pk.DB_ECAPACITY


def test_list_overflow_is_reported():
    """A clump at density about 17: the central beads have some 300 beads within the
    list cutoff, more than the 128 a list holds.  The list build keeps the first 128,
    flags the overflow, and the step reports DB_ECAPACITY (WCA at zero strength, so
    nothing else goes wrong)."""
    import paper_1108_4214_amd as pk
    rng = np.random.default_rng(41)
    n, L = 300, 20.0
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = 10.0 + d * 1.6 * rng.uniform(size=(n, 1)) ** (1.0 / 3.0)
    s = synth.System(L=L, x=x, v=np.zeros_like(x), type=np.ones(n, dtype=np.int32),
                     reactive=np.zeros(n, dtype=np.uint8), bonds=np.zeros((0, 4), dtype=np.int32))
    with pytest.raises(pk.DynBondError) as e:
        g = pk.System(s.n, s.L, 3).configure(s, synth.ForceField(eps=0.0), synth.RuleSet(every=0))
        g.step(1)
    assert e.value.code == pk.DB_ECAPACITY


def test_invalid_arguments_rejected():
    import paper_1108_4214_amd as pk
    g = pk.System(4, 10.0, 1)
    with pytest.raises(pk.DynBondError):
        pk.db_set_state(g.ctx, np.full((4, 3), 11.0), None, np.ones(4, np.int32))
    with pytest.raises(pk.DynBondError):
        pk.db_bond_create(g.ctx, 1, 1, 2, 1.5, 1.5)
    with pytest.raises(pk.DynBondError):
        pk.db_step(g.ctx, 1)   # no state yet


# ---- full-size workload (1,000,000 beads): forces and one sweep against the oracle -------

@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_full_size_c3_forces(precision, tol, c3_workload):
    w = c3_workload
    g, o = both(w.system, w.ff, w.rules, seed=w.seed, precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


def test_full_size_c3_sweep(c3_workload):
    w = c3_workload
    s = perturbed(w.system, 0.25, 1)   # stretch some hybridization bonds past the kill distance
    g, o = _sweep_both(s, w.ff, w.rules, seed=w.seed, step=0)
    assert same_topology(g, o)
    assert _stats_equal(g, o)


@pytest.fixture(scope="module")
def c3_workload():
    return synth.c3()


# ---- full-size stress workload (4,000,000 beads, sweep every step, conversion) ----------

@pytest.fixture(scope="module")
def c5_workload():
    return synth.c5()


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_full_size_c5_forces(precision, tol, c5_workload):
    w = c5_workload
    g, o = both(w.system, w.ff, w.rules, seed=w.seed, precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg
    g.close()


def test_full_size_c5_steps_with_sweeps_and_conversion(c5_workload):
    """Three NVE steps with a sweep before each: creations on the first (about 450k
    bonds and 900k angles), then creations, breaks and conversions; FP64 trajectory
    and every list against the oracle."""
    w = c5_workload
    g, o = both(w.system, w.ff, w.rules, seed=w.seed, precision=0)
    g.step(3)
    o.step(3)
    assert same_topology(g, o)
    assert _stats_equal(g, o)
    st = g.stats()
    assert st["cum_bonds_created"] > 400000
    xg, vg = g.state()
    xo, vo = o.state()
    d = xg - xo
    d -= w.system.L * np.round(d / w.system.L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    g.close()


def test_dense_cluster_sweep():
    # a dense clump in a dilute box: crowded cells (about 40 beads each) next to empty ones
    rng = np.random.default_rng(31)
    n_clump, n_gas, L = 2600, 400, 16.0
    x = np.concatenate([rng.uniform(5.0, 8.2, size=(n_clump, 3)), rng.uniform(0, L, size=(n_gas, 3))])
    s = synth.System(L=L, x=synth.wrap(x, L), v=np.zeros((n_clump + n_gas, 3)),
                     type=rng.integers(1, 5, size=n_clump + n_gas).astype(np.int32),
                     reactive=np.ones(n_clump + n_gas, dtype=np.uint8), bonds=np.zeros((0, 4), dtype=np.int32))
    rules = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 0.8), ("create", 1, 3, 4, 1.5, 0.8),
                                          ("maxbond", 1, 0, 1)])
    g, o = _sweep_both(s, synth.ForceField(eps=0.01), rules, seed=4, step=1)
    assert same_topology(g, o), topo_diff(g, o)
    assert g.stats()["bonds_created"] > 100


def test_dense_slab_forces():
    # a slab three cells thick at density 2.2: long cell runs, up to about 55 list
    # neighbours per bead with the 0.4 skin (the list holds 64)
    rng = np.random.default_rng(32)
    L, n = 30.0, 9000
    x = np.column_stack([rng.uniform(0, L, n), rng.uniform(0, L, n), rng.uniform(10.0, 14.6, n)])
    s = synth.System(L=L, x=synth.wrap(x, L), v=np.zeros((n, 3)), type=np.ones(n, dtype=np.int32),
                     reactive=np.ones(n, dtype=np.uint8), bonds=np.zeros((0, 4), dtype=np.int32))
    import paper_1108_4214_amd as pk
    g = pk.System(s.n, s.L, 7)
    pk.db_tune(g.ctx, 0.4, 1)      # list cutoff 1.52: under 64 neighbours at this density
    g.configure(s, synth.ForceField(eps=0.01), synth.RuleSet(every=0))
    o = oracle.Oracle.from_system(s, synth.ForceField(eps=0.01), synth.RuleSet(every=0), seed=7)
    ok, msg = forces_close(g.forces(), o.forces(), FP64_TOL)
    assert ok, msg


# ---- brick tiles of the step kernel against the per-bead kernel -------------------------

def _run_shape(s, ff, rules, precision, enable, edge, steps, seed=5):
    import paper_1108_4214_amd as pk
    g = pk.System(s.n, s.L, seed, precision)
    pk.db_tile_shape(g.ctx, enable, edge)
    g.configure(s, ff, rules)
    g.step(steps)
    x, v = g.state()
    out = (x, v, g.bonds(), g.angles(), g.dihedrals(), g.stats())
    g.close()
    return out


@pytest.mark.parametrize("precision,steps,xtol", [(0, 60, 1e-9), (1, 20, 1e-6)])
@pytest.mark.parametrize("edge", [0, 3, 12])
def test_tile_kernel_trajectory_matches_per_bead_kernel(precision, steps, xtol, edge):
    """The tile step kernel stages each tile's partners in LDS as images next to the
    tile, so its separations are differences of stored positions rather than
    minimum images of differences: the same values to rounding.  With sweeps that
    kill and re-create bonds, its trajectory follows the per-bead kernel's to xtol
    and the topology is the same.  Edge 12 makes regions too large to stage (those
    tiles read partners from memory); 3 gives small bricks; 0 the density's choice."""
    s = _duplex_system(150, 12, 0.3, seed=21, scale=0.06)
    rules = synth.rules_t2(p=0.6, every=4, r_kill=1.3)
    ff = synth.ff_t2()
    a = _run_shape(s, ff, rules, precision, 1, edge, steps)
    b = _run_shape(s, ff, rules, precision, 0, 0, steps)
    d = a[0] - b[0]
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < xtol
    assert np.abs(a[1] - b[1]).max() < 1e3 * xtol
    for k in (2, 3, 4):
        assert np.array_equal(a[k], b[k])
    assert a[5]["cum_bonds_killed"] > 0 and a[5]["cum_bonds_created"] > 0


def test_tile_kernel_trajectory_against_oracle():
    """Duplexes in a box of several tiles, FP64, 30 steps with sweeps every 5 steps:
    the tile kernel's positions against the oracle's to 1e-9, topology bit-exact."""
    s = _duplex_system(60, 10, 0.3, seed=23, scale=0.05)
    rules = synth.rules_t2(p=0.6, every=5, r_kill=1.3)
    ff = synth.ff_t2()
    import paper_1108_4214_amd as pk
    g, o = both(s, ff, rules, seed=9)
    pk.db_tile_shape(g.ctx, 1, 0)
    g.step(30)
    o.step(30)
    assert same_topology(g, o), topo_diff(g, o)
    d = g.state()[0] - o.state()[0]
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-9
    assert pk.db_tile_stats(g.ctx)["staged"] > 0


def test_tile_kernel_wide_bonded_neighbourhood():
    """Hubs whose bonded terms reach more beads than the halo holds, next to beads
    on the halo path, inside tiles: the trajectory follows the per-bead kernel's."""
    s = synth.branched_clusters(64, seed=4)
    ff = synth.ForceField(bonds={1: (30.0, 1.0)}, angles={1: (5.0, 1.9)}, dihedrals={1: (2.0, 0.4)}, gamma=1.0)
    outs = []
    for enable in (1, 0):
        import paper_1108_4214_amd as pk
        g = pk.System(s.n, s.L, 3, 1)
        pk.db_tile_shape(g.ctx, enable, 0)
        g.configure(s, ff, synth.RuleSet(), generate=False)
        g.step(25)
        outs.append(g.state())
        g.close()
    d = outs[0][0] - outs[1][0]
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-6 and np.abs(outs[0][1] - outs[1][1]).max() < 1e-4


def test_tile_shape_arguments():
    import paper_1108_4214_amd as pk
    g = pk.System(4, 10.0, 1)
    with pytest.raises(pk.DynBondError):
        pk.db_tile_shape(g.ctx, 2, 0)
    with pytest.raises(pk.DynBondError):
        pk.db_tile_shape(g.ctx, 1, -1)


# ---- HIP graphs ------------------------------------------------------------------------

def _graph_run(s, ff, rules, precision, graph, checkpoints, seed=7, tiles=0, batch_of=None):
    import paper_1108_4214_amd as pk
    g = pk.System(s.n, s.L, seed, precision)
    pk.db_graph(g.ctx, graph)
    pk.db_tile_shape(g.ctx, tiles, 0)
    g.configure(s, ff, rules)
    out = []
    done = 0
    for k in checkpoints:
        g.step(k - done)
        done = k
        out.append(g.state())
    out.append((g.bonds(), g.angles(), g.dihedrals()))
    g.close()
    return out


@pytest.mark.parametrize("precision,tiles", [(0, 0), (1, 0), (1, 1)])
def test_graph_replays_equal_eager_launches(precision, tiles):
    """Blocks replayed from captured graphs (several lengths, rollback copies, both
    buffer parities, sweeps and list rebuilds in between) give the trajectory of the
    launches issued one by one, bit for bit, at every checkpoint."""
    s = _duplex_system(40, 8, 0.3, seed=31, scale=0.05)
    rules = synth.rules_t2(p=0.6, every=7, r_kill=1.3)
    ff = synth.ff_t2()
    cps = [3, 10, 25, 60, 100, 140]
    a = _graph_run(s, ff, rules, precision, 1, cps, tiles=tiles)
    b = _graph_run(s, ff, rules, precision, 0, cps, tiles=tiles)
    for (xa, va), (xb, vb) in zip(a[:-1], b[:-1]):
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    for ta, tb in zip(a[-1], b[-1]):
        assert np.array_equal(ta, tb)


def test_graph_replays_dpd_and_batch():
    """The DPD velocity double buffer and a batch of replicas under graph replay."""
    import paper_1108_4214_amd as pk
    s = synth.dpd_solution(16, 6, 4000, 3.0, 7, 17)
    ff = synth.ff_dpd()
    rules = synth.rules_t2(p=0.5, every=5)
    a = _graph_run(s, ff, rules, 0, 1, [4, 17, 40])
    b = _graph_run(s, ff, rules, 0, 0, [4, 17, 40])
    for (xa, va), (xb, vb) in zip(a[:-1], b[:-1]):
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    outs = []
    for graph in (1, 0):
        reps = []
        for r, (nd, nbp, rho, T) in enumerate(((12, 8, 0.3, 0.8), (8, 6, 0.2, 1.2))):
            sr = perturbed(synth.duplex_box(nd, nbp, rho, 70 + r, 80 + r, T=T), 0.05, 70 + r)
            g = pk.System(sr.n, sr.L, 90 + r).configure(sr, synth.ff_t2(T0=T, T1=T), synth.rules_t2(p=0.7, every=5))
            pk.db_set_reactive(g.ctx, sr.reactive)
            reps.append(g)
        bt = pk.Batch(reps)
        pk.db_graph(bt.ctx, graph)
        bt.step(23)
        outs.append([bt.replica_state(r) for r in range(2)])
        bt.step(31)
        outs[-1] += [bt.replica_state(r) for r in range(2)]
        bt.close()
        for g in reps:
            g.close()
    for (xa, va), (xb, vb) in zip(outs[0], outs[1]):
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
