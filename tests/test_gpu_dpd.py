"""DPD pair forces and pair thermostat (section 3) on the HIP path against the
FP64 oracle: conservative forces (relative L2 <= 1e-12 in FP64, <= 1e-5 mixed),
energies, FP64 trajectories with the pair thermostat and the hybridization sweep,
the exact pairwise cancellation of the thermostat forces (momentum), the
temperature the thermostat holds, rollback with the velocity double buffer,
batches, and the full-size 1,000,000-bead solution at density 3."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import both, perturbed, rel_l2, forces_close, same_topology, topo_diff

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_4214_amd  # noqa: F401  (fails loudly without the built library)


def _solution(n_duplex=20, n_bp=10, n_total=6000, seed=3, T=1.0):
    return synth.dpd_solution(n_duplex, n_bp, n_total, 3.0, seed, seed + 10, T=T)


def _wrapped_diff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


# ---- forces and energies ---------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
@pytest.mark.parametrize("depth", [1, 2])
def test_conservative_forces_match_oracle(precision, tol, depth):
    s = perturbed(_solution(), 0.05, 1)
    ff = synth.ff_dpd()
    ff.exclude_depth = depth
    ff.angles = {1: (10.0, 2.6)}   # off the straight angle so the bonded terms are active too
    g, o = both(s, ff, synth.rules_t2(), precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_pure_fluid_forces_several_tiles_and_ragged_tail(precision, tol):
    s = synth.dpd_solution(0, 0, 3 * 11 ** 3 + 37, 3.0, 5, 15)
    g, o = both(s, synth.ff_dpd(), synth.RuleSet(every=0), precision=precision)
    ok, msg = forces_close(g.forces(), o.forces(), tol)
    assert ok, msg


@pytest.mark.parametrize("precision,tol", [(0, 1e-11), (1, 1e-5)])
def test_energy_matches_oracle(precision, tol):
    """Kinetic energy (taken from the full-step velocity, so it includes the
    step's dissipative and random pair forces), DPD pair energy and virial."""
    s = perturbed(_solution(seed=4), 0.05, 2)
    g, o = both(s, synth.ff_dpd(), synth.rules_t2(), precision=precision)
    eg, eo = g.energy(), o.energy()
    for k in (0, 1, 2, 5):
        assert abs(eg[k] - eo[k]) <= tol * max(abs(eo[k]), 1.0), (k, eg[k], eo[k])


def test_zero_friction_has_no_thermostat_forces():
    s = _solution(seed=6)
    ff = synth.ff_dpd(gamma_dpd=0.0)
    g, o = both(s, ff, synth.RuleSet(every=0))
    g.step(10)
    o.step(10)
    assert np.abs(_wrapped_diff(g.state()[0], o.state()[0], s.L)).max() < 1e-9


# ---- trajectories ------------------------------------------------------------------------

@pytest.mark.parametrize("gamma_dpd", [4.5, 100.0])
def test_trajectory_fp64_with_sweeps(gamma_dpd):
    """Pair thermostat, bonded terms and the hybridization sweep every 5 steps:
    positions, velocities and topology follow the oracle."""
    s = synth.dpd_solution(16, 6, 4000, 3.0, 7, 17)
    s = perturbed(s, 0.08, 7)
    ff = synth.ff_dpd(gamma_dpd=gamma_dpd)
    rules = synth.rules_t2(p=0.7, every=5, r_kill=1.3)
    g, o = both(s, ff, rules, seed=9)
    g.step(20)
    o.step(20)
    xg, vg = g.state()
    xo, vo = o.state()
    assert np.abs(_wrapped_diff(xg, xo, s.L)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    assert same_topology(g, o), topo_diff(g, o)
    so, _, _ = o.stats()
    assert so["bonds_killed"] + so["bonds_created"] > 0


@pytest.mark.parametrize("skin", [0.4, 0.5])
def test_list_kept_across_every_step_sweeps(skin):
    """With a sweep every step the Verlet list is kept while the measured
    displacement since its full build allows, and only the lists of beads whose
    exclusions a sweep changed are redone (with the cutoff widened by twice that
    displacement).  Forty steps with hundreds of bond events must still follow the
    oracle: a missed pair or a stale exclusion would show in the positions (two
    oracle runs started 1e-15 apart stay within 1e-10 here)."""
    import paper_1108_4214_amd as pk
    s = perturbed(synth.dpd_solution(16, 6, 4000, 3.0, 7, 17), 0.05, 7)
    ff, rules = synth.ff_dpd(), synth.rules_t2(p=0.7, every=1, r_kill=1.3)
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
    assert np.abs(_wrapped_diff(xg, xo, s.L)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    st = g.stats()
    assert st["list_patches"] > 0 and st["cum_bonds_created"] + st["cum_bonds_killed"] > 0


def test_trajectory_mixed_close_to_oracle():
    s = perturbed(_solution(seed=8), 0.05, 8)
    g, o = both(s, synth.ff_dpd(), synth.RuleSet(every=0), seed=4, precision=1)
    g.step(5)
    o.step(5)
    assert np.abs(_wrapped_diff(g.state()[0], o.state()[0], s.L)).max() < 1e-6


@pytest.mark.parametrize("precision", [0, 1])
def test_pair_forces_cancel_momentum_is_kept(precision):
    """Both beads of a pair form the same three terms with opposite sign, so with
    no Langevin force and no bonds the total momentum stays at its initial zero."""
    import paper_1108_4214_amd as pk
    s = synth.dpd_solution(0, 0, 8000, 3.0, 9, 19)
    g = pk.System(s.n, s.L, 3, precision).configure(s, synth.ff_dpd(), synth.RuleSet(every=0))
    p0 = g.state()[1].sum(axis=0)
    g.step(200)
    p1 = g.state()[1].sum(axis=0)
    assert np.abs(p0).max() < 1e-9
    assert np.abs(p1 - p0).max() < 1e-9


@pytest.mark.parametrize("gamma_dpd", [4.5, 100.0])
def test_thermostat_holds_the_temperature(gamma_dpd):
    """A fluid started at T = 3 relaxes to the set T = 1 (mixed path, whose
    Gaussian uses the single-precision hardware logarithm and cosine): the mean
    kinetic energy per bead is 3T/2 within 3 %."""
    import paper_1108_4214_amd as pk
    s = synth.dpd_solution(0, 0, 24000, 3.0, 10, 20, T=3.0)
    g = pk.System(s.n, s.L, 5, 1).configure(s, synth.ff_dpd(gamma_dpd=gamma_dpd), synth.RuleSet(every=0))
    g.step(1000)
    ke = []
    for _ in range(40):
        g.step(25)
        ke.append(g.energy()[0] / s.n)
    assert np.mean(ke) == pytest.approx(1.5, rel=0.03), np.mean(ke)


def test_rollback_with_velocity_double_buffer():
    """A skin too thin for the speeds makes the scheduler restore the block's
    input state; with the DPD thermostat the step writes velocities to a second
    buffer, and the restored trajectory must still be the oracle's."""
    import paper_1108_4214_amd as pk
    s = perturbed(_solution(seed=11, T=2.0), 0.05, 11)
    ff = synth.ff_dpd(T=2.0)
    g, o = both(s, ff, synth.rules_t2(p=0.7, every=5), seed=9)
    pk.db_tune(g.ctx, 0.02, 3)
    g.step(15)
    o.step(15)
    assert g.stats()["rollbacks"] > 0
    xg, vg = g.state()
    xo, vo = o.state()
    assert np.abs(_wrapped_diff(xg, xo, s.L)).max() < 1e-9
    assert np.abs(vg - vo).max() < 1e-7
    assert same_topology(g, o), topo_diff(g, o)


def test_batch_replicas_match_standalone():
    """Replicas at different temperatures: the batch forms sigma per bead from the
    replica's temperature."""
    import paper_1108_4214_amd as pk
    reps = []
    for r, (T, n) in enumerate(((0.8, 3000), (1.0, 4500), (1.3, 2400))):
        s = synth.dpd_solution(5, 6, n, 3.0, 30 + r, 40 + r, T=T)
        g = pk.System(s.n, s.L, 60 + r).configure(s, synth.ff_dpd(T=T), synth.rules_t2(p=0.5))
        pk.db_set_reactive(g.ctx, s.reactive)
        reps.append(g)
    b = pk.Batch(reps)
    b.step(20)
    for r, g in enumerate(reps):
        g.step(20)
        xb, vb = b.replica_state(r)
        xg, vg = g.state()
        assert np.max(np.abs(xb - xg)) < 1e-9
        assert np.max(np.abs(vb - vg)) < 1e-7


def test_dpd_rejects_bad_arguments():
    import paper_1108_4214_amd as pk
    s = _solution(n_duplex=10, n_bp=6, n_total=3000)
    g = pk.System(s.n, s.L, 1).configure(s, synth.ff_dpd(), synth.rules_t2())
    for args in ((25.0, -1.0, 1.0, 2), (25.0, 4.5, 0.0, 2), (25.0, 4.5, 1.0, 3), (25.0, 4.5, s.L, 2)):
        with pytest.raises(pk.DynBondError):
            pk.db_pair_dpd(g.ctx, *args)


# ---- full size: 1,000,000 beads at density 3 ------------------------------------------------

@pytest.fixture(scope="module")
def dpd_workload():
    w = synth.dpd_c3()
    o = oracle.Oracle.from_system(w.system, w.ff, w.rules, seed=w.seed)
    return w, o, o.forces()


@pytest.mark.parametrize("precision,tol", [(0, FP64_TOL), (1, MIXED_TOL)])
def test_full_size_forces(precision, tol, dpd_workload):
    import paper_1108_4214_amd as pk
    w, _, fo = dpd_workload
    s = w.system
    g = pk.System(s.n, s.L, w.seed, precision).configure(s, w.ff, w.rules)
    ok, msg = forces_close(g.forces(), fo, tol)
    assert ok, msg


def test_full_size_two_steps_with_sweep(dpd_workload):
    """Two FP64 steps (the first one sweeps) in the launch configuration the
    benchmark times; then the topology and every position against the oracle."""
    import paper_1108_4214_amd as pk
    w, o, _ = dpd_workload
    s = w.system
    g = pk.System(s.n, s.L, w.seed, 0).configure(s, w.ff, w.rules)
    g.step(2)
    o.step(2)
    assert np.abs(_wrapped_diff(g.state()[0], o.state()[0], s.L)).max() < 1e-9
    assert same_topology(g, o), topo_diff(g, o)
