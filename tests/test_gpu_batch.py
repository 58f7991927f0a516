"""Batches of independent replicas: every replica of a batch must evolve exactly
as it does alone (same forces bit for bit, same sweep decisions, trajectories
within rounding), with per-replica box edge, seed and temperature."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_4214_amd  # noqa: F401


def _replicas(precision, temps=(0.7, 1.0, 1.3), sizes=((12, 8, 0.3), (8, 6, 0.1), (40, 8, 0.3)), seed0=21):
    """Standalone systems of different sizes, densities, seeds and temperatures."""
    import paper_1108_4214_amd as pk
    out = []
    for r, ((nd, nbp, rho), T) in enumerate(zip(sizes, temps)):
        s = perturbed(synth.duplex_box(nd, nbp, rho, seed0 + r, seed0 + 10 + r, T=T), 0.05, seed0 + r)
        ff = synth.ff_t2(T0=T, T1=T)
        g = pk.System(s.n, s.L, seed0 + 100 + r, precision).configure(s, ff, synth.rules_t2(p=0.5))
        # round-trip the generated topology through the host, as the batch does, so
        # that both hold their per-bead table entries in the same order
        pk.db_set_reactive(g.ctx, s.reactive)
        out.append((s, ff, g))
    return out


def _split(a, sizes):
    return np.split(a, np.cumsum(sizes)[:-1])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_forces_equal_standalone_bitwise(precision):
    import paper_1108_4214_amd as pk
    reps = _replicas(precision)
    b = pk.Batch([g for _, _, g in reps])
    fb = _split(b.forces(), b.sizes)
    for (_, _, g), f in zip(reps, fb):
        assert np.array_equal(f, g.forces())


def test_batch_sweep_equal_standalone():
    """Creation acceptance is keyed by replica-local ids and the replica's seed."""
    import paper_1108_4214_amd as pk
    reps = []
    for r, m in enumerate((40, 70, 25)):
        s = synth.isolated_pairs(m, 1.2, seed=r)
        g = pk.System(s.n, s.L, 500 + r).configure(s, synth.ff_t2(), synth.rules_t2(p=0.5))
        reps.append((s, g))
    b = pk.Batch([g for _, g in reps])
    b.sweep_now()
    created = 0
    off = 0
    bb = b.bonds()
    for s, g in reps:
        g.sweep_now()
        mine = bb[(bb[:, 0] >= off) & (bb[:, 0] < off + s.n)].copy()
        mine[:, :2] -= off
        assert np.array_equal(mine, g.bonds())
        created += g.stats()["bonds_created"]
        off += s.n
    assert b.stats()["bonds_created"] == created > 0


def test_batch_trajectory_matches_standalone():
    import paper_1108_4214_amd as pk
    reps = _replicas(0)
    b = pk.Batch([g for _, _, g in reps])
    b.step(30)
    for r, (_, _, g) in enumerate(reps):
        g.step(30)
        xb, vb = b.replica_state(r)
        xg, vg = g.state()
        assert np.max(np.abs(xb - xg)) < 1e-9
        assert np.max(np.abs(vb - vg)) < 1e-7
    nb = sum(g.counts()[0] for _, _, g in reps)
    assert b.counts()[0] == nb


def test_batch_rejects_mismatched_physics_and_state_setters():
    import paper_1108_4214_amd as pk
    s = synth.duplex_box(5, 6, 0.2, 3, 13)
    g1 = pk.System(s.n, s.L, 1).configure(s, synth.ff_t2(), synth.rules_t2())
    ff = synth.ff_t2()
    ff.dt = 0.004
    g2 = pk.System(s.n, s.L, 2).configure(s, ff, synth.rules_t2())
    with pytest.raises(pk.DynBondError):
        pk.Batch([g1, g2])
    b = pk.Batch([g1, g1])
    with pytest.raises(pk.DynBondError) as e:
        pk.db_set_state(b.ctx, s.x, s.v, s.type)
    assert e.value.code == pk.DB_ESTATE


def test_autotune_picks_a_grid_point():
    import paper_1108_4214_amd as pk
    s = perturbed(synth.duplex_box(40, 8, 0.3, 5, 15), 0.05, 5)
    g = pk.System(s.n, s.L, 3, 1).configure(s, synth.ff_t2(), synth.rules_t2())
    skin, perm = pk.db_autotune(g.ctx, 3)
    assert skin in (0.4, 0.5, 0.6, 0.8) and perm in (1, 2, 4, 8)
    shape = pk.db_get_shape(g.ctx)
    assert shape["tiles"] in (0, 1) and shape["brick_edge"] in (0, 3, 4, 5) and shape["graph"] in (0, 1)
    assert g.stats()["steps"] == (16 + 4 + 2) * 4


def test_ladder_replicas_batch_forces_and_sweep():
    """Replicas of the temperature-ladder recipe (uneven sizes, own T and seed)."""
    import paper_1108_4214_amd as pk
    ws = synth.c4(n_rep=4)
    reps = []
    for w in ws:
        g = pk.System(w.system.n, w.system.L, w.seed, 1).configure(w.system, w.ff, w.rules)
        pk.db_set_reactive(g.ctx, w.system.reactive)
        reps.append(g)
    b = pk.Batch(reps)
    fb = _split(b.forces(), b.sizes)
    for g, f in zip(reps, fb):
        assert np.array_equal(f, g.forces())
    b.step(25)
    for r, g in enumerate(reps):
        g.step(25)
        xb, _ = b.replica_state(r)
        xg, _ = g.state()
        assert np.max(np.abs(xb - xg)) < 1e-4   # mixed precision, 25 steps


def test_batch_every_step_sweeps_keep_the_list():
    """A sweep every step in a batch: the lists are kept across sweeps and the
    changed beads' lists redone (per replica box), the bonded halo rebuilt for the
    beads whose tables changed (new angles and dihedrals in any role), and every
    replica still follows its standalone run and the oracle."""
    import paper_1108_4214_amd as pk
    reps, edges, systems = [], [], []
    for r, (nd, nbp, rho, T) in enumerate(((12, 8, 0.3, 0.8), (8, 6, 0.2, 1.0), (20, 8, 0.3, 1.2))):
        s = perturbed(synth.duplex_box(nd, nbp, rho, 70 + r, 80 + r, T=T), 0.05, 70 + r)
        ff = synth.ff_t2(T0=T, T1=T)
        g = pk.System(s.n, s.L, 90 + r).configure(s, ff, synth.rules_t2(p=0.7, every=1, r_kill=1.35))
        pk.db_set_reactive(g.ctx, s.reactive)
        reps.append(g)
        edges.append(s.L)
        systems.append((s, ff))
    b = pk.Batch(reps)
    b.step(30)
    for r, g in enumerate(reps):
        g.step(30)
        xb, vb = b.replica_state(r)
        xg, vg = g.state()
        d = xb - xg
        d -= edges[r] * np.round(d / edges[r])   # a bead at the boundary may sit at either end
        assert np.max(np.abs(d)) < 1e-9
        assert np.max(np.abs(vb - vg)) < 1e-7
    assert b.stats()["list_patches"] > 0
    assert b.counts()[0] == sum(g.counts()[0] for g in reps)
    s, ff = systems[0]
    o = oracle.Oracle.from_system(s, ff, synth.rules_t2(p=0.7, every=1, r_kill=1.35), seed=90)
    o.step(30)
    d = b.replica_state(0)[0] - o.state()[0]
    d -= edges[0] * np.round(d / edges[0])
    assert np.max(np.abs(d)) < 1e-9


def _replica_rows(rows, off, n, cols):
    """rows of a batch topology list whose ids (columns cols) lie in replica
    [off, off + n), with the ids made local"""
    rows = np.asarray(rows)
    if rows.size == 0:
        return rows
    keep = np.all((rows[:, cols] >= off) & (rows[:, cols] < off + n), axis=1)
    out = rows[keep].copy()
    out[:, cols] -= off
    return out


def test_ladder_batch_every_replica_against_its_oracle():
    """Six replicas of the temperature-ladder recipe (uneven sizes, own edge, seed
    and temperature) stepped together in FP64 with a sweep every 2 steps that kills
    and re-creates hybridization bonds: after 20 steps every replica's bonds, angles
    and dihedrals equal its own oracle's bit for bit, and its positions agree to
    1e-9."""
    import paper_1108_4214_amd as pk
    ws = synth.c4(n_rep=6)
    rules = synth.rules_t2(p=0.7, every=2, r_kill=1.3)
    reps, oracles = [], []
    for w in ws:
        s = w.system
        g = pk.System(s.n, s.L, w.seed, 0).configure(s, w.ff, rules)
        pk.db_set_reactive(g.ctx, s.reactive)
        reps.append((s, g))
        oracles.append(oracle.Oracle.from_system(s, w.ff, rules, seed=w.seed))
    b = pk.Batch([g for _, g in reps])
    b.step(20)
    bb, ba, bd = b.bonds(), b.angles(), b.dihedrals()
    off = 0
    events = 0
    for r, ((s, g), o) in enumerate(zip(reps, oracles)):
        o.step(20)
        assert np.array_equal(_replica_rows(bb, off, s.n, [0, 1]), o.bonds()), r
        assert np.array_equal(_replica_rows(ba, off, s.n, [1, 2, 3]), o.angles()), r
        assert np.array_equal(_replica_rows(bd, off, s.n, [1, 2, 3, 4]), o.dihedrals()), r
        xb, _ = b.replica_state(r)
        d = xb - o.state()[0]
        d -= s.L * np.round(d / s.L)
        assert np.max(np.abs(d)) < 1e-9, r
        _, cum, _ = o.stats()
        events += cum["bonds_created"] + cum["bonds_killed"]
        off += s.n
    assert events > 20


def test_batch_dense_solvent_forces_equal_standalone_bitwise():
    """DPD solvent at density 3 (conservative DPD pairs only): batched replicas of
    different sizes and edges get the same forces bit for bit as each alone, and the
    standalone forces agree with the oracle."""
    import paper_1108_4214_amd as pk
    from gpu_common import forces_close
    reps, systems = [], []
    for r, m in enumerate((3000, 5000)):
        s = synth.dpd_solution(0, 0, m, 3.0, 40 + r, 50 + r)
        ff = synth.ff_dpd(gamma_dpd=0.0)
        g = pk.System(s.n, s.L, 60 + r, 1).configure(s, ff, synth.RuleSet(every=0))
        reps.append(g)
        systems.append((s, ff))
    b = pk.Batch(reps)
    fb = _split(b.forces(), b.sizes)
    for g, f in zip(reps, fb):
        assert np.array_equal(f, g.forces())
    s, ff = systems[1]
    o = oracle.Oracle.from_system(s, ff, synth.RuleSet(every=0), seed=61)
    ok, msg = forces_close(reps[1].forces(), o.forces(), 1e-5)
    assert ok, msg
