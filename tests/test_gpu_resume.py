"""Failure handling and resume on the GPU: a non-finite state forced from the host
reaches DB_ENONFINITE through the device's error word and stays latched until a
new state is given; a checkpoint saved mid-run and loaded into a fresh handle
continues bit for bit as the uninterrupted run."""
import numpy as np
import pytest

import synth
from gpu_common import perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_4214_amd  # noqa: F401


def _coincident(s, i, j):
    """a copy of the system with bead j moved onto bead i (a zero separation)"""
    import dataclasses
    x = s.x.copy()
    x[j] = x[i]
    return dataclasses.replace(s, x=x)


@pytest.mark.parametrize("precision", [0, 1])
def test_nonfinite_state_is_reported_and_latched(precision):
    import paper_1108_4214_amd as pk
    s = perturbed(synth.duplex_box(8, 6, 0.2, 3, 13), 0.05, 3)
    # two unbonded beads of different strands on one point: the pair force is
    # not finite, so is the next position, and the step kernel flags it
    nb = 2 * 6 * 2   # beads of the first duplex (two strands of 6 nucleotides, 2 beads each)
    bad = _coincident(s, 0, nb + 5)
    g = pk.System(s.n, s.L, 5, precision).configure(bad, synth.ff_t2(), synth.rules_t2())
    with pytest.raises(pk.DynBondError) as e:
        g.step(4)
    assert e.value.code == pk.DB_ENONFINITE
    # latched: nothing runs on the undefined state
    with pytest.raises(pk.DynBondError) as e2:
        g.step(1)
    assert e2.value.code == pk.DB_ENONFINITE
    # a new state clears it and the run goes on
    pk.db_set_state(g.ctx, s.x, s.v, s.type)
    g.step(5)
    x, v = g.state()
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(v))
    assert np.all((x >= 0) & (x < s.L))


def _run_pair(precision, tiles):
    import paper_1108_4214_amd as pk
    s = perturbed(synth.duplex_box(30, 8, 0.3, 17, 27), 0.05, 17)
    ff = synth.ff_t2(T0=0.9, T1=0.9)
    rules = synth.rules_t2(p=0.6, every=5, r_kill=1.35)

    def make():
        g = pk.System(s.n, s.L, 77, precision)
        pk.db_tile_shape(g.ctx, tiles, 0)
        return g.configure(s, ff, rules)

    return s, make


@pytest.mark.parametrize("precision,tiles", [(0, 0), (1, 0), (1, 1)])
def test_checkpoint_resume_is_bitwise(precision, tiles):
    import paper_1108_4214_amd as pk
    s, make = _run_pair(precision, tiles)
    a = make()
    a.step(37)                       # mid-way between sweeps and list rebuilds
    buf = pk.db_checkpoint_save(a.ctx)
    assert buf.size == pk.db_checkpoint_bytes(a.ctx)
    a.step(58)
    b = make()
    pk.db_checkpoint_load(b.ctx, buf)
    b.step(58)
    xa, va = a.state()
    xb, vb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert np.array_equal(a.bonds(), b.bonds())
    assert np.array_equal(a.angles(), b.angles())
    assert np.array_equal(a.dihedrals(), b.dihedrals())
    sa, sb = a.stats(), b.stats()
    for k in ("steps", "sweeps", "rebuilds", "cum_bonds_created", "cum_bonds_killed", "list_patches"):
        assert sa[k] == sb[k], k
    assert sa["cum_bonds_created"] + sa["cum_bonds_killed"] > 0
    # the energies agree too (the same state in the same slots)
    assert np.array_equal(a.energy(), b.energy())


@pytest.mark.parametrize("precision", [0, 1])
def test_checkpoint_resume_dpd_is_bitwise(precision):
    """With the DPD pair thermostat the step kernels read the neighbours' input
    velocities and write a second velocity buffer, the two exchanged after each
    step: a checkpoint after an odd number of steps restores which buffer holds the
    current velocities.  Sweeps every step keep and patch the lists."""
    import paper_1108_4214_amd as pk
    s = perturbed(synth.dpd_solution(16, 6, 4000, 3.0, 7, 17), 0.05, 7)
    ff, rules = synth.ff_dpd(gamma_dpd=4.5), synth.rules_t2(p=0.7, every=1, r_kill=1.3)

    def make():
        return pk.System(s.n, s.L, 31, precision).configure(s, ff, rules)

    a = make()
    a.step(23)
    buf = pk.db_checkpoint_save(a.ctx)
    a.step(30)
    b = make()
    pk.db_checkpoint_load(b.ctx, buf)
    b.step(30)
    xa, va = a.state()
    xb, vb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert np.array_equal(a.bonds(), b.bonds())
    assert np.array_equal(a.angles(), b.angles()) and np.array_equal(a.dihedrals(), b.dihedrals())
    assert a.stats()["steps"] == b.stats()["steps"] == 53


def test_checkpoint_of_a_batch_is_refused():
    import paper_1108_4214_amd as pk
    s, make = _run_pair(0, 0)
    g1, g2 = make(), make()
    bt = pk.Batch([g1, g2])
    with pytest.raises(pk.DynBondError) as e:
        pk.db_checkpoint_bytes(bt.ctx)
    assert e.value.code == pk.DB_EINVAL


def test_checkpoint_rejects_another_system():
    import paper_1108_4214_amd as pk
    s, make = _run_pair(0, 0)
    a = make()
    a.step(3)
    buf = pk.db_checkpoint_save(a.ctx)
    other = pk.System(s.n, s.L, 78, 0).configure(s, synth.ff_t2(T0=0.9, T1=0.9),
                                                 synth.rules_t2(p=0.6, every=5, r_kill=1.35))
    x0, v0 = other.state()
    with pytest.raises(pk.DynBondError) as e:
        pk.db_checkpoint_load(other.ctx, buf)      # another seed
    assert e.value.code == pk.DB_EINVAL
    with pytest.raises(pk.DynBondError):
        pk.db_checkpoint_load(a.ctx, buf[:100])    # truncated
    x1, v1 = other.state()
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    other.step(2)
