"""db_energy_noalloc (the energy entry point that allocates nothing, for callers
that cannot allocate: graph capture, serving loops) against db_energy through
the C ABI: the same kernels in the same order, so the six sums agree bit for
bit; two calls in a row on two handles, the second smaller, share the one
scratch array of the device."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _system(pk, synth, n_duplex, n_bp, precision, seed, rho=0.3):
    s = synth.small_duplexes(n_duplex=n_duplex, n_bp=n_bp, rho=rho, seed_w=seed, seed_d=seed + 10)
    g = pk.System(s.n, s.L, seed, precision).configure(s, synth.ff_t2(), synth.rules_t2())
    return g


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_energy_equals_energy(precision):
    import paper_1108_4214_amd as pk
    import synth

    big = _system(pk, synth, 40, 12, precision, 5)      # 1,920 beads: several workgroups and a ragged tail
    small = _system(pk, synth, 3, 7, precision, 6, rho=0.05)   # 84 beads: one workgroup
    try:
        for g in (big, small):
            g.step(3)
        for g in (big, small):                            # big, then the smaller one
            ref = pk.db_energy(g.ctx)
            got = pk.db_energy_noalloc(g.ctx)
            assert np.all(np.isfinite(ref))
            np.testing.assert_array_equal(got, ref)
        g = big
        g.step(2)
        np.testing.assert_array_equal(pk.db_energy_noalloc(g.ctx), pk.db_energy(g.ctx))
    finally:
        big.close()
        small.close()


def test_noalloc_energy_needs_current_device_state():
    import paper_1108_4214_amd as pk
    import synth
    s = synth.small_duplexes(n_duplex=3, n_bp=7, rho=0.05, seed_w=6, seed_d=16)
    c = pk.db_create(s.n, s.L, 1)
    try:
        pk.db_set_state(c, s.x, s.v, s.type)
        with pytest.raises(pk.DynBondError) as e:         # nothing is on the device yet
            pk.db_energy_noalloc(c)
        assert e.value.code == pk.DB_ESTATE
        ref = pk.db_energy(c)                             # sets the device up
        np.testing.assert_array_equal(pk.db_energy_noalloc(c), ref)
    finally:
        pk.db_destroy(c)


def test_noalloc_energy_rejects_sizes_beyond_its_scratch():
    import paper_1108_4214_amd as pk
    c = pk.db_create(16777217, 400.0, 1)
    try:
        with pytest.raises(pk.DynBondError) as e:
            pk.db_energy_noalloc(c)
        assert e.value.code == pk.DB_EINVAL
    finally:
        pk.db_destroy(c)
