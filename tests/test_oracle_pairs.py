"""Pin of the oracle's neighbour search: the cell-list pair set equals an
independent numpy brute force over all pairs with the minimum-image convention."""
import numpy as np
import pytest

import oracle
import synth


def _numpy_pairs(x, L, rcut):
    d = x[None, :, :] - x[:, None, :]
    d = np.where(d > 0.5 * L, d - L, d)
    d = np.where(d < -0.5 * L, d + L, d)
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    i, j = np.nonzero(np.triu(r2 < rcut * rcut, k=1))
    return set(zip(i.tolist(), j.tolist()))


@pytest.mark.parametrize("n,L,rcut", [(1500, 14.0, 1.1225), (1200, 12.0, 1.5), (300, 5.0, 1.2), (64, 3.2, 1.5)])
def test_cell_list_equals_brute_force(n, L, rcut):
    s = synth.random_gas(n, L, seed=n)
    o = oracle.Oracle(s.n, s.L, 1)
    o.set_state(s.x, s.v, s.type)
    ref = _numpy_pairs(s.x, s.L, rcut)
    cell = set(map(tuple, o.pairs_within(rcut, brute=0).tolist()))
    brute = set(map(tuple, o.pairs_within(rcut, brute=1).tolist()))
    assert cell == ref
    assert brute == ref


def test_pairs_on_the_box_boundary():
    L = 10.0
    x = np.array([[0.0, 0.0, 0.0], [9.5, 0.0, 0.0], [0.0, 9.3, 9.3], [5.0, 5.0, 5.0]])
    o = oracle.Oracle(4, L, 1)
    o.set_state(x, np.zeros_like(x), np.ones(4, dtype=np.int32))
    got = set(map(tuple, o.pairs_within(1.0, brute=0).tolist()))
    assert got == {(0, 1), (0, 2)} == _numpy_pairs(x, L, 1.0)
