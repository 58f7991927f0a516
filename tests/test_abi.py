"""The C-ABI library loads on the host and exports every entry point that
include/dynbond.h declares; host-side argument validation needs no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    with open(os.path.join(ROOT, "include", "dynbond.h")) as f:
        for line in f:
            m = re.match(r"^(?:int|const char\*)\s+(db_\w+)\(", line.strip())
            if m:
                names.add(m.group(1))
    return names


def test_header_declares_the_call_set():
    d = _declared()
    for required in ["db_create", "db_step", "db_sweep_now", "db_bond_create", "db_bond_break", "db_bond_convert",
                     "db_angle_pattern", "db_dihedral_pattern", "db_max_bonds", "db_generate_angles_dihedrals"]:
        assert required in d


def test_library_exports_every_declared_symbol():
    import paper_1108_4214_amd as pk
    lib = ctypes.CDLL(pk.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing
    assert set(pk.EXPORTS) == _declared()


def test_host_side_validation_without_gpu():
    import numpy as np
    import paper_1108_4214_amd as pk
    with pytest.raises(pk.DynBondError):
        pk.db_create(-1, 10.0, 1)
    with pytest.raises(pk.DynBondError):
        pk.db_create(4, 10.0, 1, precision=7)
    with pytest.raises(pk.DynBondError):
        pk.db_create(4, 65536.5, 1)          # beyond the largest box edge
    c = pk.db_create(4, 10.0, 1)
    try:
        assert pk.db_workspace_bytes(c) > 0
        with pytest.raises(pk.DynBondError) as e:
            pk.db_step(c, 1)
        assert e.value.code == pk.DB_ESTATE
        with pytest.raises(pk.DynBondError):
            pk.db_bond_create(c, 1, 1, 2, 1.5, 2.0)      # probability above one
        with pytest.raises(pk.DynBondError):
            pk.db_bond_create(c, 1, 1, 2, 6.0, 0.5)      # reaction distance beyond half the box
        with pytest.raises(pk.DynBondError):
            pk.db_set_state(c, np.full((4, 3), 10.0), None, np.ones(4, np.int32))   # outside [0, L)
        pk.db_set_state(c, np.full((4, 3), 1.0), None, np.ones(4, np.int32))
        with pytest.raises(pk.DynBondError) as e:
            pk.db_set_bonds(c, np.array([[0, 1, 1, 1], [0, 2, 1, 1], [0, 3, 1, 1], [1, 2, 1, 1], [0, 0, 1, 1]]))
        assert e.value.code == pk.DB_EINVAL
        b5 = np.array([[0, k, 1, 1] for k in (1, 2, 3)] + [[1, 2, 1, 1], [2, 3, 1, 1]])
        pk.db_set_bonds(c, b5)
        assert pk.db_topology_counts(c) == (5, 0, 0)
        assert pk.db_get_bonds(c).tolist() == [[0, 1, 1, 1], [0, 2, 1, 1], [0, 3, 1, 1], [1, 2, 1, 1], [2, 3, 1, 1]]
    finally:
        pk.db_destroy(c)


def test_bonds_over_capacity_rejected_on_host():
    import numpy as np
    import paper_1108_4214_amd as pk
    c = pk.db_create(6, 10.0, 1)
    try:
        pk.db_set_state(c, np.full((6, 3), 1.0), None, np.ones(6, np.int32))
        with pytest.raises(pk.DynBondError) as e:
            pk.db_set_bonds(c, np.array([[0, k, 1, 1] for k in range(1, 6)]))
        assert e.value.code == pk.DB_ECAPACITY
    finally:
        pk.db_destroy(c)
