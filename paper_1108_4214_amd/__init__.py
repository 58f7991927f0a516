"""Python binding of libdynbond (the C-ABI in include/dynbond.h).

Argument marshalling only: every computation runs in the HIP library.  The
module-level functions carry the C names (``db_create`` ... ``db_get_stats``)
and raise ``DynBondError`` on a non-zero status; ``System`` is a small object
wrapper over them.  Host arrays are numpy; device arrays are torch tensors on
the GPU (passed with ``on_device=1``).  Importing this module fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdynbond.so")

DB_OK, DB_EINVAL, DB_ECAPACITY, DB_ENONFINITE, DB_EDEVICE, DB_ESTATE = 0, -1, -2, -3, -4, -5
DB_FP64, DB_MIXED = 0, 1
DB_ACCEPT_PAIR, DB_ACCEPT_AVERAGE = 0, 1
DB_ANY = 0
DB_ALL_BONDTYPES = 0xFFFFFFFF
MAX_BONDS_PER_BEAD, MAX_ANGLES_PER_BEAD, MAX_DIHEDRALS_PER_BEAD = 4, 12, 16

EXPORTS = [
    "db_create", "db_workspace_bytes", "db_bind_workspace", "db_destroy", "db_last_error",
    "db_set_state", "db_set_reactive", "db_set_bonds", "db_set_angles", "db_set_dihedrals",
    "db_generate_angles_dihedrals", "db_pair_wca", "db_pair_dpd", "db_bond_harmonic", "db_bond_well",
    "db_angle_harmonic",
    "db_dihedral_cosine", "db_langevin", "db_temperature_ramp", "db_sweep_every", "db_bond_create",
    "db_bond_create_dir", "db_bond_break", "db_bond_kill", "db_bond_convert", "db_max_bonds",
    "db_angle_pattern", "db_dihedral_pattern", "db_step", "db_sweep_now", "db_forces", "db_energy",
    "db_get_state", "db_topology_counts", "db_get_bonds", "db_get_angles", "db_get_dihedrals",
    "db_get_stats", "db_set_step", "db_tune", "db_profile", "db_step_kernel_time", "db_autotune",
    "db_batch_create", "db_batch_get_state", "db_track_topology_energy", "db_external_force",
    "db_energy_noalloc", "db_acceptance", "db_tile_shape", "db_tile_stats", "db_graph", "db_get_shape",
    "db_checkpoint_bytes", "db_checkpoint_save", "db_checkpoint_load",
]

STAT_FIELDS = [
    "bonds_created", "bonds_broken", "bonds_killed", "bonds_converted",
    "angles_created", "angles_removed", "dihedrals_created", "dihedrals_removed",
    "cum_bonds_created", "cum_bonds_broken", "cum_bonds_killed", "cum_bonds_converted",
    "cum_angles_created", "cum_angles_removed", "cum_dihedrals_created", "cum_dihedrals_removed",
    "sweeps", "steps", "rebuilds", "rollbacks",
]


LEDGER_FIELDS = ["du_topo_last", "du_topo_cum"]
TAIL_FIELDS = ["list_patches"]


class db_stats(C.Structure):
    _fields_ = ([(f, C.c_int64) for f in STAT_FIELDS] + [(f, C.c_double) for f in LEDGER_FIELDS] +
                [(f, C.c_int64) for f in TAIL_FIELDS])


class DynBondError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdynbond error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1108_4214_amd/build.py "
                      "(or __graft_entry__.build()); there is no fallback path")

_lib = C.CDLL(LIB_PATH)

_P, _d, _i32, _i64, _u64, _int = C.c_void_p, C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_int
_SIG = {
    "db_create": [C.POINTER(C.c_void_p), _i32, _d, _u64, _int, _P],
    "db_workspace_bytes": [_P, C.POINTER(C.c_size_t)],
    "db_bind_workspace": [_P, _P, C.c_size_t],
    "db_destroy": [_P],
    "db_set_state": [_P, _P, _P, _P, _int],
    "db_set_reactive": [_P, _P],
    "db_set_bonds": [_P, _i64, _P, _P, _P],
    "db_set_angles": [_P, _i64, _P, _P],
    "db_set_dihedrals": [_P, _i64, _P, _P],
    "db_generate_angles_dihedrals": [_P],
    "db_pair_wca": [_P, _d, _d, _d, _int],
    "db_pair_dpd": [_P, _d, _d, _d, _int],
    "db_bond_harmonic": [_P, _i32, _d, _d],
    "db_bond_well": [_P, _i32, _d, _d, _d, _d],
    "db_external_force": [_P, _i64, _P, _P],
    "db_angle_harmonic": [_P, _i32, _d, _d],
    "db_dihedral_cosine": [_P, _i32, _d, _d],
    "db_langevin": [_P, _d, _d, _d],
    "db_temperature_ramp": [_P, _d, _d, _i64],
    "db_sweep_every": [_P, _i32, _int, _int],
    "db_bond_create": [_P, _i32, _i32, _i32, _d, _d],
    "db_bond_create_dir": [_P, _i32, _i32, _i32, _i32, _d, _d],
    "db_bond_break": [_P, _i32, _d, _d],
    "db_bond_kill": [_P, _i32, _d],
    "db_bond_convert": [_P, _i32, _i32, _d, _d],
    "db_max_bonds": [_P, _i32, _i32, _i32],
    "db_angle_pattern": [_P, _i32, _P, _P],
    "db_dihedral_pattern": [_P, _i32, _P, _P],
    "db_step": [_P, _i64],
    "db_sweep_now": [_P],
    "db_forces": [_P, _P, _int],
    "db_energy": [_P, _P],
    "db_energy_noalloc": [_P, _P],
    "db_acceptance": [_P, _int],
    "db_tile_shape": [_P, _int, _i32],
    "db_tile_stats": [_P, _P],
    "db_graph": [_P, _int],
    "db_get_shape": [_P, _P],
    "db_get_state": [_P, _P, _P, _int],
    "db_topology_counts": [_P, _P, _P, _P],
    "db_get_bonds": [_P, _P, _P, _P],
    "db_get_angles": [_P, _P, _P],
    "db_get_dihedrals": [_P, _P, _P],
    "db_get_stats": [_P, C.POINTER(db_stats)],
    "db_set_step": [_P, _i64],
    "db_tune": [_P, _d, _i32],
    "db_profile": [_P, _int],
    "db_step_kernel_time": [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "db_autotune": [_P, _i64, C.POINTER(C.c_double), C.POINTER(C.c_int32)],
    "db_batch_create": [C.POINTER(C.c_void_p), _P, _i32, _P],
    "db_batch_get_state": [_P, _i32, _P, _P, _int],
    "db_track_topology_energy": [_P, _int],
    "db_checkpoint_bytes": [_P, C.POINTER(C.c_size_t)],
    "db_checkpoint_save": [_P, _P, C.c_size_t],
    "db_checkpoint_load": [_P, _P, C.c_size_t],
}
for _name, _args in _SIG.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.db_last_error.argtypes = [_P]
_lib.db_last_error.restype = C.c_char_p


def lib():
    return _lib


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _on_device(a):
    return 1 if (hasattr(a, "is_cuda") and a.is_cuda) else 0


def _check(ctx, rc):
    if rc != DB_OK:
        msg = _lib.db_last_error(ctx).decode() if ctx else ""
        raise DynBondError(rc, msg)


# ---- C-named functions ----------------------------------------------------------------

def db_create(n_beads, box_L, seed, precision=DB_FP64, hip_stream=None):
    h = C.c_void_p()
    rc = _lib.db_create(C.byref(h), int(n_beads), float(box_L), int(seed) & (2 ** 64 - 1), int(precision),
                        C.c_void_p(hip_stream) if hip_stream else None)
    if rc != DB_OK:
        raise DynBondError(rc, "db_create rejected its arguments")
    return h


def db_destroy(ctx):
    _check(None, _lib.db_destroy(ctx))


def db_workspace_bytes(ctx):
    v = C.c_size_t()
    _check(ctx, _lib.db_workspace_bytes(ctx, C.byref(v)))
    return int(v.value)


def db_bind_workspace(ctx, tensor):
    _check(ctx, _lib.db_bind_workspace(ctx, C.c_void_p(tensor.data_ptr()), int(tensor.numel() * tensor.element_size())))


def db_set_state(ctx, x, v, type_):
    if _on_device(x):
        _check(ctx, _lib.db_set_state(ctx, _ptr(x), _ptr(v), _ptr(type_), 1))
        return
    x = _host(x, np.float64)
    v = None if v is None else _host(v, np.float64)
    t = _host(type_, np.int32)
    _check(ctx, _lib.db_set_state(ctx, _ptr(x), _ptr(v), _ptr(t), 0))


def db_set_reactive(ctx, flag):
    f = _host(flag, np.uint8)
    _check(ctx, _lib.db_set_reactive(ctx, _ptr(f)))


def db_set_bonds(ctx, bonds):
    """bonds: (nb, 4) rows i, j, type stored by i, type stored by j"""
    b = _host(bonds, np.int32).reshape(-1, 4)
    ij = np.ascontiguousarray(b[:, :2])
    a = np.ascontiguousarray(b[:, 2])
    c = np.ascontiguousarray(b[:, 3])
    _check(ctx, _lib.db_set_bonds(ctx, b.shape[0], _ptr(ij), _ptr(a), _ptr(c)))


def db_set_angles(ctx, angles):
    """angles: (na, 4) rows type, a, b, c"""
    a = _host(angles, np.int32).reshape(-1, 4)
    abc = np.ascontiguousarray(a[:, 1:])
    t = np.ascontiguousarray(a[:, 0])
    _check(ctx, _lib.db_set_angles(ctx, a.shape[0], _ptr(abc), _ptr(t)))


def db_set_dihedrals(ctx, dihedrals):
    """dihedrals: (nd, 5) rows type, a, b, c, d"""
    d = _host(dihedrals, np.int32).reshape(-1, 5)
    abcd = np.ascontiguousarray(d[:, 1:])
    t = np.ascontiguousarray(d[:, 0])
    _check(ctx, _lib.db_set_dihedrals(ctx, d.shape[0], _ptr(abcd), _ptr(t)))


def db_generate_angles_dihedrals(ctx):
    _check(ctx, _lib.db_generate_angles_dihedrals(ctx))


def db_pair_wca(ctx, eps, sigma, rc, exclude_depth):
    _check(ctx, _lib.db_pair_wca(ctx, eps, sigma, rc, int(exclude_depth)))


def db_pair_dpd(ctx, a, gamma, rc, exclude_depth):
    _check(ctx, _lib.db_pair_dpd(ctx, a, gamma, rc, int(exclude_depth)))


def db_bond_harmonic(ctx, t, K, r0):
    _check(ctx, _lib.db_bond_harmonic(ctx, int(t), K, r0))


def db_external_force(ctx, ids, f):
    i = np.ascontiguousarray(np.asarray(ids, dtype=np.int32).reshape(-1))
    fv = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, 3))
    if fv.shape[0] != i.shape[0]:
        raise ValueError("one force per id")
    _check(ctx, _lib.db_external_force(ctx, i.shape[0], i.ctypes.data, fv.ctypes.data))


def db_bond_well(ctx, t, umin, r_well, r_zero, r_cut):
    _check(ctx, _lib.db_bond_well(ctx, int(t), umin, r_well, r_zero, r_cut))


def db_angle_harmonic(ctx, t, K, theta0):
    _check(ctx, _lib.db_angle_harmonic(ctx, int(t), K, theta0))


def db_dihedral_cosine(ctx, t, K, phi0):
    _check(ctx, _lib.db_dihedral_cosine(ctx, int(t), K, phi0))


def db_langevin(ctx, T, gamma, dt):
    _check(ctx, _lib.db_langevin(ctx, T, gamma, dt))


def db_temperature_ramp(ctx, T0, T1, n_steps):
    _check(ctx, _lib.db_temperature_ramp(ctx, T0, T1, int(n_steps)))


def db_sweep_every(ctx, every, paircheck13=0, paircheck14=0):
    _check(ctx, _lib.db_sweep_every(ctx, int(every), int(paircheck13), int(paircheck14)))


def db_tile_shape(ctx, enable, brick_edge=0):
    _check(ctx, _lib.db_tile_shape(ctx, int(enable), int(brick_edge)))


def db_get_shape(ctx):
    out = np.zeros(3, dtype=np.int32)
    _check(ctx, _lib.db_get_shape(ctx, _ptr(out)))
    return {"tiles": int(out[0]), "brick_edge": int(out[1]), "graph": int(out[2])}


def db_graph(ctx, enable):
    _check(ctx, _lib.db_graph(ctx, int(enable)))


def db_tile_stats(ctx):
    out = np.zeros(4, dtype=np.int64)
    _check(ctx, _lib.db_tile_stats(ctx, _ptr(out)))
    return {"tiles": int(out[0]), "staged": int(out[1]),
            "mean_region": float(out[2]) / max(1, int(out[1])), "max_region": int(out[3])}


def db_acceptance(ctx, mode):
    _check(ctx, _lib.db_acceptance(ctx, int(mode)))


def db_bond_create(ctx, bt, bead1, bead2, r_max, p):
    _check(ctx, _lib.db_bond_create(ctx, int(bt), int(bead1), int(bead2), r_max, p))


def db_bond_create_dir(ctx, bt1, bt2, bead1, bead2, r_max, p):
    _check(ctx, _lib.db_bond_create_dir(ctx, int(bt1), int(bt2), int(bead1), int(bead2), r_max, p))


def db_bond_break(ctx, bt, r_min, p):
    _check(ctx, _lib.db_bond_break(ctx, int(bt), r_min, p))


def db_bond_kill(ctx, bt, r_min):
    _check(ctx, _lib.db_bond_kill(ctx, int(bt), r_min))


def db_bond_convert(ctx, bt_from, bt_to, r_min, p):
    _check(ctx, _lib.db_bond_convert(ctx, int(bt_from), int(bt_to), r_min, p))


def db_max_bonds(ctx, bt, bead_type, max_):
    _check(ctx, _lib.db_max_bonds(ctx, int(bt), int(bead_type), int(max_)))


def db_angle_pattern(ctx, atype, beads, masks):
    b = _host(beads, np.int32)
    m = _host([int(v) & 0xFFFFFFFF for v in masks], np.uint32)
    _check(ctx, _lib.db_angle_pattern(ctx, int(atype), _ptr(b), _ptr(m)))


def db_dihedral_pattern(ctx, dtype, beads, masks):
    b = _host(beads, np.int32)
    m = _host([int(v) & 0xFFFFFFFF for v in masks], np.uint32)
    _check(ctx, _lib.db_dihedral_pattern(ctx, int(dtype), _ptr(b), _ptr(m)))


def db_step(ctx, n):
    _check(ctx, _lib.db_step(ctx, int(n)))


def db_sweep_now(ctx):
    _check(ctx, _lib.db_sweep_now(ctx))


def db_forces(ctx, out):
    """out: (N,3) float64 numpy array or CUDA tensor"""
    _check(ctx, _lib.db_forces(ctx, _ptr(out), _on_device(out)))
    return out


def db_energy(ctx):
    e = np.zeros(6)
    _check(ctx, _lib.db_energy(ctx, _ptr(e)))
    return e


def db_energy_noalloc(ctx):
    e = np.zeros(6)
    _check(ctx, _lib.db_energy_noalloc(ctx, _ptr(e)))
    return e


def db_checkpoint_bytes(ctx):
    v = C.c_size_t()
    _check(ctx, _lib.db_checkpoint_bytes(ctx, C.byref(v)))
    return int(v.value)


def db_checkpoint_save(ctx):
    """the handle's checkpoint as a uint8 array"""
    buf = np.zeros(db_checkpoint_bytes(ctx), dtype=np.uint8)
    _check(ctx, _lib.db_checkpoint_save(ctx, _ptr(buf), buf.size))
    return buf


def db_checkpoint_load(ctx, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(ctx, _lib.db_checkpoint_load(ctx, _ptr(buf), buf.size))


def db_get_state(ctx, x, v):
    dev = _on_device(x) if x is not None else _on_device(v)
    _check(ctx, _lib.db_get_state(ctx, _ptr(x), _ptr(v), dev))
    return x, v


def db_topology_counts(ctx):
    a = np.zeros(3, dtype=np.int64)
    _check(ctx, _lib.db_topology_counts(ctx, _ptr(a[0:1]), _ptr(a[1:2]), _ptr(a[2:3])))
    return tuple(int(t) for t in a)


def db_get_bonds(ctx):
    nb, _, _ = db_topology_counts(ctx)
    ij = np.zeros((max(nb, 1), 2), np.int32)
    a = np.zeros(max(nb, 1), np.int32)
    b = np.zeros(max(nb, 1), np.int32)
    _check(ctx, _lib.db_get_bonds(ctx, _ptr(ij), _ptr(a), _ptr(b)))
    return np.column_stack([ij, a, b])[:nb]


def db_get_angles(ctx):
    _, na, _ = db_topology_counts(ctx)
    abc = np.zeros((max(na, 1), 3), np.int32)
    t = np.zeros(max(na, 1), np.int32)
    _check(ctx, _lib.db_get_angles(ctx, _ptr(abc), _ptr(t)))
    return np.column_stack([t, abc])[:na]


def db_get_dihedrals(ctx):
    _, _, nd = db_topology_counts(ctx)
    abcd = np.zeros((max(nd, 1), 4), np.int32)
    t = np.zeros(max(nd, 1), np.int32)
    _check(ctx, _lib.db_get_dihedrals(ctx, _ptr(abcd), _ptr(t)))
    return np.column_stack([t, abcd])[:nd]


def db_get_stats(ctx):
    s = db_stats()
    _check(ctx, _lib.db_get_stats(ctx, C.byref(s)))
    out = {f: int(getattr(s, f)) for f in STAT_FIELDS}
    out.update({f: float(getattr(s, f)) for f in LEDGER_FIELDS})
    out.update({f: int(getattr(s, f)) for f in TAIL_FIELDS})
    return out


def db_set_step(ctx, step):
    _check(ctx, _lib.db_set_step(ctx, int(step)))


def db_tune(ctx, skin, permute_every):
    _check(ctx, _lib.db_tune(ctx, float(skin), int(permute_every)))


def db_profile(ctx, every):
    _check(ctx, _lib.db_profile(ctx, int(every)))


def db_step_kernel_time(ctx):
    us = C.c_double()
    n = C.c_int64()
    _check(ctx, _lib.db_step_kernel_time(ctx, C.byref(us), C.byref(n)))
    return float(us.value), int(n.value)


def db_autotune(ctx, steps_per_trial):
    sk = C.c_double()
    pe = C.c_int32()
    _check(ctx, _lib.db_autotune(ctx, int(steps_per_trial), C.byref(sk), C.byref(pe)))
    return float(sk.value), int(pe.value)


def db_track_topology_energy(ctx, enable):
    _check(ctx, _lib.db_track_topology_energy(ctx, int(enable)))


def db_batch_create(replica_ctxs, hip_stream=None):
    arr = (C.c_void_p * len(replica_ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in replica_ctxs])
    h = C.c_void_p()
    rc = _lib.db_batch_create(C.byref(h), C.cast(arr, C.c_void_p), len(replica_ctxs),
                              C.c_void_p(hip_stream) if hip_stream else None)
    if rc != DB_OK:
        raise DynBondError(rc, "db_batch_create rejected its replicas")
    return h


def db_batch_get_state(ctx, replica, x, v):
    dev = _on_device(x) if x is not None else _on_device(v)
    _check(ctx, _lib.db_batch_get_state(ctx, int(replica), _ptr(x), _ptr(v), dev))
    return x, v


# ---- object wrapper ---------------------------------------------------------------------

class System:
    """One simulation box on the GPU (wraps a db_ctx handle)."""

    def __init__(self, n_beads, box_L, seed, precision=DB_FP64, hip_stream=None):
        self.n = int(n_beads)
        self.ctx = db_create(n_beads, box_L, seed, precision, hip_stream)

    def close(self):
        if getattr(self, "ctx", None):
            db_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def configure(self, system, ff=None, rules=None, generate=True):
        """Marshal a description (positions, velocities, types, reactive flags,
        bonds, optional angle/dihedral lists; force field; ordered rules) into calls."""
        c = self.ctx
        db_set_state(c, system.x, system.v, system.type)
        db_set_reactive(c, system.reactive)
        db_set_bonds(c, system.bonds)
        if ff is not None:
            if getattr(ff, "pair", "wca") == "dpd":
                db_pair_dpd(c, ff.dpd_a, ff.dpd_gamma, ff.rc, ff.exclude_depth)
            else:
                db_pair_wca(c, ff.eps, ff.sigma, ff.rc, ff.exclude_depth)
            for t, (K, r0) in ff.bonds.items():
                db_bond_harmonic(c, t, K, r0)
            for t, (umin, rw, rz, rcut) in getattr(ff, "wells", {}).items():
                db_bond_well(c, t, umin, rw, rz, rcut)
            for t, (K, th0) in ff.angles.items():
                db_angle_harmonic(c, t, K, th0)
            for t, (K, p0) in ff.dihedrals.items():
                db_dihedral_cosine(c, t, K, p0)
            db_langevin(c, ff.T0, ff.gamma, ff.dt)
            if ff.ramp_steps > 0:
                db_temperature_ramp(c, ff.T0, ff.T1, ff.ramp_steps)
        if rules is not None:
            db_sweep_every(c, rules.every, rules.paircheck13, rules.paircheck14)
            db_acceptance(c, DB_ACCEPT_AVERAGE if rules.accept == "average" else DB_ACCEPT_PAIR)
            for r in rules.rules:
                k = r[0]
                if k == "create":
                    db_bond_create(c, *r[1:])
                elif k == "createdir":
                    db_bond_create_dir(c, *r[1:])
                elif k == "break":
                    db_bond_break(c, *r[1:])
                elif k == "kill":
                    db_bond_kill(c, *r[1:])
                elif k == "convert":
                    db_bond_convert(c, *r[1:])
                elif k == "maxbond":
                    db_max_bonds(c, *r[1:])
                elif k == "angle":
                    db_angle_pattern(c, r[1], r[2], r[3])
                elif k == "dihedral":
                    db_dihedral_pattern(c, r[1], r[2], r[3])
                else:
                    raise ValueError(f"unknown rule {k}")
        if getattr(system, "angles", None) is not None:
            db_set_angles(c, system.angles)
        if getattr(system, "dihedrals", None) is not None:
            db_set_dihedrals(c, system.dihedrals)
        if generate and getattr(system, "angles", None) is None and getattr(system, "dihedrals", None) is None \
                and rules is not None:
            db_generate_angles_dihedrals(c)
        return self

    def step(self, n):
        db_step(self.ctx, n)

    def sweep_now(self):
        db_sweep_now(self.ctx)

    def forces(self):
        f = np.zeros((self.n, 3))
        return db_forces(self.ctx, f)

    def energy(self):
        return db_energy(self.ctx)

    def state(self):
        x = np.zeros((self.n, 3))
        v = np.zeros((self.n, 3))
        db_get_state(self.ctx, x, v)
        return x, v

    def counts(self):
        return db_topology_counts(self.ctx)

    def bonds(self):
        return db_get_bonds(self.ctx)

    def angles(self):
        return db_get_angles(self.ctx)

    def dihedrals(self):
        return db_get_dihedrals(self.ctx)

    def stats(self):
        return db_get_stats(self.ctx)

    def set_step(self, st):
        db_set_step(self.ctx, st)


class Batch(System):
    """Independent replicas (configured ``System`` objects) advanced by shared
    kernel launches; the replicas are copied, not referenced."""

    def __init__(self, replicas, hip_stream=None):
        self.sizes = [r.n for r in replicas]
        self.n = int(sum(self.sizes))
        self.ctx = db_batch_create([r.ctx for r in replicas], hip_stream)

    def replica_state(self, r):
        x = np.zeros((self.sizes[r], 3))
        v = np.zeros((self.sizes[r], 3))
        db_batch_get_state(self.ctx, r, x, v)
        return x, v
