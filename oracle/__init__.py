"""ctypes binding of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never loads it.

``build()`` compiles ``oracle.c`` with gcc (``-ffp-contract=off`` so cutoff
decisions use plain IEEE double arithmetic in source order).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-Wall", "-shared",
           "-o", LIB, os.path.join(HERE, "oracle.c"), "-lm"]
    subprocess.check_call(cmd)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        d, i32, i64, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "or_create": (P, [i32, d, u64]),
            "or_destroy": (None, [P]),
            "or_set_state": (C.c_int, [P, P, P, P]),
            "or_set_reactive": (C.c_int, [P, P]),
            "or_set_bonds": (C.c_int, [P, i64, P, P, P]),
            "or_set_angles": (C.c_int, [P, i64, P, P]),
            "or_set_dihedrals": (C.c_int, [P, i64, P, P]),
            "or_generate_angles_dihedrals": (C.c_int, [P]),
            "or_pair_wca": (C.c_int, [P, d, d, d, C.c_int]),
            "or_pair_dpd": (C.c_int, [P, d, d, d, C.c_int]),
            "or_bond_harmonic": (C.c_int, [P, i32, d, d]),
            "or_bond_well": (C.c_int, [P, i32, d, d, d, d]),
            "or_external_force": (C.c_int, [P, i64, P, P]),
            "or_angle_harmonic": (C.c_int, [P, i32, d, d]),
            "or_dihedral_cosine": (C.c_int, [P, i32, d, d]),
            "or_langevin": (C.c_int, [P, d, d, d]),
            "or_temperature_ramp": (C.c_int, [P, d, d, i64]),
            "or_sweep_every": (C.c_int, [P, i32, C.c_int, C.c_int]),
            "or_acceptance": (C.c_int, [P, C.c_int]),
            "or_bond_create": (C.c_int, [P, i32, i32, i32, d, d]),
            "or_bond_create_dir": (C.c_int, [P, i32, i32, i32, i32, d, d]),
            "or_bond_break": (C.c_int, [P, i32, d, d]),
            "or_bond_kill": (C.c_int, [P, i32, d]),
            "or_bond_convert": (C.c_int, [P, i32, i32, d, d]),
            "or_max_bonds": (C.c_int, [P, i32, i32, i32]),
            "or_angle_pattern": (C.c_int, [P, i32, P, P]),
            "or_dihedral_pattern": (C.c_int, [P, i32, P, P]),
            "or_set_step": (C.c_int, [P, i64]),
            "or_step": (C.c_int, [P, i64]),
            "or_sweep_now": (C.c_int, [P]),
            "or_forces": (C.c_int, [P, P]),
            "or_energy": (C.c_int, [P, P]),
            "or_get_state": (C.c_int, [P, P, P]),
            "or_topology_counts": (C.c_int, [P, P, P, P]),
            "or_get_bonds": (C.c_int, [P, P, P, P]),
            "or_get_angles": (C.c_int, [P, P, P]),
            "or_get_dihedrals": (C.c_int, [P, P, P]),
            "or_get_stats": (C.c_int, [P, P]),
            "or_last_nominations": (C.c_int, [P, P, P]),
            "or_philox4x32_10": (None, [P, P, P]),
            "or_pairs_within": (i64, [P, d, C.c_int, P, i64]),
            "or_graph_distance": (C.c_int, [P, i32, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    pass


def _chk(rc, what):
    if rc != 0:
        raise OracleError(f"{what} returned {rc}")


def philox4x32_10(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(o))
    return o


STAT_NAMES = ["bonds_created", "bonds_broken", "bonds_killed", "bonds_converted",
              "angles_created", "angles_removed", "dihedrals_created", "dihedrals_removed"]


class Oracle:
    """One oracle system.  Mirrors the library's call set with the ``or_`` prefix."""

    def __init__(self, n, L, seed):
        self.n = int(n)
        self._h = lib().or_create(int(n), float(L), int(seed) & (2 ** 64 - 1))
        if not self._h:
            raise OracleError("or_create failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    # -- configuration -----------------------------------------------------
    def set_state(self, x, v, type_):
        self._x = _c(x, np.float64); self._v = _c(v, np.float64); self._t = _c(type_, np.int32)
        _chk(lib().or_set_state(self._h, _p(self._x), _p(self._v), _p(self._t)), "or_set_state")

    def set_reactive(self, flag):
        f = _c(flag, np.uint8)
        _chk(lib().or_set_reactive(self._h, _p(f)), "or_set_reactive")

    def set_bonds(self, bonds):
        b = _c(bonds, np.int32).reshape(-1, 4)
        ij = np.ascontiguousarray(b[:, :2]); tij = np.ascontiguousarray(b[:, 2]); tji = np.ascontiguousarray(b[:, 3])
        _chk(lib().or_set_bonds(self._h, b.shape[0], _p(ij), _p(tij), _p(tji)), "or_set_bonds")

    def set_angles(self, ang):
        a = _c(ang, np.int32).reshape(-1, 4)
        abc = np.ascontiguousarray(a[:, 1:4]); t = np.ascontiguousarray(a[:, 0])
        _chk(lib().or_set_angles(self._h, a.shape[0], _p(abc), _p(t)), "or_set_angles")

    def set_dihedrals(self, dih):
        a = _c(dih, np.int32).reshape(-1, 5)
        abcd = np.ascontiguousarray(a[:, 1:5]); t = np.ascontiguousarray(a[:, 0])
        _chk(lib().or_set_dihedrals(self._h, a.shape[0], _p(abcd), _p(t)), "or_set_dihedrals")

    def set_external_force(self, ids, f):
        """constant external force f[k] (3 components) on bead ids[k]; empty ids clears"""
        i = _c(ids, np.int32).reshape(-1)
        fv = _c(f, np.float64).reshape(-1, 3)
        _chk(lib().or_external_force(self._h, i.shape[0], _p(i), _p(fv)), "or_external_force")

    def generate_angles_dihedrals(self):
        _chk(lib().or_generate_angles_dihedrals(self._h), "or_generate_angles_dihedrals")

    def set_forcefield(self, ff):
        L = lib()
        if getattr(ff, "pair", "wca") == "dpd":
            _chk(L.or_pair_dpd(self._h, ff.dpd_a, ff.dpd_gamma, ff.rc, ff.exclude_depth), "or_pair_dpd")
        else:
            _chk(L.or_pair_wca(self._h, ff.eps, ff.sigma, ff.rc, ff.exclude_depth), "or_pair_wca")
        for t, (K, r0) in ff.bonds.items():
            _chk(L.or_bond_harmonic(self._h, t, K, r0), "or_bond_harmonic")
        for t, (umin, rw, rz, rcut) in getattr(ff, "wells", {}).items():
            _chk(L.or_bond_well(self._h, t, umin, rw, rz, rcut), "or_bond_well")
        for t, (K, th0) in ff.angles.items():
            _chk(L.or_angle_harmonic(self._h, t, K, th0), "or_angle_harmonic")
        for t, (K, p0) in ff.dihedrals.items():
            _chk(L.or_dihedral_cosine(self._h, t, K, p0), "or_dihedral_cosine")
        _chk(L.or_langevin(self._h, ff.T0, ff.gamma, ff.dt), "or_langevin")
        if ff.ramp_steps > 0:
            _chk(L.or_temperature_ramp(self._h, ff.T0, ff.T1, ff.ramp_steps), "or_temperature_ramp")

    def set_rules(self, rs):
        L = lib()
        _chk(L.or_sweep_every(self._h, rs.every, rs.paircheck13, rs.paircheck14), "or_sweep_every")
        _chk(L.or_acceptance(self._h, 1 if rs.accept == "average" else 0), "or_acceptance")
        for r in rs.rules:
            k = r[0]
            if k == "create":
                rc = L.or_bond_create(self._h, r[1], r[2], r[3], r[4], r[5])
            elif k == "createdir":
                rc = L.or_bond_create_dir(self._h, r[1], r[2], r[3], r[4], r[5], r[6])
            elif k == "break":
                rc = L.or_bond_break(self._h, r[1], r[2], r[3])
            elif k == "kill":
                rc = L.or_bond_kill(self._h, r[1], r[2])
            elif k == "convert":
                rc = L.or_bond_convert(self._h, r[1], r[2], r[3], r[4])
            elif k == "maxbond":
                rc = L.or_max_bonds(self._h, r[1], r[2], r[3])
            elif k == "angle":
                b = _c(r[2], np.int32); m = _c(r[3], np.uint32)
                rc = L.or_angle_pattern(self._h, r[1], _p(b), _p(m))
            elif k == "dihedral":
                b = _c(r[2], np.int32); m = _c(r[3], np.uint32)
                rc = L.or_dihedral_pattern(self._h, r[1], _p(b), _p(m))
            else:
                raise ValueError(k)
            _chk(rc, f"rule {r}")

    @classmethod
    def from_system(cls, system, ff=None, rules=None, seed=0, generate=True):
        o = cls(system.n, system.L, seed)
        o.set_state(system.x, system.v, system.type)
        o.set_reactive(system.reactive)
        o.set_bonds(system.bonds)
        if ff is not None:
            o.set_forcefield(ff)
        if rules is not None:
            o.set_rules(rules)
        if system.angles is not None:
            o.set_angles(system.angles)
        if system.dihedrals is not None:
            o.set_dihedrals(system.dihedrals)
        if generate and system.angles is None and system.dihedrals is None and rules is not None:
            o.generate_angles_dihedrals()
        return o

    # -- running -----------------------------------------------------------
    def set_step(self, st):
        _chk(lib().or_set_step(self._h, int(st)), "or_set_step")

    def step(self, n):
        _chk(lib().or_step(self._h, int(n)), "or_step")

    def sweep_now(self):
        _chk(lib().or_sweep_now(self._h), "or_sweep_now")

    def forces(self):
        f = np.zeros((self.n, 3))
        _chk(lib().or_forces(self._h, _p(f)), "or_forces")
        return f

    def energy(self):
        e = np.zeros(6)
        _chk(lib().or_energy(self._h, _p(e)), "or_energy")
        return e

    def state(self):
        x = np.zeros((self.n, 3)); v = np.zeros((self.n, 3))
        _chk(lib().or_get_state(self._h, _p(x), _p(v)), "or_get_state")
        return x, v

    def counts(self):
        a = np.zeros(3, dtype=np.int64)
        _chk(lib().or_topology_counts(self._h, _p(a[0:1]), _p(a[1:2]), _p(a[2:3])), "or_topology_counts")
        return tuple(int(t) for t in a)

    def bonds(self):
        nb, _, _ = self.counts()
        ij = np.zeros((nb, 2), dtype=np.int32); a = np.zeros(nb, dtype=np.int32); b = np.zeros(nb, dtype=np.int32)
        _chk(lib().or_get_bonds(self._h, _p(ij), _p(a), _p(b)), "or_get_bonds")
        return np.column_stack([ij, a, b]) if nb else np.zeros((0, 4), dtype=np.int32)

    def angles(self):
        _, na, _ = self.counts()
        abc = np.zeros((na, 3), dtype=np.int32); t = np.zeros(na, dtype=np.int32)
        _chk(lib().or_get_angles(self._h, _p(abc), _p(t)), "or_get_angles")
        return np.column_stack([t, abc]) if na else np.zeros((0, 4), dtype=np.int32)

    def dihedrals(self):
        _, _, nd = self.counts()
        abcd = np.zeros((nd, 4), dtype=np.int32); t = np.zeros(nd, dtype=np.int32)
        _chk(lib().or_get_dihedrals(self._h, _p(abcd), _p(t)), "or_get_dihedrals")
        return np.column_stack([t, abcd]) if nd else np.zeros((0, 5), dtype=np.int32)

    def stats(self):
        a = np.zeros(17, dtype=np.int64)
        _chk(lib().or_get_stats(self._h, _p(a)), "or_get_stats")
        last = dict(zip(STAT_NAMES, (int(t) for t in a[:8])))
        cum = dict(zip(STAT_NAMES, (int(t) for t in a[8:16])))
        return last, cum, int(a[16])

    def nominations(self):
        c = np.zeros(self.n, dtype=np.int32); k = np.zeros(self.n, dtype=np.int32)
        _chk(lib().or_last_nominations(self._h, _p(c), _p(k)), "or_last_nominations")
        return c, k

    def pairs_within(self, rcut, brute):
        n = lib().or_pairs_within(self._h, float(rcut), int(brute), None, 0)
        out = np.zeros((max(n, 1), 2), dtype=np.int32)
        lib().or_pairs_within(self._h, float(rcut), int(brute), _p(out), n)
        return out[:n]

    def graph_distance(self, i, j):
        return lib().or_graph_distance(self._h, int(i), int(j))
