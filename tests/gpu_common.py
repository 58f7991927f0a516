"""Shared helpers of the GPU parity tests: build the same system in the HIP
library and in the oracle, and compare."""
import math
import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def fig2_rules():
    with open(os.path.join(HERE, "golden", "fig2_rules.txt")) as f:
        return synth.parse_script(f.read())


def both(system, ff, rules, seed=7, precision=0, generate=True):
    import paper_1108_4214_amd as pk
    g = pk.System(system.n, system.L, seed, precision).configure(system, ff, rules, generate=generate)
    o = oracle.Oracle.from_system(system, ff, rules, seed=seed, generate=generate)
    return g, o


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_bead_err(a, b):
    """max over beads of |a_i - b_i| / max(|b_i|, F_rms): a wrong force on a few beads
    shows here even where the global relative L2 norm averages it away"""
    nb = np.linalg.norm(b, axis=1)
    rms = float(np.sqrt(np.mean(nb * nb))) if nb.size else 0.0
    den = np.maximum(nb, max(rms, 1e-300))
    return float(np.max(np.linalg.norm(a - b, axis=1) / den)) if nb.size else 0.0


def forces_close(a, b, tol, tol_bead=None):
    """(ok, message): relative L2 norm of the difference <= tol and every bead's error
    <= tol_bead relative to max(|F_i|, F_rms).

    tol_bead defaults to 10 tol.  A bead's force is a sum of terms each correct to
    about 1e-6 of itself in float arithmetic (the WCA force goes as r^-14, so the
    6e-8 rounding of a separation is amplified about 14 times, plus some ten more
    roundings) and to about 1e-15 in double; in the packed fixtures single terms
    reach ten times F_rms on beads whose net force is far smaller, so the error of
    one bead relative to F_rms can reach ten times the per-term figure.  A bead on a
    wrong code path is off by order one."""
    tb = 10.0 * tol if tol_bead is None else tol_bead
    g, p = rel_l2(a, b), per_bead_err(a, b)
    return (g <= tol and p <= tb), f"relative L2 {g:.3e} (tol {tol:.1e}), per bead {p:.3e} (tol {tb:.1e})"


def as_set(rows):
    return {tuple(r) for r in np.asarray(rows).tolist()}


def same_topology(g, o):
    return (np.array_equal(g.bonds(), o.bonds()) and np.array_equal(g.angles(), o.angles())
            and np.array_equal(g.dihedrals(), o.dihedrals()))


def topo_diff(g, o):
    out = {}
    for name in ("bonds", "angles", "dihedrals"):
        a, b = as_set(getattr(g, name)()), as_set(getattr(o, name)())
        out[name] = (sorted(a - b)[:5], sorted(b - a)[:5])
    return out


def copy_oracle_from_gpu(g, system, ff, rules, seed, step):
    """A fresh oracle holding the GPU's current state and topology (shadow mode)."""
    x, v = g.state()
    o = oracle.Oracle(system.n, system.L, seed)
    o.set_state(x, v, system.type)
    o.set_reactive(system.reactive)
    o.set_bonds(g.bonds())
    o.set_angles(g.angles())
    o.set_dihedrals(g.dihedrals())
    o.set_forcefield(ff)
    o.set_rules(rules)
    o.set_step(step)
    return o


def perturbed(system, scale, seed):
    """A copy of the system with Gaussian-jittered positions."""
    import dataclasses
    rng = np.random.default_rng(seed)
    return dataclasses.replace(system, x=synth.wrap(system.x + rng.normal(0, scale, size=system.x.shape), system.L))


def fig2_dynamic_setup(n_strand=30, n_nt=5, L=6.0, seed=3):
    rng = np.random.default_rng(seed)
    xs, ts, bonds = [], [], []
    for s_ in range(n_strand):
        o = rng.uniform(0, L, size=3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        base = len(ts)
        for k in range(n_nt):
            xs.append(o + 0.5 * k * u)
            ts.append(int(rng.integers(1, 5)))
        for k in range(n_nt - 1):
            bonds.append((base + k, base + k + 1, 2, 3))
    x = synth.wrap(np.array(xs), L)
    n = len(ts)
    sysm = synth.System(L=L, x=x, v=synth.maxwell_boltzmann(rng, n, 1.0), type=np.array(ts, dtype=np.int32),
                        reactive=np.ones(n, dtype=np.uint8), bonds=np.array(bonds, dtype=np.int32))
    ff = synth.ForceField(eps=0.0, gamma=1.0, dt=0.005)
    ff.bonds = {1: (5.0, 0.6), 2: (20.0, 0.5), 3: (20.0, 0.5)}
    ff.angles = {1: (1.0, math.pi), 2: (1.0, 0.5 * math.pi)}
    ff.dihedrals = {1: (1.0, 0.0), 2: (1.0, 0.0), 3: (1.0, math.pi)}
    return sysm, ff, fig2_rules()
