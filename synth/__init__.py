"""Seeded synthetic inputs for the dynamic-bonding hot path.

This module builds *inputs only*: bead coordinates, velocities, bead types,
reactive flags, the initial bond graph, force-field parameters and rule tables.
It holds none of the method's arithmetic (no forces, no matching, no
enumeration), so that both the GPU library and the CPU oracle can be fed from
it without sharing any computation.

Two bead models are generated:

* the 2-bead/nucleotide model (backbone bead P, type 5, plus a base bead of
  type 1-4 = A, T, C, G) used by the benchmark workloads, with bond types
  1 = hybridization, 2/3 = directional backbone (a P bead stores 2 towards its
  3' neighbour and 3 towards its 5' neighbour, following the directional-bond
  convention of section 2 of the paper), 4 = P-base, 5 = weak;
* the paper's own 1-bead/nucleotide model (section 3, Fig. 2), used as a
  topology fixture for the pattern rules.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# bead types (section 3: A, T, C, G = 1..4); 5 = backbone bead of the 2-bead model,
# 6 = DPD solvent bead
A, T, C, G, P = 1, 2, 3, 4, 5
SOLVENT = 6
COMPLEMENT = {A: T, T: A, C: G, G: C}
# bond types
H_BOND, BB_3P, BB_5P, PB_BOND, WEAK = 1, 2, 3, 4, 5
ANY = 0            # bead-type wildcard
ALL_TYPES = 0xFFFFFFFF  # bond-type wildcard mask


def mask(*types: int) -> int:
    """Bond-type set as a bitmask (bit t <=> bond type t)."""
    m = 0
    for t in types:
        m |= 1 << t
    return m


@dataclasses.dataclass
class System:
    """One simulation box. Global bead id = row index."""
    L: float
    x: np.ndarray            # (N,3) float64, wrapped into [0, L)
    v: np.ndarray            # (N,3) float64 (half-step velocity of the leapfrog state)
    type: np.ndarray         # (N,) int32
    reactive: np.ndarray     # (N,) uint8
    bonds: np.ndarray        # (nb,4) int32: i, j, type stored by i, type stored by j
    angles: Optional[np.ndarray] = None     # (na,4) int32: type, a, b, c
    dihedrals: Optional[np.ndarray] = None  # (nd,5) int32: type, a, b, c, d

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclasses.dataclass
class ForceField:
    eps: float = 1.0
    sigma: float = 1.0
    rc: float = 2.0 ** (1.0 / 6.0)
    exclude_depth: int = 1
    pair: str = "wca"        # "wca" or "dpd" (soft conservative + dissipative + random pair forces)
    dpd_a: float = 25.0
    dpd_gamma: float = 4.5
    bonds: dict = dataclasses.field(default_factory=dict)      # type -> (K, r0)
    wells: dict = dataclasses.field(default_factory=dict)      # type -> (U_min, r_well, r_zero, r_cut)
    angles: dict = dataclasses.field(default_factory=dict)     # type -> (K, theta0)
    dihedrals: dict = dataclasses.field(default_factory=dict)  # type -> (K, phi0)
    T0: float = 1.0
    T1: float = 1.0
    ramp_steps: int = 0
    gamma: float = 1.0
    dt: float = 0.005


@dataclasses.dataclass
class RuleSet:
    """Rules in call order (the order decides 'last matching rule wins')."""
    every: int = 10
    paircheck13: int = 0
    paircheck14: int = 0
    rules: List[tuple] = dataclasses.field(default_factory=list)
    accept: str = "pair"     # "pair": one uniform per pair; "average": the mean of one uniform per bead


@dataclasses.dataclass
class Workload:
    name: str
    system: System
    ff: ForceField
    rules: RuleSet
    steps: int
    seed: int


# ----------------------------------------------------------------------------------
# rule tables
# ----------------------------------------------------------------------------------

def rules_t2(p: float = 0.5, every: int = 10, r_create: float = 1.5, r_kill: float = 2.0,
             convert: bool = False) -> RuleSet:
    """Pattern/rule table for the 2-bead model.

    Hybridization bonds between complementary bases, killed beyond r_kill, at most
    one per bead; straight backbone angles (as the paper's first angle rule), the
    straight rung angle P-base-base' that appears with a hybridization bond, and
    cis stacking dihedrals base-P-P-base across each backbone bond.
    With ``convert`` the stress-test extension is added: a weak bond type 5,
    hybridization bonds converted to it beyond 1.8 with probability 0.9, weak bonds
    killed beyond 2.5, at most one weak bond per bead.
    """
    r = [
        ("create", H_BOND, A, T, r_create, p),
        ("create", H_BOND, C, G, r_create, p),
    ]
    if convert:
        r.append(("convert", H_BOND, WEAK, 1.8, 0.9))
        r.append(("kill", WEAK, 2.5))
        r.append(("maxbond", WEAK, ANY, 1))
    r += [
        ("kill", H_BOND, r_kill),
        ("maxbond", H_BOND, ANY, 1),
        ("angle", 1, (P, P, P), (mask(BB_3P), mask(BB_5P))),
        ("angle", 1, (P, ANY, ANY), (mask(PB_BOND), mask(H_BOND))),
        ("dihedral", 1, (ANY, P, P, ANY), (mask(PB_BOND), mask(BB_3P, BB_5P), mask(PB_BOND))),
    ]
    return RuleSet(every=every, rules=r)


def ff_t2(T0=1.0, T1=1.0, ramp_steps=0, gamma=1.0, dt=0.005, weak=False) -> ForceField:
    ff = ForceField(T0=T0, T1=T1, ramp_steps=ramp_steps, gamma=gamma, dt=dt)
    ff.bonds = {H_BOND: (50.0, 1.2), BB_3P: (100.0, 1.0), BB_5P: (100.0, 1.0), PB_BOND: (100.0, 1.0)}
    if weak:
        ff.bonds[WEAK] = (10.0, 1.5)
    ff.angles = {1: (10.0, math.pi)}
    ff.dihedrals = {1: (5.0, 0.0)}
    return ff


def ff_dpd(T=1.0, gamma_dpd=100.0, dt=0.01, a=25.0) -> ForceField:
    """The 2-bead model's bonded terms in the paper's DPD setting (section 3):
    a = 25, rc = 1, pair interactions off below three bonds apart, dt = 0.01, the
    DPD pair thermostat alone (no Langevin force); gamma_dpd = 100 is the
    friction read from the paper's stated value (its units are the friction's)."""
    ff = ff_t2(T0=T, T1=T, gamma=0.0, dt=dt)
    ff.pair, ff.dpd_a, ff.dpd_gamma, ff.rc, ff.exclude_depth = "dpd", a, gamma_dpd, 1.0, 2
    return ff


def ff_dna1(T=1.0, gamma_dpd=100.0, dt=0.01) -> ForceField:
    """The paper's 1-bead DNA force field (section 3) in DPD solvent: hybridization
    well (U_min 1, well 0.6, zero and cutoff 1.0), backbone wells of both
    directions (U_min 10, well 0.3, zero 0.6), straight backbone angles (K 20) and
    backbone-hybridization right angles (K 1), stacking dihedrals K (1 + d cos phi)
    with d = -1 (cis: types 1, 2) and d = +1 (trans: type 3), i.e. cosine
    dihedrals at phi0 = 0 and pi; DPD as in ff_dpd."""
    ff = ff_dpd(T=T, gamma_dpd=gamma_dpd, dt=dt)
    ff.bonds = {}
    ff.wells = {H_BOND: (1.0, 0.6, 1.0, 1.0), BB_3P: (10.0, 0.3, 0.6, math.inf), BB_5P: (10.0, 0.3, 0.6, math.inf)}
    ff.angles = {1: (20.0, math.pi), 2: (1.0, 0.5 * math.pi)}
    ff.dihedrals = {1: (1.0, 0.0), 2: (1.0, 0.0), 3: (1.0, math.pi)}
    return ff


def rules_fig2() -> RuleSet:
    """The rule table of the paper's 1-bead DNA model (Fig. 2): hybridization of
    complementary bases within 0.6 with p = 1, directional backbone ligation
    between bead types 2 and 3 within 0.3 with p = 0.1, hybridization bonds killed
    beyond 1.0, at most one bond of each type per bead, straight-backbone and
    backbone-hybridization angles, three stacking dihedral patterns; a sweep every
    step with paircheck14."""
    any3, any4 = (ANY, ANY, ANY), (ANY, ANY, ANY, ANY)
    return RuleSet(every=1, paircheck14=1, rules=[
        ("create", H_BOND, A, T, 0.6, 1.0),
        ("create", H_BOND, C, G, 0.6, 1.0),
        ("createdir", BB_3P, BB_5P, T, C, 0.3, 0.1),
        ("kill", H_BOND, 1.0),
        ("maxbond", H_BOND, ANY, 1),
        ("maxbond", BB_3P, ANY, 1),
        ("maxbond", BB_5P, ANY, 1),
        ("angle", 1, any3, (mask(BB_3P), mask(BB_5P))),
        ("angle", 2, any3, (mask(H_BOND), mask(BB_3P, BB_5P))),
        ("dihedral", 1, any4, (mask(H_BOND), mask(BB_3P, BB_5P), mask(H_BOND))),
        ("dihedral", 2, any4, (mask(BB_3P), mask(H_BOND), mask(BB_5P))),
        ("dihedral", 3, any4, (mask(BB_3P), mask(H_BOND), mask(BB_3P))),
        ("dihedral", 3, any4, (mask(BB_5P), mask(H_BOND), mask(BB_5P))),
    ])


def parse_script(text: str) -> RuleSet:
    """Parse the rule syntax of the paper's Fig. 1 (one rule per line).

    The first non-empty line is ``fix <id> <group> bonddynamics <every> [paircheck13]
    [paircheck14]``.  A line may carry a leading ``N:`` label.  Bead types use ``*``
    for any; bond types in pattern rules are comma-separated sets or ``*``.
    """
    rs = RuleSet(rules=[])
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0].endswith(":") and tok[0][:-1].isdigit():
            tok = tok[1:]
        if not tok:
            continue
        key = tok[0].lower()

        def bead(s):
            return ANY if s == "*" else int(s)

        def bset(s):
            if s == "*":
                return ALL_TYPES
            return mask(*[int(t) for t in s.split(",")])

        if key == "fix":
            i = [t.lower() for t in tok].index("bonddynamics")
            rs.every = int(tok[i + 1])
            rest = [t.lower() for t in tok[i + 2:]]
            rs.paircheck13 = int("paircheck13" in rest)
            rs.paircheck14 = int("paircheck14" in rest)
        elif key == "createbond":
            rs.rules.append(("create", int(tok[1]), bead(tok[2]), bead(tok[3]), float(tok[4]), float(tok[5])))
        elif key == "createdirbond":
            rs.rules.append(("createdir", int(tok[1]), int(tok[2]), bead(tok[3]), bead(tok[4]),
                             float(tok[5]), float(tok[6])))
        elif key == "breakbond":
            rs.rules.append(("break", int(tok[1]), float(tok[2]), float(tok[3])))
        elif key == "killbond":
            rs.rules.append(("kill", int(tok[1]), float(tok[2])))
        elif key == "convertbond":
            # Fig. 1 gives no distance; an optional one may follow the types
            if len(tok) == 4:
                rs.rules.append(("convert", int(tok[1]), int(tok[2]), 0.0, float(tok[3])))
            else:
                rs.rules.append(("convert", int(tok[1]), int(tok[2]), float(tok[3]), float(tok[4])))
        elif key == "maxbond":
            rs.rules.append(("maxbond", int(tok[1]), bead(tok[2]), int(tok[3])))
        elif key == "createangle":
            rs.rules.append(("angle", int(tok[1]), tuple(bead(t) for t in tok[2:5]),
                             tuple(bset(t) for t in tok[5:7])))
        elif key == "createdihedral":
            rs.rules.append(("dihedral", int(tok[1]), tuple(bead(t) for t in tok[2:6]),
                             tuple(bset(t) for t in tok[6:9])))
        else:
            raise ValueError(f"unknown rule keyword: {tok[0]}")
    return rs


# ----------------------------------------------------------------------------------
# geometry builders (2-bead model)
# ----------------------------------------------------------------------------------

class _Builder:
    def __init__(self):
        self.x: List[np.ndarray] = []
        self.type: List[int] = []
        self.bonds: List[Tuple[int, int, int, int]] = []

    @property
    def n(self):
        return len(self.type)

    def add(self, pos, t):
        self.x.append(np.asarray(pos, dtype=np.float64))
        self.type.append(int(t))
        return self.n - 1

    def strand(self, P_pos, B_pos, seq):
        """One strand listed 5'->3'; P_pos/B_pos are per-nucleotide positions in that order.
        Returns (P ids, base ids) in 5'->3' order."""
        pid, bid = [], []
        for m, s in enumerate(seq):
            pid.append(self.add(P_pos[m], P))
            bid.append(self.add(B_pos[m], s))
            self.bonds.append((pid[-1], bid[-1], PB_BOND, PB_BOND))
        for m in range(len(seq) - 1):
            # P_m's 3' neighbour is P_{m+1}: P_m stores 2 for it, P_{m+1} stores 3 for P_m
            self.bonds.append((pid[m], pid[m + 1], BB_3P, BB_5P))
        return pid, bid


def _rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def random_sequence(rng, n) -> List[int]:
    return [int(t) for t in rng.integers(1, 5, size=n)]


def add_duplex(b: _Builder, seq, origin, flip_x=False, flip_y=False, hybridized=True):
    """Ideal ladder: strand 1 P at (k,0,0), base at (k,1,0); strand 2 base at
    (k,2.2,0), P at (k,3.2,0). Strand 1 runs 5'->3' along +x, strand 2 antiparallel."""
    n = len(seq)
    k = np.arange(n, dtype=np.float64)
    if flip_x:
        k = (n - 1) - k
    ys = np.array([0.0, 1.0, 2.2, 3.2])
    if flip_y:
        ys = 3.2 - ys
    o = np.asarray(origin, dtype=np.float64)
    P1 = [o + [k[m], ys[0], 0.0] for m in range(n)]
    B1 = [o + [k[m], ys[1], 0.0] for m in range(n)]
    p1, b1 = b.strand(P1, B1, seq)
    seq2 = [COMPLEMENT[s] for s in reversed(seq)]   # partner strand 5'->3'
    P2 = [o + [k[n - 1 - m], ys[3], 0.0] for m in range(n)]
    B2 = [o + [k[n - 1 - m], ys[2], 0.0] for m in range(n)]
    p2, b2 = b.strand(P2, B2, seq2)
    if hybridized:
        for m in range(n):
            b.bonds.append((b1[m], b2[n - 1 - m], H_BOND, H_BOND))
    return p1, b1, p2, b2


def maxwell_boltzmann(rng, n, T) -> np.ndarray:
    v = rng.normal(0.0, math.sqrt(T), size=(n, 3)) if n else np.zeros((0, 3))
    if n > 1:
        v -= v.mean(axis=0)
    return v


def wrap(x, L):
    """Bring coordinates into [0, L) (input preparation only)."""
    y = np.mod(x, L)
    y[y >= L] = 0.0
    return y


def _finish(b: _Builder, L, rng_v, T, reactive=None) -> System:
    x = wrap(np.array(b.x, dtype=np.float64).reshape(-1, 3), L)
    n = x.shape[0]
    typ = np.array(b.type, dtype=np.int32)
    bonds = np.array(b.bonds, dtype=np.int32).reshape(-1, 4)
    react = np.ones(n, dtype=np.uint8) if reactive is None else reactive
    return System(L=float(L), x=x, v=maxwell_boltzmann(rng_v, n, T), type=typ, reactive=react, bonds=bonds)


def pack_duplexes(lengths: Sequence[int], L: float, rng, hybridized=True, seqs=None,
                  jitter=0.1) -> _Builder:
    """Place flat ladders into a slot lattice (random slot order, jitter and flips)."""
    b = _Builder()
    if len(lengths) == 0:
        return b
    lmax = max(lengths)
    nx = max(1, int(L // (lmax + 1.5)))
    ny = max(1, int(L // 4.3))
    per_layer = nx * ny
    nz = -(-len(lengths) // per_layer)
    dz = L / nz
    if dz < 1.1 or (lmax + 1.5) > L:
        raise ValueError("duplexes do not fit in the box")
    sx, sy = L / nx, L / ny
    slots = rng.permutation(nx * ny * nz)[: len(lengths)]
    for d, n in enumerate(lengths):
        s = int(slots[d])
        ix, iy, iz = s % nx, (s // nx) % ny, s // per_layer
        org = np.array([ix * sx, iy * sy, iz * dz]) + rng.uniform(-jitter, jitter, size=3)
        seq = seqs[d] if seqs is not None else random_sequence(rng, n)
        add_duplex(b, seq, org, flip_x=bool(rng.integers(2)), flip_y=bool(rng.integers(2)),
                   hybridized=hybridized)
    return b


def pack_duplexes_rows(lengths: Sequence[int], L: float, rng, jitter=0.1) -> _Builder:
    """Flat ladders laid end to end along x-rows (each takes its length + 1.5 sigma),
    rows on a ny x nz lattice (row pitch at least 4.2 sigma in y, 1 sigma in z) in
    random order, with jitter and flips; for boxes too small for one ladder per slot."""
    b = _Builder()
    order = rng.permutation(len(lengths))
    rows, cur, used = [], [], 0.0
    for d in order:
        w = lengths[d] + 1.5
        if w > L:
            raise ValueError("duplexes do not fit in the box")
        if used + w > L and cur:
            rows.append(cur)
            cur, used = [], 0.0
        cur.append(int(d))
        used += w
    if cur:
        rows.append(cur)
    ny = max(1, int(L // 4.2))
    nz = -(-len(rows) // ny)
    dz = L / nz
    if dz < 1.0:
        raise ValueError("duplexes do not fit in the box")
    sy = L / ny
    slots = rng.permutation(ny * nz)[: len(rows)]
    for row, sl in zip(rows, slots):
        iy, iz = int(sl) % ny, int(sl) // ny
        x0 = 0.0
        for d in row:
            n = lengths[d]
            org = np.array([x0, iy * sy, iz * dz]) + rng.uniform(-jitter, jitter, size=3)
            add_duplex(b, random_sequence(rng, n), org, flip_x=bool(rng.integers(2)), flip_y=bool(rng.integers(2)))
            x0 += n + 1.5
    return b


# ----------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------

def c1(seed_w=1, seed_d=11) -> Workload:
    """Two complementary 10-nt strands as straight, unhybridized rods at random
    position and orientation in a 20 sigma periodic cube."""
    rng = np.random.default_rng(seed_w)
    L = 20.0
    seq = random_sequence(rng, 10)
    seqs = [seq, [COMPLEMENT[s] for s in reversed(seq)]]
    while True:
        b = _Builder()
        for s in seqs:
             R = _rotation(rng)
             o = rng.uniform(0, L, size=3)
             P_pos = [o + R @ np.array([m, 0.0, 0.0]) for m in range(10)]
             B_pos = [o + R @ np.array([m, 1.0, 0.0]) for m in range(10)]
             b.strand(P_pos, B_pos, s)
        x = np.array(b.x)
        d = x[:20, None, :] - x[None, 20:, :]
        d -= L * np.round(d / L)
        if np.sqrt((d ** 2).sum(-1)).min() >= 1.0:
            break
    sysm = _finish(b, L, np.random.default_rng(seed_d), 1.0)
    return Workload("c1: 2 x 10-nt strands, 40 beads, L=20", sysm, ff_t2(), rules_t2(p=0.5, every=10),
                    10000, seed_d)


def duplex_box(n_duplex, n_bp, rho, seed_w, seed_d, T=1.0) -> System:
    n_beads = 4 * n_bp * n_duplex
    L = (n_beads / rho) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed_w)
    b = pack_duplexes([n_bp] * n_duplex, L, rng)
    return _finish(b, L, np.random.default_rng(seed_d), T)


def dpd_solution(n_duplex, n_bp, n_total, rho=3.0, seed_w=9, seed_d=19, T=1.0) -> System:
    """Duplexes of the 2-bead model in explicit DPD solvent at number density rho
    (the paper's DNA runs use 3): the duplexes are packed as in duplex_box, the
    remaining n_total - 4 n_bp n_duplex beads are solvent (type 6, not reactive)
    at uniform random positions (the DPD pair force is soft, so overlaps are
    harmless)."""
    n_dna = 4 * n_bp * n_duplex
    if n_total < n_dna:
        raise ValueError("n_total below the duplex beads")
    L = (n_total / rho) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed_w)
    b = pack_duplexes([n_bp] * n_duplex, L, rng) if n_duplex else _Builder()
    for p in rng.uniform(0.0, L, size=(n_total - n_dna, 3)):
        b.add(p, SOLVENT)
    react = np.zeros(n_total, dtype=np.uint8)
    react[:n_dna] = 1
    return _finish(b, L, np.random.default_rng(seed_d), T, reactive=react)


def dpd_c3(seed_w=23, seed_d=33) -> Workload:
    """1,000,000 beads at density 3 (the paper's DPD solvent density): 2,500
    hybridized 20-bp duplexes of the 2-bead model (200,000 beads) in 800,000
    solvent beads; DPD a = 25, friction 100, T = 1, dt = 0.01; hybridization
    sweep every 10 steps."""
    s = dpd_solution(2500, 20, 1_000_000, 3.0, seed_w, seed_d)
    return Workload("dpd: 2500 x 20-bp duplexes in DPD solvent, 1000000 beads, rho=3", s, ff_dpd(),
                    rules_t2(p=0.5, every=10), 10000, seed_d)


def dna1_solution(n_duplex, n_bp, n_total, rho=3.0, seed_w=29, seed_d=39, T=1.0, bb=0.3, hyb=0.6) -> System:
    """Duplexes of the paper's 1-bead model (ladders of ladder_1bead's layout:
    backbone spacing bb, strands hyb apart, random sequences) in DPD solvent
    (type 5, not reactive) at number density rho.  The flat ladders sit on a slot
    lattice (pitch: length + 1 sigma along x, 1.6 sigma in y, 1 sigma in z) in
    random slot order with random flips and jitter; solvent beads are uniform."""
    n_dna = 2 * n_bp * n_duplex
    if n_total < n_dna:
        raise ValueError("n_total below the duplex beads")
    L = (n_total / rho) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed_w)
    px, py, pz = (n_bp - 1) * bb + 1.0, 1.6, 1.0
    nx, ny, nz = int(L // px), int(L // py), int(L // pz)
    if nx * ny * nz < n_duplex:
        raise ValueError("duplexes do not fit in the box")
    slots = rng.permutation(nx * ny * nz)[:n_duplex]
    b = _Builder()
    for sl in slots:
        sl = int(sl)
        org = np.array([(sl % nx) * px, ((sl // nx) % ny) * py, (sl // (nx * ny)) * pz]) + rng.uniform(-0.05, 0.05, 3)
        seq = random_sequence(rng, n_bp)
        k = np.arange(n_bp, dtype=np.float64)
        if rng.integers(2):
            k = (n_bp - 1) - k
        y1, y2 = (0.0, hyb) if rng.integers(2) else (hyb, 0.0)
        s1 = [b.add(org + [k[m] * bb, y1, 0.0], seq[m]) for m in range(n_bp)]
        s2 = [b.add(org + [k[m] * bb, y2, 0.0], COMPLEMENT[seq[m]]) for m in range(n_bp)]
        for m in range(n_bp - 1):
            b.bonds.append((s1[m], s1[m + 1], BB_3P, BB_5P))   # strand 1: m+1 is 3' of m
            b.bonds.append((s2[m], s2[m + 1], BB_5P, BB_3P))   # strand 2 antiparallel: m is 3' of m+1
        for m in range(n_bp):
            b.bonds.append((s1[m], s2[m], H_BOND, H_BOND))
    for p in rng.uniform(0.0, L, size=(n_total - n_dna, 3)):
        b.add(p, P)
    react = np.zeros(n_total, dtype=np.uint8)
    react[:n_dna] = 1
    return _finish(b, L, np.random.default_rng(seed_d), T, reactive=react)


def dna1_c3(seed_w=29, seed_d=39) -> Workload:
    """1,000,000 beads at density 3: 5,000 hybridized 20-bp duplexes of the
    paper's 1-bead model (200,000 beads) in 800,000 DPD solvent beads; the paper's
    force field (ff_dna1) and Fig. 2 rule table (sweep every step)."""
    s = dna1_solution(5000, 20, 1_000_000, 3.0, seed_w, seed_d)
    return Workload("dna1: 5000 x 20-bp duplexes of the 1-bead model in DPD solvent, 1000000 beads, rho=3", s,
                    ff_dna1(), rules_fig2(), 10000, seed_d)


def c2(seed_w=2, seed_d=12) -> Workload:
    """1,000 pre-hybridized 20-bp duplexes (80,000 beads) at density 0.5."""
    s = duplex_box(1000, 20, 0.5, seed_w, seed_d)
    return Workload("c2: 1000 x 20-bp duplexes, 80000 beads, rho=0.5", s, ff_t2(), rules_t2(p=0.5, every=10),
                    10000, seed_d)


def c3(seed_w=3, seed_d=13) -> Workload:
    """6,250 pre-hybridized 40-bp duplexes (12,500 strands, 1,000,000 beads) at
    density 0.5; temperature ramp 0.5 -> 1.5 over 1e5 steps."""
    s = duplex_box(6250, 40, 0.5, seed_w, seed_d, T=0.5)
    return Workload("c3: 12500 x 40-nt strands (6250 duplexes), 1000000 beads, rho=0.5", s,
                    ff_t2(T0=0.5, T1=1.5, ramp_steps=100000), rules_t2(p=0.5, every=10), 100000, seed_d)


def c3_shard(k, n_shards, seed_w=3, seed_d=13) -> Workload:
    """One of n_shards independent boxes that together hold the 1,000,000-bead
    workload's recipe: 6250 / n_shards pre-hybridized 40-bp duplexes at density 0.5,
    the same force field, temperature ramp and rules, seeds offset by the shard."""
    nd = max(1, int(round(6250 / n_shards)))
    s = duplex_box(nd, 40, 0.5, seed_w + 1000 * (k + 1), seed_d + 1000 * (k + 1), T=0.5)
    return Workload(f"c3 shard {k} of {n_shards}: {nd} duplexes, {s.n} beads, rho=0.5", s,
                    ff_t2(T0=0.5, T1=1.5, ramp_steps=100000), rules_t2(p=0.5, every=10), 100000,
                    seed_d + 1000 * (k + 1))


def c5(seed_w=5, seed_d=15, n_strands=100000) -> Workload:
    """Random 20-nt single strands on a cubic lattice at density 0.85 (4,000,000
    beads at the default size), sweep every step, conversion to a weak type."""
    rng = np.random.default_rng(seed_w)
    n_beads = 40 * n_strands
    L = (n_beads / 0.85) ** (1.0 / 3.0)
    m = 160
    while (m // 20) * (m // 2) * m < n_strands:
        m += 20
    # rows of m sites along x hold m//20 ribbons; P row and base row are adjacent in y
    a = L / m
    per_row = m // 20
    n_rows = (m // 2) * m
    slots = np.sort(rng.permutation(per_row * n_rows)[:n_strands])
    b = _Builder()
    for s in slots:
        row, k = divmod(int(s), per_row)
        iy, iz = row % (m // 2), row // (m // 2)
        up = bool(rng.integers(2))
        yP = (2 * iy + (0 if up else 1)) * a
        yB = (2 * iy + (1 if up else 0)) * a
        xs = (20 * k + np.arange(20)) * a
        if rng.integers(2):
            xs = xs[::-1]
        P_pos = [np.array([xs[q], yP, iz * a]) for q in range(20)]
        B_pos = [np.array([xs[q], yB, iz * a]) for q in range(20)]
        b.strand(P_pos, B_pos, random_sequence(rng, 20))
    sysm = _finish(b, L, np.random.default_rng(seed_d), 1.0)
    ff = ff_t2(gamma=0.0, dt=0.002, weak=True)
    return Workload(f"c5: {n_strands} x 20-nt strands, {n_beads} beads, rho=0.85", sysm, ff,
                    rules_t2(p=0.9, every=1, convert=True), 10000, seed_d)


def c4(seed_w=4, seed_d=14, n_rep=64) -> List[Workload]:
    """Temperature ladder of uneven replicas (log-uniform 2k..50k beads) filled with
    duplexes at density 0.5; T_r = 0.6 + 0.8 r/63.  Duplex lengths are uniform on
    10..40 bp, capped by the box edge minus 3; ladders are laid end to end along
    x-rows.  When a draw does not fit, the cap is lowered by 1 and the replica is
    drawn again."""
    rng = np.random.default_rng(seed_w)
    out = []
    for r in range(n_rep):
        target = int(round(math.exp(rng.uniform(math.log(2000), math.log(50000)))))
        L = (target / 0.5) ** (1.0 / 3.0)
        cap = min(40, int(L - 3.0))
        while True:
            lo = min(10, cap)
            lengths, tot = [], 0
            while tot < target:
                n = int(rng.integers(lo, cap + 1))
                lengths.append(n)
                tot += 4 * n
            Lr = (tot / 0.5) ** (1.0 / 3.0)
            try:
                b = pack_duplexes_rows(lengths, Lr, rng)
                break
            except ValueError:
                if cap <= 3:
                    raise
                cap -= 1
        T = 0.6 + 0.8 * r / max(1, n_rep - 1)
        s = _finish(b, Lr, np.random.default_rng(seed_d + 1000 * r), T)
        out.append(Workload(f"c4 replica {r}", s, ff_t2(T0=T, T1=T), rules_t2(p=0.5, every=10), 10000,
                            seed_d + r))
    return out


def small_duplexes(n_duplex=6, n_bp=8, rho=0.05, seed_w=7, seed_d=17, T=1.0) -> System:
    return duplex_box(n_duplex, n_bp, rho, seed_w, seed_d, T)


def single_strands(n_strand, n_nt, L, seed_w=8, seed_d=18, T=1.0) -> System:
    """Unhybridized flat strands (P row + base row) packed into slots."""
    rng = np.random.default_rng(seed_w)
    b = _Builder()
    nx = max(1, int(L // (n_nt + 1.5)))
    ny = max(1, int(L // 2.2))
    nz = -(-n_strand // (nx * ny))
    dz = L / nz
    if dz < 1.1:
        raise ValueError("strands do not fit")
    slots = rng.permutation(nx * ny * nz)[:n_strand]
    for s in slots:
        ix, iy, iz = int(s) % nx, (int(s) // nx) % ny, int(s) // (nx * ny)
        o = np.array([ix * L / nx, iy * L / ny, iz * dz])
        P_pos = [o + [m, 0.0, 0.0] for m in range(n_nt)]
        B_pos = [o + [m, 1.0, 0.0] for m in range(n_nt)]
        b.strand(P_pos, B_pos, random_sequence(rng, n_nt))
    return _finish(b, L, np.random.default_rng(seed_d), T)


def random_gas(n, L, seed=0, n_types=5, min_dist=0.0) -> System:
    """Uniform random beads (no bonds); optional rejection of close pairs."""
    rng = np.random.default_rng(seed)
    if min_dist <= 0:
        x = rng.uniform(0, L, size=(n, 3))
    else:
        pts = []
        while len(pts) < n:
            p = rng.uniform(0, L, size=3)
            ok = True
            for q in pts:
                d = p - q
                d -= L * np.round(d / L)
                if (d @ d) < min_dist * min_dist:
                    ok = False
                    break
            if ok:
                pts.append(p)
        x = np.array(pts).reshape(-1, 3)
    typ = rng.integers(1, n_types + 1, size=n).astype(np.int32)
    return System(L=float(L), x=wrap(x, L), v=maxwell_boltzmann(rng, n, 1.0), type=typ,
                  reactive=np.ones(n, dtype=np.uint8), bonds=np.zeros((0, 4), dtype=np.int32))


def isolated_pairs(m, r, L_per_pair=4.0, seed=0, types=(A, T)) -> System:
    """m unbonded bead pairs (types[0], types[1]) at separation r, on a lattice with
    spacing L_per_pair, random orientations."""
    rng = np.random.default_rng(seed)
    k = int(math.ceil(m ** (1.0 / 3.0)))
    L = k * L_per_pair
    xs, ts = [], []
    for q in range(m):
        c = np.array([q % k, (q // k) % k, q // (k * k)], dtype=np.float64) * L_per_pair + 1.0
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        xs += [c, c + r * u]
        ts += [types[0], types[1]]
    x = wrap(np.array(xs), L)
    n = len(ts)
    return System(L=float(L), x=x, v=np.zeros((n, 3)), type=np.array(ts, dtype=np.int32),
                  reactive=np.ones(n, dtype=np.uint8), bonds=np.zeros((0, 4), dtype=np.int32))


def boundary_pairs(m, r_in, r_out, L, seed=0, types=(A, T)) -> System:
    """m unbonded bead pairs (types[0], types[1]) straddling the faces, edges and one
    corner of a large periodic box: the first bead within 0.3 of the upper face(s),
    the partner across it.  Alternate pairs sit at separation r_in and r_out.  First
    beads take distinct points of a lattice of spacing 8 on the faces (and along the
    edges) whose other coordinates are also near L, where float copies of the
    coordinates are coarsest; beads of different pairs stay more than 2.4 apart."""
    rng = np.random.default_rng(seed)
    g = int(math.sqrt(m)) + 2
    grid = L - 4.0 - 8.0 * np.arange(g)
    if grid[-1] < 4.0:
        raise ValueError("box too small for that many pairs")
    slots = []                                   # (straddled axes mask, point)
    for k in range(3):                           # faces
        o1, o2 = [a for a in range(3) if a != k]
        for u in grid:
            for v in grid:
                pnt = np.zeros(3)
                pnt[o1], pnt[o2] = u, v
                slots.append((1 << k, pnt))
    for k in range(3):                           # edges parallel to axis k
        for u in grid:
            pnt = np.zeros(3)
            pnt[k] = u
            slots.append((7 & ~(1 << k), pnt))
    slots.append((7, np.zeros(3)))               # the corner
    n_edge = 3 * len(grid) + 1
    if m > len(slots):
        raise ValueError("box too small for that many pairs")
    # every edge and corner slot first (up to a third of the pairs), then faces at random
    take_e = min(n_edge, m // 3)
    pick = list(range(len(slots) - n_edge, len(slots)))[-take_e:] if take_e else []
    pick += list(rng.choice(len(slots) - n_edge, size=m - take_e, replace=False))
    xs, ts = [], []
    for q, idx in enumerate(pick):
        mask, a = slots[int(idx)]
        a = a.copy()
        d = rng.normal(size=3)
        for k in range(3):
            if (mask >> k) & 1:
                a[k] = L - rng.uniform(0.0, 0.3)
                d[k] = abs(d[k]) + 0.2           # crosses the face
        d /= np.linalg.norm(d)
        r = r_in if q % 2 == 0 else r_out
        xs += [a, a + r * d]
        ts += [types[0], types[1]]
    x = wrap(np.array(xs), L)
    n = len(ts)
    return System(L=float(L), x=x, v=np.zeros((n, 3)), type=np.array(ts, dtype=np.int32),
                  reactive=np.ones(n, dtype=np.uint8), bonds=np.zeros((0, 4), dtype=np.int32))


def branched_clusters(m, spacing=6.0, seed=0, T=1.0) -> System:
    """m star-shaped clusters on a cubic lattice: a hub bonded to three arms, each
    arm bonded to two leaves (bond length about 1), with explicit angles (arm-hub-arm,
    hub-arm-leaf, leaf-arm-leaf; type 1) and dihedrals (leaf-arm-hub-arm; type 1).
    Hubs and arms each meet nine distinct beads through their bonded terms, leaves
    five.  Bonds are type 1 on both sides."""
    rng = np.random.default_rng(seed)
    k = int(math.ceil(m ** (1.0 / 3.0)))
    L = k * spacing
    xs, bonds, angles, dihedrals = [], [], [], []
    arm_dirs = np.array([[1.0, 0.0, 0.0], [-0.5, 0.866, 0.0], [-0.5, -0.866, 0.0]])
    for q in range(m):
        c = np.array([q % k, (q // k) % k, q // (k * k)], dtype=np.float64) * spacing + 0.5 * spacing
        R = _rotation(rng)
        base = len(xs)
        hub = base
        xs.append(c)
        arms, leaves = [], []
        for a in range(3):
            d = R @ arm_dirs[a]
            pa = c + d
            arms.append(len(xs))
            xs.append(pa)
        for a in range(3):
            d = R @ arm_dirs[a]
            side = R @ np.array([0.0, 0.0, 1.0])
            two = []
            for sgn in (1.0, -1.0):
                u = d + 0.9 * sgn * side
                u /= np.linalg.norm(u)
                two.append(len(xs))
                xs.append(xs[arms[a]] + u)
            leaves.append(two)
        for a in range(3):
            bonds.append((hub, arms[a], 1, 1))
            for lf in leaves[a]:
                bonds.append((arms[a], lf, 1, 1))
        for a in range(3):
            for b in range(a + 1, 3):
                angles.append((1, arms[a], hub, arms[b]))
            for lf in leaves[a]:
                angles.append((1, hub, arms[a], lf))
            angles.append((1, leaves[a][0], arms[a], leaves[a][1]))
        for a in range(3):
            for b in range(3):
                if a != b:
                    for lf in leaves[a]:
                        dihedrals.append((1, lf, arms[a], hub, arms[b]))
    x = wrap(np.array(xs) + rng.normal(0, 0.03, size=(len(xs), 3)), L)
    n = len(xs)
    return System(L=float(L), x=x, v=maxwell_boltzmann(rng, n, T), type=np.full(n, 1, dtype=np.int32),
                  reactive=np.zeros(n, dtype=np.uint8), bonds=np.array(bonds, dtype=np.int32),
                  angles=np.array(angles, dtype=np.int32), dihedrals=np.array(dihedrals, dtype=np.int32))


# ----------------------------------------------------------------------------------
# the paper's 1-bead model (Fig. 2), as a topology fixture
# ----------------------------------------------------------------------------------

def ladder_1bead(n_bp, seq=None, hyb_dist=0.6, bb_dist=0.6, hybridized=True) -> System:
    """Ideal double strand of the 1-bead model.

    Strand 1 (5'->3' along +x) beads at (k*bb, 0, 0); strand 2 antiparallel at
    (k*bb, hyb, 0).  Backbone bonds are directional: a bead stores 2 (3') towards
    its 3' neighbour and 3 (5') towards its 5' neighbour.  Hybridization bonds
    (type 1) join the beads at equal k."""
    if seq is None:
        seq = [(k % 4) + 1 for k in range(n_bp)]
    L = max(4.0 * n_bp * bb_dist + 10.0, 20.0)
    xs, ts, bonds = [], [], []
    for k in range(n_bp):
        xs.append([2.0 + k * bb_dist, 2.0, 2.0]); ts.append(seq[k])
    for k in range(n_bp):
        xs.append([2.0 + k * bb_dist, 2.0 + hyb_dist, 2.0]); ts.append(COMPLEMENT[seq[k]])
    for k in range(n_bp - 1):
        bonds.append((k, k + 1, BB_3P, BB_5P))                      # strand 1: k+1 is 3' of k
        bonds.append((n_bp + k, n_bp + k + 1, BB_5P, BB_3P))        # strand 2: k is 3' of k+1
    if hybridized:
        for k in range(n_bp):
            bonds.append((k, n_bp + k, H_BOND, H_BOND))
    x = np.array(xs, dtype=np.float64)
    n = x.shape[0]
    return System(L=L, x=x, v=np.zeros((n, 3)), type=np.array(ts, dtype=np.int32),
                  reactive=np.ones(n, dtype=np.uint8), bonds=np.array(bonds, dtype=np.int32).reshape(-1, 4))


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5}
