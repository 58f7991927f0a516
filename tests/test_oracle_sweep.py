"""Pins of the oracle's dynamic-bonding sweep against the behaviour the paper states
(section 2 and the appendix): formation frequencies equal to the stated
probability, at most one new and one broken bond per bead per sweep, maximal
functionality never exceeded, closest-partner / most-distant-partner matching,
breakbond versus killbond, rule shadowing, no re-matching of rejected partners,
removal of angles/dihedrals crossing broken bonds and the invariant that the
angle/dihedral lists always equal the full enumeration of the current graph."""
import math

import numpy as np
import pytest

import oracle
import synth


def _sys(positions, types, bonds=(), L=30.0):
    x = np.array(positions, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    return synth.System(L=L, x=synth.wrap(x, L), v=np.zeros((n, 3)), type=np.array(types, dtype=np.int32),
                        reactive=np.ones(n, dtype=np.uint8), bonds=np.array(bonds, dtype=np.int32).reshape(-1, 4))


def _bond_set(o):
    return {tuple(r) for r in o.bonds().tolist()}


@pytest.mark.parametrize("p", [0.1, 0.5, 0.9])
def test_formation_frequency_matches_probability(p):
    m = 3000
    s = synth.isolated_pairs(m, 1.0, seed=int(p * 100))
    rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, p), ("maxbond", 1, 0, 1)])
    o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=12345)
    o.sweep_now()
    k = o.counts()[0]
    sd = math.sqrt(m * p * (1 - p))
    assert abs(k - m * p) < 5 * sd
    assert o.stats()[0]["bonds_created"] == k


def _average_law(p):
    """P[(u1 + u2)/2 < p] for independent uniforms: the triangular distribution of their mean"""
    return 2 * p * p if p <= 0.5 else 1 - 2 * (1 - p) ** 2


@pytest.mark.parametrize("p", [0.1, 0.3, 0.5, 0.9])
def test_averaged_acceptance_frequency_creation(p):
    """The appendix's literal acceptance (each bead draws a uniform, the pair takes
    their mean): the created fraction follows 2p^2 / 1 - 2(1-p)^2, not p."""
    m = 4000
    s = synth.isolated_pairs(m, 1.0, seed=int(p * 100) + 7)
    rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, p), ("maxbond", 1, 0, 1)], accept="average")
    o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=2024)
    o.sweep_now()
    k = o.counts()[0]
    q = _average_law(p)
    assert abs(k - m * q) < 5 * math.sqrt(m * q * (1 - q))
    if p != 0.5:   # distinguishable from the one-uniform-per-pair law
        assert abs(k - m * p) > 5 * math.sqrt(m * p * (1 - p))


@pytest.mark.parametrize("p", [0.2, 0.8])
def test_averaged_acceptance_frequency_breakage(p):
    m = 4000
    s = synth.isolated_pairs(m, 1.3, seed=int(p * 100) + 9)
    s.bonds = np.array([(2 * k, 2 * k + 1, 1, 1) for k in range(m)], dtype=np.int32)
    for accept, q in [("average", _average_law(p)), ("pair", p)]:
        rs = synth.RuleSet(every=1, rules=[("break", 1, 1.2, p)], accept=accept)
        o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=99)
        o.sweep_now()
        k = m - o.counts()[0]
        assert o.stats()[0]["bonds_broken"] == k
        assert abs(k - m * q) < 5 * math.sqrt(m * q * (1 - q))


def test_averaged_acceptance_edge_probabilities():
    s = synth.isolated_pairs(300, 1.0, seed=5)
    for p, exp in [(1.0, 300), (0.0, 0)]:
        rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, p)], accept="average")
        o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=1)
        o.sweep_now()
        assert o.counts()[0] == exp


def test_large_box_pairs_at_the_creation_distance():
    """The strict FP64 cutoff decision in a box of edge 4000 (pairs straddling faces,
    edges and a corner, 1e-7 inside or outside the creation distance): exactly the
    inside pairs bond, as a brute-force distance check says."""
    L, r = 4000.0, 1.5
    s = synth.boundary_pairs(1000, r * (1 - 1e-7), r * (1 + 1e-7), L, seed=3)
    rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, r, 1.0), ("maxbond", 1, 0, 1)])
    o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=1)
    o.sweep_now()
    d = s.x[1::2] - s.x[0::2]
    d -= L * np.round(d / L)
    inside = np.flatnonzero(np.sum(d * d, axis=1) < r * r)
    assert len(inside) == 500
    assert _bond_set(o) == {(2 * k, 2 * k + 1, 1, 1) for k in inside.tolist()}


def test_unit_probability_creates_every_pair_and_zero_none():
    s = synth.isolated_pairs(200, 1.2, seed=3)
    for p, exp in [(1.0, 200), (0.0, 0)]:
        o = oracle.Oracle.from_system(s, synth.ForceField(),
                                      synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, p)]), seed=1)
        o.sweep_now()
        assert o.counts()[0] == exp


def test_cutoff_is_strict():
    s = _sys([[5, 5, 5], [6.5, 5, 5]], [1, 2])
    o = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0)]))
    o.sweep_now()
    assert o.counts()[0] == 0
    o2 = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5000001, 1.0)]))
    o2.sweep_now()
    assert o2.counts()[0] == 1


def _eligible_partners_bruteforce(s, bonds, i, rmax, comp):
    """Independent eligibility for a single symmetric rule set: complementary types,
    r < rmax, graph distance > 3 (no paircheck), no existing bond of type 1."""
    adj = {k: set() for k in range(s.n)}
    hcount = np.zeros(s.n, int)
    for a, b, ta, tb in bonds:
        adj[a].add(b); adj[b].add(a)
        hcount[a] += ta == 1
        hcount[b] += tb == 1
    # beads within 3 hops of i
    near = {i}
    frontier = {i}
    for _ in range(3):
        frontier = {w for u in frontier for w in adj[u]} - near
        near |= frontier
    out = []
    for j in range(s.n):
        if j in near or comp.get(int(s.type[i])) != int(s.type[j]) or hcount[i] >= 1 or hcount[j] >= 1:
            continue
        d = s.x[j] - s.x[i]
        d = np.where(d > s.L / 2, d - s.L, np.where(d < -s.L / 2, d + s.L, d))
        r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        if r2 < rmax * rmax:
            out.append((r2, j))
    return sorted(out)


def test_matching_closest_partner_and_one_bond_per_bead():
    rng = np.random.default_rng(5)
    n = 400
    L = 9.0
    s = synth.random_gas(n, L, seed=5, n_types=4)
    # a few pre-existing hybridization bonds so maxbond and graph exclusion matter
    bonds = [(2 * k, 2 * k + 1, 1, 1) for k in range(0, 40)]
    s.bonds = np.array(bonds, dtype=np.int32)
    rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0), ("create", 1, 3, 4, 1.5, 1.0),
                                       ("maxbond", 1, 0, 1)])
    o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=2)
    before = _bond_set(o)
    o.sweep_now()
    after = _bond_set(o)
    new = after - before
    nomC, _ = o.nominations()
    comp = {1: 2, 2: 1, 3: 4, 4: 3}
    per_bead = np.zeros(n, int)
    for i, j, ti, tj in new:
        per_bead[i] += 1; per_bead[j] += 1
        assert nomC[i] == j and nomC[j] == i
        for a in (i, j):
            el = _eligible_partners_bruteforce(s, bonds, a, 1.5, comp)
            assert el[0][1] == (j if a == i else i)
    assert per_bead.max() <= 1
    assert len(new) > 10
    # every nomination is the closest eligible candidate (ties -> lower id)
    for i in range(n):
        el = _eligible_partners_bruteforce(s, bonds, i, 1.5, comp)
        assert nomC[i] == (el[0][1] if el else -1)
    # maxbond: nobody holds two hybridization bonds
    cnt = np.zeros(n, int)
    for i, j, ti, tj in after:
        cnt[i] += ti == 1; cnt[j] += tj == 1
    assert cnt.max() <= 1
    _ = rng


def test_breakbond_takes_one_killbond_takes_all():
    # bead 0 (type 1) holds two long type-1 bonds
    pos = [[10, 10, 10], [12.5, 10, 10], [10, 12.6, 10]]
    s = _sys(pos, [1, 2, 2], [(0, 1, 1, 1), (0, 2, 1, 1)])
    ob = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("break", 1, 2.0, 1.0)]))
    ob.sweep_now()
    assert _bond_set(ob) == {(0, 1, 1, 1)}        # only the most distant partner (bead 2) went
    assert ob.stats()[0]["bonds_broken"] == 1
    ok = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("kill", 1, 2.0)]))
    ok.sweep_now()
    assert _bond_set(ok) == set()
    assert ok.stats()[0]["bonds_killed"] == 2


def test_break_is_strictly_longer_and_symmetric_only():
    pos = [[10, 10, 10], [12.0, 10, 10], [10, 13, 10], [13, 13, 10]]
    s = _sys(pos, [1, 2, 1, 2], [(0, 1, 1, 1), (2, 3, 2, 3)])
    o = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("kill", 1, 2.0), ("kill", 2, 2.0)]))
    o.sweep_now()
    # r = 2.0 is not longer than 2.0; the directional 2/3 bond is not symmetric
    assert _bond_set(o) == {(0, 1, 1, 1), (2, 3, 2, 3)}


def test_last_matching_rule_shadows():
    s = synth.isolated_pairs(50, 1.0, seed=4)
    rs1 = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0), ("create", 2, 1, 2, 1.5, 0.0)])
    o = oracle.Oracle.from_system(s, None, rs1, seed=1)
    o.sweep_now()
    assert o.counts()[0] == 0                         # later p=0 rule shadows the earlier p=1 rule
    rs2 = synth.RuleSet(every=1, rules=[("create", 2, 1, 2, 1.5, 0.0), ("create", 1, 1, 2, 1.5, 1.0)])
    o = oracle.Oracle.from_system(s, None, rs2, seed=1)
    o.sweep_now()
    b = o.bonds()
    assert len(b) == 50 and set(b[:, 2].tolist()) == {1}
    # a later rule that does not reach (shorter distance) does not shadow
    rs3 = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0), ("create", 2, 1, 2, 0.5, 0.0)])
    o = oracle.Oracle.from_system(s, None, rs3, seed=1)
    o.sweep_now()
    assert o.counts()[0] == 50


def test_no_rematching_of_rejected_partners():
    # A0 -- T1 -- A2 on a line; T1's closest A is A2, so A0 stays single this sweep
    s = _sys([[10, 10, 10], [11.0, 10, 10], [11.8, 10, 10]], [1, 2, 1])
    o = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0),
                                                                         ("maxbond", 1, 0, 1)]))
    o.sweep_now()
    assert _bond_set(o) == {(1, 2, 1, 1)}
    nomC, _ = o.nominations()
    assert nomC.tolist() == [1, 2, 1]


def test_maxbond_bead_type_specific():
    # maxbond applies to bead type 1 only: the type-2 bead may take two bonds
    s = _sys([[10, 10, 10], [11, 10, 10], [12, 10, 10], [20, 20, 20]], [1, 2, 1, 2], [(0, 1, 1, 1)])
    rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0), ("maxbond", 1, 1, 1)])
    o = oracle.Oracle.from_system(s, None, rs)
    o.sweep_now()
    assert _bond_set(o) == {(0, 1, 1, 1), (1, 2, 1, 1)}
    rs = synth.RuleSet(every=1, rules=[("create", 1, 1, 2, 1.5, 1.0), ("maxbond", 1, 0, 1)])
    o = oracle.Oracle.from_system(s, None, rs)
    o.sweep_now()
    assert _bond_set(o) == {(0, 1, 1, 1)}


def test_createdir_types_follow_bead_roles():
    # type-3 bead id 0, type-2 bead id 1: bead1 of the rule is type 2 -> it stores bt1 = 2
    s = _sys([[10, 10, 10], [10.2, 10, 10]], [3, 2])
    o = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("createdir", 2, 3, 2, 3, 0.3, 1.0)]))
    o.sweep_now()
    assert _bond_set(o) == {(0, 1, 3, 2)}
    # equal bead types: the lower id plays bead1
    s = _sys([[10, 10, 10], [10.2, 10, 10]], [2, 2])
    o = oracle.Oracle.from_system(s, None, synth.RuleSet(every=1, rules=[("createdir", 2, 3, 2, 2, 0.3, 1.0)]))
    o.sweep_now()
    assert _bond_set(o) == {(0, 1, 2, 3)}


def test_paircheck_switches():
    # chain 0-1-2-3 of type-5 linkers with reactive ends of types 1 and 2
    pos = [[10, 10, 10], [10.5, 10.5, 10], [11.0, 10.5, 10], [10.6, 10.0, 10]]
    bonds = [(0, 1, 4, 4), (1, 2, 4, 4), (2, 3, 4, 4)]
    s = _sys(pos, [1, 5, 5, 2], bonds)
    for pc14, expect in [(0, 0), (1, 1)]:
        rs = synth.RuleSet(every=1, paircheck14=pc14, rules=[("create", 1, 1, 2, 1.5, 1.0)])
        o = oracle.Oracle.from_system(s, None, rs)
        o.sweep_now()
        assert o.stats()[0]["bonds_created"] == expect
    s3 = _sys(pos[:3], [1, 5, 2], bonds[:2])   # 1-3 pair
    for pc13, expect in [(0, 0), (1, 1)]:
        rs = synth.RuleSet(every=1, paircheck13=pc13, rules=[("create", 1, 1, 2, 1.5, 1.0)])
        o = oracle.Oracle.from_system(s3, None, rs)
        o.sweep_now()
        assert o.stats()[0]["bonds_created"] == expect


def test_kill_purges_rung_angles():
    s = synth.small_duplexes(n_duplex=1, n_bp=5, rho=0.005)
    o = oracle.Oracle.from_system(s, synth.ff_t2(), synth.rules_t2(), seed=1)
    _, na0, nd0 = o.counts()
    # pull the middle base pair apart beyond the kill distance
    h = [b for b in s.bonds.tolist() if b[2] == 1][2]
    x = s.x.copy()
    d = x[h[1]] - x[h[0]]
    x[h[1]] += 2.0 * d / np.linalg.norm(d)
    o.set_state(synth.wrap(x, s.L), s.v, s.type)
    o.sweep_now()
    last = o.stats()[0]
    assert last["bonds_killed"] == 1
    assert last["angles_removed"] == 2          # the two rung angles through that hybridization bond
    assert last["dihedrals_removed"] == 0       # stacking dihedrals do not cross hybridization bonds
    assert o.counts()[1] == na0 - 2


def test_conversion_changes_type_and_regenerates():
    s = synth.small_duplexes(n_duplex=1, n_bp=4, rho=0.005)
    rs = synth.RuleSet(every=1, rules=[("convert", 1, 5, 1.0, 1.0), ("maxbond", 5, 0, 1),
                                       ("angle", 1, (5, 0, 0), (synth.mask(4), synth.mask(1))),
                                       ("angle", 2, (5, 0, 0), (synth.mask(4), synth.mask(5)))])
    o = oracle.Oracle.from_system(s, synth.ff_t2(weak=True), rs, seed=1)
    assert np.bincount(o.angles()[:, 0]).tolist() == [0, 8]
    o.sweep_now()
    st = o.stats()[0]
    assert st["bonds_converted"] == 4              # every 1.2-long hybridization bond exceeds 1.0
    assert set(o.bonds()[:, 2:].ravel().tolist()) == {2, 3, 4, 5}
    a = o.angles()
    assert np.bincount(a[:, 0]).tolist() == [0, 0, 8]   # rung angles removed and re-created as type 2
    assert st["angles_removed"] == 8 and st["angles_created"] == 8


def test_conversion_blocks_creation_of_its_beads():
    # beads 0(A)-1(T) hold a long hybridization bond being converted; bead 2 (T) near bead 0
    s = _sys([[10, 10, 10], [11.5, 10, 10], [9.0, 10, 10], [30, 30, 30]], [1, 2, 2, 1], [(0, 1, 1, 1)], L=40)
    rs = synth.RuleSet(every=1, rules=[("create", 6, 1, 2, 1.5, 1.0), ("convert", 1, 5, 1.0, 1.0)])
    o = oracle.Oracle.from_system(s, None, rs)
    o.sweep_now()
    assert _bond_set(o) == {(0, 1, 5, 5)}


def _full_enumeration(o, s, rules):
    b = o.bonds()
    x, v = o.state()
    ref = synth.System(L=s.L, x=x, v=v, type=s.type, reactive=s.reactive, bonds=b)
    r = oracle.Oracle.from_system(ref, None, rules)
    return {tuple(t) for t in r.angles().tolist()}, {tuple(t) for t in r.dihedrals().tolist()}


def test_lists_equal_full_enumeration_through_a_dynamic_run():
    # complementary single strands in a small box, frequent creation and a short kill distance
    s = synth.single_strands(24, 6, L=11.0, seed_w=3, seed_d=4)
    rules = synth.rules_t2(p=0.7, every=2, r_create=1.5, r_kill=1.35)
    ff = synth.ff_t2(T0=1.0, T1=1.0, gamma=1.0, dt=0.005)
    o = oracle.Oracle.from_system(s, ff, rules, seed=9)
    created = removed = 0
    for _ in range(60):
        o.step(10)
        last, cum, _ = o.stats()
        a, d = _full_enumeration(o, s, rules)
        assert {tuple(t) for t in o.angles().tolist()} == a
        assert {tuple(t) for t in o.dihedrals().tolist()} == d
    last, cum, sweeps = o.stats()
    assert sweeps == 300
    assert cum["bonds_created"] > 5 and cum["bonds_killed"] > 2
    assert cum["angles_created"] > 0 and cum["angles_removed"] > 0
    _ = created, removed


def fig2_dynamic_setup(n_strand=30, n_nt=5, L=6.0, seed=3):
    """1-bead strands (Fig. 2 rule table) in a small box without pair repulsion,
    so complementary beads meet within the 0.6 reaction distance."""
    import os
    rng = np.random.default_rng(seed)
    xs, ts, bonds = [], [], []
    for s_ in range(n_strand):
        o = rng.uniform(0, L, size=3)
        u = rng.normal(size=3); u /= np.linalg.norm(u)
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
    here = os.path.dirname(__file__)
    with open(os.path.join(here, "golden", "fig2_rules.txt")) as f:
        rules = synth.parse_script(f.read())
    ff = synth.ForceField(eps=0.0, gamma=1.0, dt=0.005)
    ff.bonds = {1: (5.0, 0.6), 2: (20.0, 0.5), 3: (20.0, 0.5)}
    ff.angles = {1: (1.0, math.pi), 2: (1.0, 0.5 * math.pi)}
    ff.dihedrals = {1: (1.0, 0.0), 2: (1.0, 0.0), 3: (1.0, math.pi)}
    return sysm, ff, rules


def test_fig2_dynamic_run_keeps_lists_consistent():
    s, ff, rules = fig2_dynamic_setup()
    o = oracle.Oracle.from_system(s, ff, rules, seed=21)
    for _ in range(30):
        o.step(10)
        a, d = _full_enumeration(o, s, rules)
        assert {tuple(t) for t in o.angles().tolist()} == a
        assert {tuple(t) for t in o.dihedrals().tolist()} == d
        b = o.bonds()
        # functionality: at most one bond of each of the types 1, 2, 3 per bead
        for col_t in (1, 2, 3):
            cnt = np.bincount(np.concatenate([b[b[:, 2] == col_t, 0], b[b[:, 3] == col_t, 1]]), minlength=s.n)
            assert cnt.max() <= 1
    _, cum, _ = o.stats()
    assert cum["bonds_created"] > 10 and cum["bonds_killed"] > 5
    assert cum["dihedrals_created"] > 0 and cum["dihedrals_removed"] > 0
