"""Pins of the oracle's pattern-driven angle/dihedral generation against closed-form
counts derived by hand from the pattern semantics of section 2 (golden fixtures
under tests/golden/), and against an independent brute-force enumeration."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fig2_rules():
    with open(os.path.join(GOLDEN, "fig2_rules.txt")) as f:
        return synth.parse_script(f.read())


def test_golden_files_present():
    with open(os.path.join(GOLDEN, "ladder_counts.json")) as f:
        d = json.load(f)
    assert "fig2_1bead" in d and "t2_2bead_duplex" in d


def test_fig2_script_parses_as_printed():
    rs = fig2_rules()
    assert rs.every == 1 and rs.paircheck13 == 0 and rs.paircheck14 == 1
    kinds = [r[0] for r in rs.rules]
    assert kinds == ["create", "create", "createdir", "kill", "maxbond", "maxbond", "maxbond",
                     "angle", "angle", "dihedral", "dihedral", "dihedral", "dihedral"]
    assert rs.rules[2] == ("createdir", 2, 3, 2, 3, 0.3, 0.1)
    assert rs.rules[8] == ("angle", 2, (0, 0, 0), (synth.mask(1), synth.mask(2, 3)))


@pytest.mark.parametrize("n", [2, 3, 4, 7, 10])
def test_fig2_ladder_closed_form_counts(n):
    lad = synth.ladder_1bead(n)
    o = oracle.Oracle.from_system(lad, synth.ForceField(), fig2_rules(), seed=1)
    a = o.angles()
    d = o.dihedrals()
    ca = np.bincount(a[:, 0], minlength=3) if len(a) else np.zeros(3, int)
    cd = np.bincount(d[:, 0], minlength=4) if len(d) else np.zeros(4, int)
    assert ca[1] == max(0, 2 * n - 4)
    assert ca[2] == 4 * n - 4
    assert cd[1] == 2 * n - 2
    assert cd[2] == 2 * n - 2
    assert cd[3] == max(0, 2 * n - 4)


def test_fig2_unhybridized_strands_have_only_backbone_angles():
    n = 6
    lad = synth.ladder_1bead(n, hybridized=False)
    o = oracle.Oracle.from_system(lad, synth.ForceField(), fig2_rules(), seed=1)
    a = o.angles()
    assert len(o.dihedrals()) == 0
    assert set(a[:, 0].tolist()) == {1} and len(a) == 2 * (n - 2)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_t2_duplex_closed_form_counts(n):
    s = synth.small_duplexes(n_duplex=1, n_bp=n, rho=0.005)
    o = oracle.Oracle.from_system(s, synth.ff_t2(), synth.rules_t2(), seed=1)
    nb, na, nd = o.counts()
    assert nb == 2 * (n - 1) + 2 * n + n
    assert na == 2 * max(0, n - 2) + 2 * n
    assert nd == 2 * (n - 1)


@pytest.mark.parametrize("n", [2, 3, 10])
def test_t2_single_strand_counts(n):
    s = synth.single_strands(1, n, L=30.0)
    o = oracle.Oracle.from_system(s, synth.ff_t2(), synth.rules_t2(), seed=1)
    _, na, nd = o.counts()
    assert na == max(0, n - 2)
    assert nd == n - 1


def test_lists_are_canonical_and_unique():
    lad = synth.ladder_1bead(9)
    o = oracle.Oracle.from_system(lad, synth.ForceField(), fig2_rules(), seed=1)
    a = o.angles()
    d = o.dihedrals()
    assert np.all(a[:, 1] < a[:, 3])
    assert np.all(d[:, 1] < d[:, 4])
    assert len({tuple(r[1:]) for r in a.tolist()}) == len(a)
    assert len({tuple(r[1:]) for r in d.tolist()}) == len(d)


# ---------------------------------------------------------------------------------
# independent brute force: all ordered tuples of distinct beads, path test through
# the bond set, pattern predicates written out from section 2

def _brute(system, rs):
    n = system.n
    stored = {}
    for i, j, tij, tji in system.bonds.tolist():
        stored[(i, j)] = tij
        stored[(j, i)] = tji
    typ = system.type.tolist()

    def bead_ok(r, t):
        return r == 0 or r == t

    def inm(m, t):
        return t is not None and (m >> t) & 1

    angs = set()
    arules = [r for r in rs.rules if r[0] == "angle"]
    drules = [r for r in rs.rules if r[0] == "dihedral"]
    for a, b, c in itertools.permutations(range(n), 3):
        if (a, b) not in stored or (b, c) not in stored or a > c:
            continue
        for _, t, bt, m in arules:
            fwd = all(bead_ok(bt[k], typ[v]) for k, v in enumerate((a, b, c))) and inm(m[0], stored[(b, a)]) \
                and inm(m[1], stored[(b, c)])
            rev = all(bead_ok(bt[k], typ[v]) for k, v in enumerate((c, b, a))) and inm(m[0], stored[(b, c)]) \
                and inm(m[1], stored[(b, a)])
            if fwd or rev:
                angs.add((t, a, b, c))
                break
    dihs = set()
    for a, b, c, d in itertools.permutations(range(n), 4):
        if (a, b) not in stored or (b, c) not in stored or (c, d) not in stored or a > d:
            continue
        for _, t, bt, m in drules:
            fwd = all(bead_ok(bt[k], typ[v]) for k, v in enumerate((a, b, c, d))) and inm(m[0], stored[(b, a)]) \
                and (inm(m[1], stored[(c, b)]) or inm(m[1], stored[(b, c)])) and inm(m[2], stored[(c, d)])
            rev = all(bead_ok(bt[k], typ[v]) for k, v in enumerate((d, c, b, a))) and inm(m[0], stored[(c, d)]) \
                and (inm(m[1], stored[(b, c)]) or inm(m[1], stored[(c, b)])) and inm(m[2], stored[(b, a)])
            if fwd or rev:
                dihs.add((t, a, b, c, d))
                break
    return angs, dihs


def _random_graph(n, nb, seed, n_types=5, n_btypes=4):
    rng = np.random.default_rng(seed)
    bonds = set()
    deg = np.zeros(n, int)
    while len(bonds) < nb:
        i, j = sorted(rng.choice(n, 2, replace=False).tolist())
        if (i, j) in bonds or deg[i] >= 4 or deg[j] >= 4:
            continue
        bonds.add((i, j))
        deg[i] += 1
        deg[j] += 1
    b = np.array([(i, j, int(rng.integers(1, n_btypes + 1)), int(rng.integers(1, n_btypes + 1)))
                  for i, j in sorted(bonds)], dtype=np.int32)
    s = synth.random_gas(n, 10.0, seed=seed, n_types=n_types)
    s.bonds = b
    return s


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_generation_equals_brute_force_random_graph(seed):
    s = _random_graph(16, 20, seed)
    rs = synth.RuleSet(rules=[
        ("angle", 1, (0, 0, 0), (synth.mask(1, 2), synth.mask(3))),
        ("angle", 2, (1, 0, 2), (synth.ALL_TYPES, synth.mask(2))),
        ("angle", 3, (0, 3, 0), (synth.mask(4), synth.ALL_TYPES)),
        ("dihedral", 1, (0, 0, 0, 0), (synth.mask(1), synth.mask(2), synth.mask(3, 4))),
        ("dihedral", 2, (2, 0, 0, 1), (synth.ALL_TYPES, synth.mask(1, 4), synth.ALL_TYPES)),
        ("dihedral", 3, (0, 5, 0, 0), (synth.mask(2), synth.ALL_TYPES, synth.mask(2))),
    ])
    o = oracle.Oracle.from_system(s, synth.ForceField(), rs, seed=1)
    ang, dih = _brute(s, rs)
    got_a = {tuple(r) for r in o.angles().tolist()}
    got_d = {tuple(r) for r in o.dihedrals().tolist()}
    assert got_a == ang
    assert got_d == dih
    assert len(ang) > 3 and len(dih) > 3


def test_fig2_generation_equals_brute_force():
    lad = synth.ladder_1bead(5)
    rs = fig2_rules()
    o = oracle.Oracle.from_system(lad, synth.ForceField(), rs, seed=1)
    ang, dih = _brute(lad, rs)
    assert {tuple(r) for r in o.angles().tolist()} == ang
    assert {tuple(r) for r in o.dihedrals().tolist()} == dih


def test_graph_distance_on_a_chain():
    s = _random_graph(8, 0, 1)
    s.bonds = np.array([(k, k + 1, 1, 1) for k in range(7)], dtype=np.int32)
    o = oracle.Oracle.from_system(s, None, None)
    for j in range(8):
        assert o.graph_distance(0, j) == min(j, 4)
