"""Pins of the oracle's per-vertex graphlet orbit counts (orbits 4..14 of the
connected 4-vertex graphs; column o - 4 of an (n, 11) array) against facts
fixed outside the oracle: per-vertex closed forms of named graph families,
derived here from the induced-occurrence definition; the two enumerations
(all subsets, ESU) against each other; the orbit sums against the six global
counts of the pinned oracle tiers (each pattern's vertices split over its
orbits: a path has 2 ends and 2 middles, a claw 3 leaves and 1 centre, a
paw 1 tail, 2 degree-2 and 1 degree-3 vertex, a diamond 2 + 2); and
relabelling and disjoint-union invariance."""
from math import comb

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs as G

O = {o: o - 4 for o in range(4, 15)}


def table(n, rows):
    """(n, 11) array from {vertex or vertex list: {orbit: count}}."""
    a = np.zeros((n, 11), dtype=np.uint64)
    for vs, orb in rows:
        for v in (vs if isinstance(vs, (list, range)) else [vs]):
            for o, c in orb.items():
                a[v, O[o]] = c
    return a


def cf_complete(n):
    # every 3 other vertices close a 4-clique with v
    return table(n, [(range(n), {14: comb(n - 1, 3)})])


def cf_star(k):
    # the hub is the centre of every claw, a leaf is in C(k-1, 2) of them
    return table(k + 1, [(0, {7: comb(k, 3)}), (list(range(1, k + 1)), {6: comb(k - 1, 2)})])


def cf_path(n):
    # the induced 4-paths are the windows of 4 consecutive vertices
    rows = []
    for v in range(n):
        ends = int(v + 3 < n) + int(v >= 3)
        mids = int(v >= 1 and v + 2 < n) + int(v >= 2 and v + 1 < n)
        rows.append((v, {4: ends, 5: mids}))
    return table(n, rows)


def cf_cycle(n):
    # C_4 is one cycle; for n >= 5 every vertex ends 2 windows and is in the
    # middle of 2
    if n == 4:
        return table(4, [(range(4), {8: 1})])
    return table(n, [(range(n), {4: 2, 5: 2})])


def cf_bipartite(a, b):
    # side A vertex: centre of claws on 3 of the b others, leaf of claws
    # centred in B with 2 more leaves from A, in a cycle with one more A
    # vertex and 2 of B
    return table(a + b, [(list(range(a)), {7: comb(b, 3), 6: b * comb(a - 1, 2), 8: (a - 1) * comb(b, 2)}),
                         (list(range(a, a + b)), {7: comb(a, 3), 6: a * comb(b - 1, 2),
                                                  8: (b - 1) * comb(a, 2)})])


def cf_wheel(k):
    # hub 0, rim 1..k (k >= 5).  Rim-only 4-sets are the k windows of the rim
    # cycle (2 ends, 2 middles per rim vertex).  Hub + 3 consecutive rim
    # vertices: diamond with the hub and the middle one of degree 3.  Hub +
    # an adjacent rim pair + a rim vertex next to neither: paw, hub of
    # degree 3, the pair of degree 2, the third the tail (k - 4 pairs avoid
    # a rim vertex and its neighbours).  Hub + 3 pairwise non-adjacent rim
    # vertices: claw centred at the hub; a rim vertex has (k-4)(k-5)/2 pairs
    # of non-adjacent partners among the k - 3 rim vertices not next to it.
    hub = {7: k * (k - 4) * (k - 5) // 6, 11: k * (k - 4), 13: k}
    rim = {4: 2, 5: 2, 12: 2, 13: 1, 10: 2 * (k - 4), 9: k - 4, 6: (k - 4) * (k - 5) // 2}
    return table(k + 1, [(0, hub), (list(range(1, k + 1)), rim)])


CLOSED = [
    ("K4", lambda: G.complete(4), lambda: cf_complete(4)),
    ("K9", lambda: G.complete(9), lambda: cf_complete(9)),
    ("K1,7", lambda: G.star(7), lambda: cf_star(7)),
    ("P4", lambda: G.path(4), lambda: cf_path(4)),
    ("P10", lambda: G.path(10), lambda: cf_path(10)),
    ("C4", lambda: G.cycle(4), lambda: cf_cycle(4)),
    ("C11", lambda: G.cycle(11), lambda: cf_cycle(11)),
    ("K3,5", lambda: G.complete_bipartite(3, 5), lambda: cf_bipartite(3, 5)),
    ("W5", lambda: G.wheel(5), lambda: cf_wheel(5)),
    ("W9", lambda: G.wheel(9), lambda: cf_wheel(9)),
    # one copy of each pattern on its own: the orbit of each vertex by hand
    ("paw", lambda: G.csr(4, [(0, 1), (1, 2), (0, 2), (0, 3)]),
     lambda: table(4, [(0, {11: 1}), ([1, 2], {10: 1}), (3, {9: 1})])),
    ("diamond", lambda: G.csr(4, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3)]),
     lambda: table(4, [([0, 1], {13: 1}), ([2, 3], {12: 1})])),
    # K_{2,2,2}: 3 cycles and 12 diamonds over 6 equivalent vertices
    ("octahedron", G.octahedron, lambda: table(6, [(range(6), {8: 2, 12: 4, 13: 4})])),
    # Petersen: each vertex the centre of its own claw and a leaf of its 3
    # neighbours'; 60 paths over 10 equivalent vertices
    ("petersen", G.petersen, lambda: table(10, [(range(10), {7: 1, 6: 3, 4: 12, 5: 12})])),
    ("empty6", lambda: G.csr(6, []), lambda: table(6, [])),
]


@pytest.mark.parametrize("name,make,expected", CLOSED, ids=[c[0] for c in CLOSED])
def test_orbit_closed_forms(name, make, expected):
    g = make()
    want = expected()
    assert (oracle.orbits_brute(*g) == want).all(), name
    assert (oracle.orbits_esu(*g) == want).all(), name


def orbit_sums_to_counts(orb):
    """The six global counts from per-vertex orbit totals."""
    s = [int(x) for x in orb.sum(axis=0)]
    c = {o: s[o - 4] for o in range(4, 15)}
    return (c[7], c[5] // 2, c[11], c[8] // 4, c[13] // 2, c[14] // 4), c


RANDOM = [
    ("gnm", lambda: gg.gnm(70, 400, 3)),
    ("ba", lambda: gg.ba(80, 4, 2)),
    ("rmat", lambda: gg.rmat(6, 6, 0.57, 0.19, 0.19, 1)),
    ("planted", lambda: G.planted_cliques(60, 200, [6, 7], 4)),
    ("dense", lambda: G.gnp(30, 0.5, 9)),
]


@pytest.mark.parametrize("name,make", RANDOM, ids=[r[0] for r in RANDOM])
def test_enumerations_agree_and_sum_to_global_counts(name, make):
    g = make()
    a, b = oracle.orbits_brute(*g), oracle.orbits_esu(*g)
    assert (a == b).all()
    glob, c = orbit_sums_to_counts(a)
    assert glob == oracle.brute(*g) == oracle.closure(*g)
    # the fixed ratios inside each pattern
    assert c[4] == c[5] and c[6] == 3 * c[7] and c[10] == 2 * c[9] == 2 * c[11]
    assert c[12] == c[13] and c[8] % 4 == 0 and c[14] % 4 == 0


def test_er_workload_orbits_sum_to_counts():
    # the 2000-vertex ER workload: ESU orbits against the stored counts
    import json
    import os
    g = gg.gnm(2000, 20000, 1)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "er_2000_20000.json")))
    glob, _ = orbit_sums_to_counts(oracle.orbits_esu(*g))
    assert list(glob) == gold["counts"]


def test_relabel_and_union_invariance():
    g = gg.gnm(50, 220, 5)
    h = G.wheel(8)
    a = oracle.orbits_esu(*g)
    perm = np.random.default_rng(2).permutation(50)
    # vertex v of g is vertex perm[v] of the relabelled graph
    r = oracle.orbits_esu(*G.relabel(g, perm))
    assert (r[perm] == a).all()
    u = oracle.orbits_esu(*G.disjoint_union(g, h))
    assert (u[:50] == a).all() and (u[50:] == oracle.orbits_esu(*h)).all()


# ---------------------------------------------------------------- mutants
# plausible mistakes in the orbit assignment, each planted in a copy of the
# oracle source: the closed forms above must catch every one
ORBIT_MUTANTS = [
    ("case PATH: return d == 1 ? 4 : 5;", "case PATH: return d == 1 ? 5 : 4;"),
    ("case STAR: return d == 1 ? 6 : 7;", "case STAR: return d == 1 ? 7 : 6;"),
    ("case PAW: return d == 1 ? 9 : (d == 2 ? 10 : 11);", "case PAW: return d == 1 ? 10 : (d == 2 ? 9 : 11);"),
    ("case PAW: return d == 1 ? 9 : (d == 2 ? 10 : 11);", "case PAW: return d == 1 ? 9 : (d == 2 ? 11 : 10);"),
    ("case DIAMOND: return d == 2 ? 12 : 13;", "case DIAMOND: return d == 2 ? 13 : 12;"),
    ("for (int j = i + 1; j < 4; j++)\n      if (adjacent(rp, col, s[i], s[j])) { deg[i]++; deg[j]++; }\n  int c = classify",
     "for (int j = i + 1; j < 4; j++)\n      if (adjacent(rp, col, s[i], s[j])) { deg[i]++; }\n  int c = classify"),
    ("for (int i = 0; i < 4; i++) orb[(int64_t)s[i] * 11 + orbit_of(c, deg[i]) - 4]++;",
     "for (int i = 0; i < 3; i++) orb[(int64_t)s[i] * 11 + orbit_of(c, deg[i]) - 4]++;"),
]


@pytest.mark.parametrize("i", range(len(ORBIT_MUTANTS)))
def test_orbit_mutant_is_caught(tmp_path, i):
    import ctypes
    import os
    import subprocess
    old, new = ORBIT_MUTANTS[i]
    src_path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "oracle", "m4ref.c")
    src = open(src_path).read()
    assert src.count(old) == 1, old
    path = tmp_path / f"omut{i}.c"
    path.write_text(src.replace(old, new))
    lib_path = tmp_path / f"libomut{i}.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-I", os.path.dirname(src_path),
                    str(path), "-o", str(lib_path)], check=True)
    lib = ctypes.CDLL(str(lib_path))
    caught = {}
    for fn in ("m4ref_orbits_brute", "m4ref_orbits_esu"):
        f = getattr(lib, fn)
        f.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 3
        caught[fn] = False
        for _, make, expected in CLOSED:
            rp, col = make()
            rp = np.ascontiguousarray(rp, dtype=np.int64)
            col = np.ascontiguousarray(col if len(col) else np.zeros(1), dtype=np.int32)
            n = len(rp) - 1
            orb = np.zeros((max(n, 1), 11), dtype=np.uint64)
            rc = f(n, rp.ctypes.data, col.ctypes.data, orb.ctypes.data)
            if rc != 0 or not (orb[:n] == expected()).all():
                caught[fn] = True
                break
    assert all(caught.values()), caught
