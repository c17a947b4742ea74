"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each oracle tier (all subsets, ESU, the printed closure equations, the plain
closure counter) is checked against:
  * closed forms derived from the definition of an induced occurrence as a
    4-vertex subset (Section II) for named graph families;
  * an independent classifier (networkx graph isomorphism against the six
    pattern graphs) and networkx connectivity on tiny graphs;
  * networkx triangle, common-neighbour and clique routines and the trace
    identities of the adjacency matrix for the anchor basis;
  * invariants: disjoint-union additivity and relabelling invariance.
"""
import itertools
from math import comb

import numpy as np
import pytest

import oracle
import graphgen as gg
from tests import graphs as G

TIERS = [oracle.brute, oracle.esu, oracle.paper, oracle.closure]
FAST_TIERS = [oracle.esu, oracle.paper, oracle.closure]


def all_tiers(g, tiers=TIERS):
    res = [f(*g) for f in tiers]
    return res


# ------------------------------------------------------------ closed forms
# Counts are (star, path, paw, cycle, diamond, clique).

def cf_complete(n):
    # every 4-subset of K_n induces K_4
    return (0, 0, 0, 0, 0, comb(n, 4))


def cf_star(leaves):
    # hub + 3 leaves induce a claw; 4 leaves induce no edge
    return (comb(leaves, 3), 0, 0, 0, 0, 0)


def cf_path(n):
    # connected 4-subsets of a path are 4 consecutive vertices
    return (0, max(n - 3, 0), 0, 0, 0, 0)


def cf_cycle(n):
    # C_4 is itself one 4-cycle; for n >= 5 the connected 4-subsets are the
    # n runs of 4 consecutive vertices, each an induced path
    return (0, 0, 0, 1, 0, 0) if n == 4 else (0, n, 0, 0, 0, 0)


def cf_bipartite(a, b):
    # 1 + 3 split -> claw, 2 + 2 split -> 4-cycle, 4 + 0 -> no edge
    return (a * comb(b, 3) + b * comb(a, 3), 0, 0, comb(a, 2) * comb(b, 2), 0, 0)


def cf_tree(g):
    # a tree has no cycles: claws are 3 neighbours of one centre; an induced
    # 4-path is a middle edge (u, v) plus one more neighbour on each side
    rp, col = g
    d = np.diff(rp)
    n = len(d)
    star = sum(comb(int(x), 3) for x in d)
    path = 0
    for u in range(n):
        for p in range(rp[u], rp[u + 1]):
            v = col[p]
            if v > u:
                path += (int(d[u]) - 1) * (int(d[v]) - 1)
    return (star, path, 0, 0, 0, 0)


def cf_wheel(k):
    # hub h + rim cycle of k >= 5 vertices.  Rim-only 4-sets: k paths.  Hub +
    # 3 rim vertices: 3 consecutive -> diamond (k), exactly one adjacent rim
    # pair -> paw (k(k-4)), no adjacent rim pair -> claw.
    return (comb(k, 3) - k - k * (k - 4), k, k * (k - 4), 0, k, 0)


CLOSED = [
    ("K4", lambda: G.complete(4), cf_complete(4)),
    ("K7", lambda: G.complete(7), cf_complete(7)),
    ("K12", lambda: G.complete(12), cf_complete(12)),
    ("K1,6", lambda: G.star(6), cf_star(6)),
    ("K1,15", lambda: G.star(15), cf_star(15)),
    ("P4", lambda: G.path(4), cf_path(4)),
    ("P9", lambda: G.path(9), cf_path(9)),
    ("C4", lambda: G.cycle(4), cf_cycle(4)),
    ("C5", lambda: G.cycle(5), cf_cycle(5)),
    ("C9", lambda: G.cycle(9), cf_cycle(9)),
    ("K3,4", lambda: G.complete_bipartite(3, 4), cf_bipartite(3, 4)),
    ("K5,6", lambda: G.complete_bipartite(5, 6), cf_bipartite(5, 6)),
    # K_{2,2,2}: omitting an antipodal pair leaves a 4-cycle (3 ways); any
    # other 4-set holds one antipodal non-edge only -> diamond (12 ways)
    ("octahedron", G.octahedron, (0, 0, 0, 3, 12, 0)),
    # Petersen: girth 5, 3-regular -> 10 * C(3,3) claws; every 4-path is a
    # middle edge with 2 x 2 extensions: 15 * 4 = 60
    ("petersen", G.petersen, (10, 60, 0, 0, 0, 0)),
    ("W7", lambda: G.wheel(7), cf_wheel(7)),
    ("W11", lambda: G.wheel(11), cf_wheel(11)),
    ("empty10", lambda: G.csr(10, []), (0,) * 6),
    ("K3", lambda: G.complete(3), (0,) * 6),
    ("single", lambda: G.csr(1, []), (0,) * 6),
    ("nothing", lambda: G.csr(0, []), (0,) * 6),
]


@pytest.mark.parametrize("name,make,expected", CLOSED, ids=[c[0] for c in CLOSED])
def test_closed_forms(name, make, expected):
    g = make()
    for f in TIERS:
        assert f(*g) == expected, f.__name__


def test_wheel_instance_printed_value():
    # W8 (hub + 7-cycle) evaluates to (7, 7, 21, 0, 7, 0)
    assert cf_wheel(7) == (7, 7, 21, 0, 7, 0)


@pytest.mark.parametrize("seed", range(6))
def test_trees(seed):
    g = G.random_tree(30 + 7 * seed, seed)
    exp = cf_tree(g)
    for f in TIERS:
        assert f(*g) == exp, f.__name__


def test_tree_no_cycles_large():
    g = G.random_tree(3000, 99)
    cnt = oracle.closure(*g)
    assert cnt == cf_tree(g)
    assert cnt[3] == 0


# ------------------------------------------- independent classifier (networkx)

def _patterns():
    import networkx as nx
    paw = nx.Graph([(0, 1), (1, 2), (2, 0), (2, 3)])
    diamond = nx.complete_graph(4)
    diamond.remove_edge(0, 1)
    return [nx.star_graph(3), nx.path_graph(4), paw, nx.cycle_graph(4),
            diamond, nx.complete_graph(4)]


def nx_counts(g):
    import networkx as nx
    H = G.to_networkx(g)
    pats = _patterns()
    out = [0] * 6
    connected = 0
    for S in itertools.combinations(H.nodes(), 4):
        sub = H.subgraph(S)
        if nx.is_connected(sub):
            connected += 1
        for i, p in enumerate(pats):
            if sub.number_of_edges() == p.number_of_edges() and nx.is_isomorphic(sub, p):
                out[i] += 1
    return tuple(out), connected


@pytest.mark.parametrize("seed", range(12))
def test_networkx_isomorphism_classifier(seed):
    n = 7 + seed % 5
    g = G.gnp(n, 0.25 + 0.05 * (seed % 7), 1000 + seed)
    exp, connected = nx_counts(g)
    got = oracle.brute(*g)
    assert got == exp
    assert sum(got) == connected


def _random_graphs():
    out = []
    for s in range(40):
        n = 8 + (s * 7) % 33
        out.append(("gnp", G.gnp(n, 0.08 + 0.3 * ((s * 13) % 10) / 10, s)))
    for s in range(10):
        out.append(("ba", gg.ba(20 + 3 * s, 2 + s % 4, s)))
    for s in range(8):
        out.append(("planted", G.planted_cliques(40, 60, [5 + s % 4, 4], s)))
    return out


RANDOM = _random_graphs()


@pytest.mark.parametrize("idx", range(len(RANDOM)))
def test_tiers_agree_with_brute_force(idx):
    kind, g = RANDOM[idx]
    ref = oracle.brute(*g)
    for f in FAST_TIERS:
        assert f(*g) == ref, (kind, f.__name__)


def test_connected_sets_equal_sum_of_counts():
    import networkx as nx
    for s in range(5):
        g = G.gnp(10, 0.3, 77 + s)
        H = G.to_networkx(g)
        conn = sum(1 for S in itertools.combinations(range(10), 4)
                   if nx.is_connected(H.subgraph(S)))
        assert sum(oracle.esu(*g)) == conn
        assert sum(oracle.closure(*g)) == conn


# ------------------------------------------------------------- invariants

def test_disjoint_union_is_additive():
    a = G.gnp(25, 0.3, 5)
    b = gg.ba(30, 3, 6)
    u = G.disjoint_union(a, b)
    for f in FAST_TIERS:
        ca, cb, cu = f(*a), f(*b), f(*u)
        assert cu == tuple(x + y for x, y in zip(ca, cb)), f.__name__


def test_relabel_invariance():
    g = G.planted_cliques(60, 200, [6], 3)
    perm = np.random.default_rng(0).permutation(60)
    h = G.relabel(g, perm)
    for f in FAST_TIERS:
        assert f(*g) == f(*h), f.__name__


# ------------------------------------------------------ anchor-basis pins

def test_basis_trace_identities():
    # tr(A^3) = 6 T and tr(A^4) = 8 C4_ni + 2 sum d^2 - 2m (closed walks)
    for s, g in enumerate([G.gnp(120, 0.1, 1), gg.ba(400, 5, 2), gg.gnm(800, 6000, 3),
                           G.planted_cliques(300, 1500, [12, 9], 4)]):
        A = G.adjacency(g)
        d = A.sum(1)
        m = int(d.sum()) // 2
        A2 = A @ A
        tr3 = int(np.trace(A2 @ A))
        tr4 = int((A2 * A2).sum())
        _, basis = oracle.closure(*g, want_basis=True)
        assert tr3 == 6 * basis["T"], s
        assert tr4 == 8 * basis["C4_ni"] + 2 * int((d * d).sum()) - 2 * m, s
        assert basis["S"] == sum(comb(int(x), 3) for x in d)


def test_per_edge_triangles_match_networkx():
    import networkx as nx
    g = gg.gnm(500, 6000, 11)
    H = G.to_networkx(g)
    _, t = oracle.closure(*g, want_t=True)
    rp, col = g
    for u in range(0, 500, 7):
        for p in range(rp[u], rp[u + 1]):
            v = int(col[p])
            assert t[p] == len(list(nx.common_neighbors(H, u, v)))
            assert t[p] == oracle.common(rp, col, u, v)
    assert sum(nx.triangles(H).values()) == int(t.sum()) // 2


def test_cliques_match_networkx():
    import networkx as nx
    g = G.planted_cliques(300, 900, [15, 11, 8], 21)
    H = G.to_networkx(g)
    k4 = sum(1 for c in nx.enumerate_all_cliques(H) if len(c) == 4)
    _, basis = oracle.closure(*g, want_basis=True)
    assert basis["K4"] == k4
    assert oracle.closure(*g)[5] == k4


def test_complete_graph_basis():
    g = G.complete(9)
    _, t, basis = oracle.closure(*g, want_t=True, want_basis=True)
    assert (t == 7).all()  # every edge of K_n lies in n - 2 triangles
    assert basis["C4_ni"] == 3 * comb(9, 4)
    assert basis["K4"] == comb(9, 4)


def test_bipartite_cycles():
    g = G.complete_bipartite(6, 7)
    _, basis = oracle.closure(*g, want_basis=True)
    assert basis["C4_ni"] == comb(6, 2) * comb(7, 2)
    assert basis["T"] == 0


def test_validate():
    g = G.gnp(30, 0.2, 1)
    assert oracle.validate(*g)
    rp, col = g
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]
    assert not oracle.validate(rp, bad)


def _edges_csr(n, pairs):
    """CSR straight from directed (row, column) pairs, no symmetrisation or
    cleaning, rows sorted: for malformed inputs the generators would repair."""
    pairs = sorted(pairs)
    rp = np.zeros(n + 1, dtype=np.int64)
    for a, _ in pairs:
        rp[a + 1] += 1
    rp = np.cumsum(rp).astype(np.int64)
    return rp, np.array([b for _, b in pairs], dtype=np.int32)


def test_validate_rejects_each_malformation():
    path = [(0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 2)]
    assert oracle.validate(*_edges_csr(4, path))
    # an edge listed in one row only (asymmetric)
    assert not oracle.validate(*_edges_csr(4, path + [(0, 3)]))
    # a self-loop, listed symmetrically
    assert not oracle.validate(*_edges_csr(4, path + [(2, 2)]))
    # a duplicate entry in a row (not strictly increasing)
    assert not oracle.validate(*_edges_csr(4, path + [(0, 1), (1, 0)]))
    # ids out of range: n and -1
    rp, col = _edges_csr(4, path)
    for bad_id in (4, -1, 1 << 30):
        c2 = col.copy()
        c2[-1] = bad_id
        assert not oracle.validate(rp, c2), bad_id
    # row offsets that go backwards, and a first offset that is not 0
    rp2 = rp.copy()
    rp2[2], rp2[3] = rp2[3], rp2[2]
    assert not oracle.validate(rp2, col)
    rp3 = rp.copy()
    rp3[0] = 1
    assert not oracle.validate(rp3, col)


@pytest.mark.slow
def test_overflow_boundary_of_the_star():
    # K_{1,n} has C(n,3) induced 3-stars: 4 801 000 leaves stay below 2^64,
    # 4 801 500 do not, and the oracle reports that as status 3
    ok = G.star(4_801_000)
    assert oracle.closure(*ok) == (comb(4_801_000, 3), 0, 0, 0, 0, 0)
    with pytest.raises(oracle.OracleError, match="code 3"):
        oracle.closure(*G.star(4_801_500))


@pytest.mark.slow
def test_er_workload_closure_equals_esu():
    g = gg.er_c1()
    assert oracle.closure(*g) == oracle.esu(*g) == oracle.paper(*g)
