"""Small named graphs for the tests (edge lists -> symmetric CSR)."""
import itertools

import numpy as np

import graphgen as gg


def csr(n, edges):
    e = np.array(list(edges), dtype=np.int32).reshape(-1, 2)
    return gg.from_edges(n, e[:, 0], e[:, 1])


def complete(n):
    return csr(n, itertools.combinations(range(n), 2))


def star(leaves):
    return csr(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def path(n):
    return csr(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n):
    return csr(n, [(i, (i + 1) % n) for i in range(n)])


def complete_bipartite(a, b):
    return csr(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def wheel(k):
    """Hub 0 joined to every vertex of the cycle 1..k."""
    return csr(k + 1, [(0, i) for i in range(1, k + 1)] +
               [(i, i % k + 1) for i in range(1, k + 1)])


def octahedron():
    return csr(6, [(a, b) for a in range(6) for b in range(a + 1, 6) if b != a + 3 or a >= 3])


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return csr(10, outer + spokes + inner)


def random_tree(n, seed):
    rng = np.random.default_rng(seed)
    return csr(n, [(i, int(rng.integers(0, i))) for i in range(1, n)])


def gnp(n, p, seed):
    rng = np.random.default_rng(seed)
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    return csr(n, edges)


def planted_cliques(n, m, sizes, seed):
    """G(n, m) plus cliques of the given sizes on random vertex sets."""
    rng = np.random.default_rng(seed)
    rp, col = gg.gnm(n, m, seed)
    src = np.repeat(np.arange(n, dtype=np.int32), np.diff(rp))
    edges = list(zip(src.tolist(), col.tolist()))
    for s in sizes:
        vs = rng.choice(n, size=s, replace=False)
        edges += list(itertools.combinations(vs.tolist(), 2))
    return csr(n, edges)


def disjoint_union(g1, g2):
    rp1, c1 = g1
    rp2, c2 = g2
    n1 = len(rp1) - 1
    rp = np.concatenate([rp1, rp2[1:] + rp1[-1]]).astype(np.int64)
    col = np.concatenate([c1, c2 + n1]).astype(np.int32)
    return rp, col


def relabel(g, perm):
    """Vertex v becomes perm[v]."""
    rp, col = g
    n = len(rp) - 1
    src = np.repeat(np.arange(n, dtype=np.int32), np.diff(rp))
    return gg.from_edges(n, np.asarray(perm)[src], np.asarray(perm)[col])


def to_networkx(g):
    import networkx as nx
    rp, col = g
    n = len(rp) - 1
    G = nx.Graph()
    G.add_nodes_from(range(n))
    for u in range(n):
        for p in range(rp[u], rp[u + 1]):
            if col[p] > u:
                G.add_edge(u, int(col[p]))
    return G


def adjacency(g):
    rp, col = g
    n = len(rp) - 1
    A = np.zeros((n, n), dtype=np.int64)
    src = np.repeat(np.arange(n), np.diff(rp))
    A[src, col] = 1
    return A
