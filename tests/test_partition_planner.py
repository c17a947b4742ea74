"""Host planner of the halo-partitioned path (Section III-E), checked without a
GPU: owner ranges tile the owners in order (so every anchor has exactly one
owner range, the one holding its canonical vertex), each range holds every
row its anchors read with exactly the stored prefix the kernels assume, and
the rows fit the device budget by the path's own accounting unless a range
is a single owner."""
import numpy as np
import pytest

import graphgen as gg
from tests import graphs as G


def rank_space(rp, col):
    """Rank-space CSR in (degree, id) order with sorted rows, as the library
    builds it: (nptr, col, dlo, dplus, r1) with r1 the first rank of degree
    at least 2."""
    rp = np.asarray(rp, np.int64)
    col = np.asarray(col, np.int64)
    n = len(rp) - 1
    d = np.diff(rp)
    order = np.lexsort((np.arange(n), d))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    src = np.repeat(np.arange(n), d)
    key = np.sort(rank[src] * n + rank[col])
    rs, rc = key // n, key % n
    dr = d[order]
    nptr = np.zeros(n + 1, np.int64)
    nptr[1:] = np.cumsum(dr)
    dlo = np.bincount(rs[rc < rs], minlength=n).astype(np.int32)
    dplus = (dr - dlo).astype(np.int32)
    r1 = int(np.searchsorted(dr, 2))
    return nptr, rc.astype(np.int32), dlo, dplus, r1


def rows_of(nptr, col):
    return [col[nptr[v]:nptr[v + 1]] for v in range(len(nptr) - 1)]


def tri_bytes(rows, dplus):
    return sum(4 * int(dplus[v]) + 28 for v, _, _ in rows)


def c4_bytes(rows, owners, dlo):
    return 512 + sum(4 * ln + 32 for _, _, ln in rows) + sum(16 * int(dlo[u]) + 4 for u in owners)


GRAPHS = [
    ("rmat10", lambda: gg.rmat(10, 8, 0.57, 0.19, 0.19, 3)),
    ("ba", lambda: gg.ba(600, 4, 5)),
    ("wheel", lambda: G.wheel(300)),
    ("bipartite", lambda: G.complete_bipartite(6, 150)),
    ("gnm", lambda: gg.gnm(400, 3000, 2)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("parts", [1, 3, 9])
def test_triangle_ranges(name, make, parts):
    import paper_2607_12074_amd as m4
    nptr, col, dlo, dplus, _ = rank_space(*make())
    n = len(nptr) - 1
    R = rows_of(nptr, col)
    total = sum(4 * int(dplus[v]) + 28 for v in range(n))
    cap = max(total // parts, 1)
    rc, ends, rows = m4.plan_partitions(0, nptr, col, dlo, dplus, 0, cap)
    if rc == m4.M4_ENOMEM:
        # only a lone owner may exceed the budget
        assert ends == [] or ends[-1] < n
        return
    assert rc == 0
    assert ends and ends[-1] == n and all(a < b for a, b in zip([0] + ends, ends))
    lo = 0
    for hi, rs in zip(ends, rows):
        vs = [v for v, _, _ in rs]
        assert len(vs) == len(set(vs))
        for v, first, ln in rs:
            assert first == dlo[v] and ln == dplus[v]
        held = set(vs)
        for u in range(lo, hi):
            assert u in held
            for w in R[u][dlo[u]:]:
                assert int(w) in held
        assert tri_bytes(rs, dplus) <= cap or hi - lo == 1
        lo = hi
    if parts == 1:
        assert len(ends) == 1


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("parts", [1, 3, 9])
def test_four_cycle_ranges(name, make, parts):
    import paper_2607_12074_amd as m4
    nptr, col, dlo, dplus, r1 = rank_space(*make())
    n = len(nptr) - 1
    R = rows_of(nptr, col)
    total = 512 + sum(4 * len(R[v]) + 32 + 16 * int(dlo[v]) + 4 for v in range(n))
    cap = max(total // parts, 1)
    rc, ends, rows = m4.plan_partitions(1, nptr, col, dlo, dplus, r1, cap)
    if rc == m4.M4_ENOMEM:
        assert ends == [] or ends[-1] < n
        return
    assert rc == 0
    if r1 == n:
        assert ends == []
        return
    assert ends[-1] == n and all(a < b for a, b in zip([r1] + ends, ends))
    lo = r1
    for hi, rs in zip(ends, rows):
        got = {v: (first, ln) for v, first, ln in rs}
        assert len(got) == len(rs)
        owners = range(lo, hi)
        # members: the owners and their lower neighbours, nothing else
        want = set(owners)
        for u in owners:
            want.update(int(v) for v in R[u][:dlo[u]])
        assert set(got) == want
        for v, (first, ln) in got.items():
            # row v cut below the range's end: every wedge endpoint w < u of
            # an owner u in the range is held
            assert first == 0 and ln == int(np.searchsorted(R[v], hi))
        assert c4_bytes(rs, owners, dlo) <= cap or hi - lo == 1
        lo = hi


def test_every_anchor_has_one_owner_range():
    # triangles by their lowest vertex and 4-cycles by their highest, brute
    # force on a small graph: each lies in exactly one range, which holds
    # the rows the anchor reads
    import paper_2607_12074_amd as m4
    nptr, col, dlo, dplus, r1 = rank_space(*gg.gnm(60, 300, 7))
    n = len(nptr) - 1
    R = rows_of(nptr, col)
    adj = [set(map(int, r)) for r in R]
    rc, tends, trows = m4.plan_partitions(0, nptr, col, dlo, dplus, 0, 2000)
    assert rc == 0 and len(tends) >= 3
    rc, cends, crows = m4.plan_partitions(1, nptr, col, dlo, dplus, r1, 3000)
    assert rc == 0 and len(cends) >= 3

    def range_of(ends, start, x):
        lo = start
        for k, hi in enumerate(ends):
            if lo <= x < hi:
                return k
            lo = hi
        return None

    for u in range(n):
        for v in adj[u]:
            for w in adj[u] & adj[v]:
                if u < v < w:
                    k = range_of(tends, 0, u)
                    held = {r[0] for r in trows[k]}
                    assert u in held and v in held
    for u in range(n):
        for v in adj[u]:
            for x in adj[v]:
                if v < u and x < u and x != u:
                    k = range_of(cends, r1, u)
                    assert k is not None
                    held = {r[0]: r[2] for r in crows[k]}
                    # the wedge endpoint x of owner u via v is in v's stored prefix
                    assert x in set(map(int, R[v][:held[v]]))


def test_lone_owner_beyond_budget():
    import paper_2607_12074_amd as m4
    nptr, col, dlo, dplus, r1 = rank_space(*G.wheel(400))
    rc, _, _ = m4.plan_partitions(1, nptr, col, dlo, dplus, r1, 2048)
    assert rc == m4.M4_ENOMEM
    rc, _, _ = m4.plan_partitions(0, nptr, col, dlo, dplus, 0, 64)
    assert rc == m4.M4_ENOMEM
    rc, _, _ = m4.plan_partitions(0, nptr, col, dlo, dplus, 0, 1 << 30, max_ranges=0)
    assert rc == m4.M4_ERANGE
