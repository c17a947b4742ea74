"""Per-vertex graphlet orbit counts (orbits 4..14) through the C-ABI entry
point m4_count_orbits4, element by element against the oracle's ESU
enumeration and the per-vertex closed forms; on larger graphs the orbit
totals against the resident count (a property that holds at any size)."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs as G
from tests.test_oracle_orbits import CLOSED, cf_complete, orbit_sums_to_counts

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    import paper_2607_12074_amd as m4
    c = m4.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,make,expected", CLOSED, ids=[c[0] for c in CLOSED])
def test_closed_forms(ctx, name, make, expected):
    got = ctx.orbits(*make())
    assert got.dtype == np.uint64 and (got == expected()).all(), name


RANDOM = [
    ("gnm", lambda: gg.gnm(700, 6000, 4)),
    ("ba", lambda: gg.ba(900, 5, 6)),
    ("rmat", lambda: gg.rmat(11, 8, 0.57, 0.19, 0.19, 8)),
    ("rmat_web", lambda: gg.rmat(11, 16, 0.45, 0.22, 0.22, 3)),
    ("planted", lambda: G.planted_cliques(300, 1500, [9, 12, 20], 3)),
    ("bipartite", lambda: G.complete_bipartite(12, 40)),
    ("wheel_cycle", lambda: G.disjoint_union(G.wheel(200), G.cycle(50))),
    ("dense", lambda: G.gnp(120, 0.35, 2)),
    ("tree", lambda: G.random_tree(500, 4)),
]


@pytest.mark.parametrize("name,make", RANDOM, ids=[r[0] for r in RANDOM])
def test_random_graphs_match_oracle(ctx, name, make):
    g = make()
    got = ctx.orbits(*g)
    want = oracle.orbits_esu(*g)
    bad = np.argwhere(got != want)
    assert bad.size == 0, (name, bad[:5].tolist())
    # the totals are the resident count's
    assert orbit_sums_to_counts(got)[0] == ctx.count(*g)


def test_counters_in_lds_and_device_memory(ctx):
    # 50000 vertices: the wedge counters of the top 32768 ranks sit in LDS,
    # the lower ranks' in device memory; every row still matches the oracle
    g = gg.gnm(50000, 150000, 9)
    got = ctx.orbits(*g)
    assert (got == oracle.orbits_esu(*g)).all()


def test_er_workload(ctx):
    gold = json.load(open(os.path.join(HERE, "golden", "er_2000_20000.json")))
    g = gg.gnm(2000, 20000, 1)
    got = ctx.orbits(*g)
    assert (got == oracle.orbits_esu(*g)).all()
    assert list(orbit_sums_to_counts(got)[0]) == gold["counts"]


def test_out_degree_beyond_the_lds_bitmap(ctx):
    # K_600 has out-degrees up to 599: owners above 512 keep their bitmap in
    # device scratch; beside a sparse graph, rows stay independent
    k, small = G.complete(600), gg.gnm(300, 1500, 2)
    got = ctx.orbits(*G.disjoint_union(k, small))
    assert (got[:600] == cf_complete(600)).all()
    assert (got[600:] == oracle.orbits_esu(*small)).all()


def test_degree_beyond_16_bit_counters(ctx):
    # K_{2,70000}: the top vertex's lower neighbours all reach the other
    # side-A vertex, 70000 wedges on one endpoint (wide 4-cycle counters)
    from tests.test_oracle_orbits import cf_bipartite
    got = ctx.orbits(*G.complete_bipartite(2, 70000))
    assert (got == cf_bipartite(2, 70000)).all()


def test_device_inputs_and_edge_cases(ctx):
    import torch
    import paper_2607_12074_amd as m4
    g = gg.ba(3000, 6, 1)
    host = ctx.orbits(*g)
    rp, col = torch.from_numpy(g[0]).cuda(), torch.from_numpy(g[1]).cuda()
    dev = ctx.orbits(rp, col)
    assert dev.is_cuda and (dev.cpu().numpy().view(np.uint64) == host).all()
    for n in (0, 1, 3, 7):
        e = G.csr(n, [])
        assert ctx.orbits(*e).shape == (n, 11) and not ctx.orbits(*e).any()
    assert not ctx.orbits(*G.complete(3)).any()
    # a device budget (halo partitions) is not offered for per-vertex counts
    with pytest.raises(m4.M4Error) as e:
        ctx.orbits(*g, budget=1 << 30)
    assert e.value.code == m4.M4_EINVAL


def test_social_scale18_totals(ctx):
    # every vertex's orbits at a size the oracle cannot enumerate: the totals
    # equal the resident count, and every row is consistent with its degree
    import torch
    rp, col = gg.rmat(18, 10, 0.57, 0.19, 0.19, 2)
    rpd, cold = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    got = ctx.orbits(rpd, cold).cpu().numpy().view(np.uint64)
    assert orbit_sums_to_counts(got)[0] == ctx.count(rpd, cold)
    d = np.diff(rp).astype(object)
    # claw centres: C(d, 3) minus the denser orbits that hold a 3-leaf star
    # at v (paw degree 3, diamond degree 3, clique)
    c = got.astype(object)
    assert (c[:, 3] + c[:, 7] + c[:, 9] + c[:, 10] == d * (d - 1) * (d - 2) // 6).all()


def test_validation_stream_and_range_errors(ctx):
    import torch
    import paper_2607_12074_amd as m4
    rp, col = G.gnp(40, 0.2, 1)
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]  # unsorted row
    with pytest.raises(m4.M4Error) as e:
        ctx.orbits(rp, bad, flags=m4.M4_VALIDATE)
    assert e.value.code == m4.M4_EINVAL
    with pytest.raises(m4.M4Error) as e:
        ctx.orbits(rp, col[:-2])  # row_ptr[n] != nnz
    assert e.value.code == m4.M4_ERANGE
    assert (ctx.orbits(rp, col, flags=m4.M4_VALIDATE) == oracle.orbits_brute(rp, col)).all()
    # on a caller stream, output on the device
    g = gg.rmat(12, 8, 0.57, 0.19, 0.19, 4)
    want = ctx.orbits(*g)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        rpd, cold = torch.from_numpy(g[0]).cuda(), torch.from_numpy(g[1]).cuda()
        got = ctx.orbits(rpd, cold)
    side.synchronize()
    assert (got.cpu().numpy().view(np.uint64) == want).all()
