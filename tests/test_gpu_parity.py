"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact on every count and on every per-edge triangle count."""
import json
import os
from math import comb

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs as G
from tests.test_oracle_pins import CLOSED, cf_wheel

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    import paper_2607_12074_amd as m4
    c = m4.Context(0)
    yield c
    c.close()


def test_closed_forms(ctx):
    # by the basis the anchor-selection objective picks (the edge basis for
    # most of these small graphs) and by the wedge basis
    import paper_2607_12074_amd as m4
    for name, make, exp in CLOSED:
        assert ctx.count(*make()) == exp, name
        assert ctx.count(*make(), flags=m4.M4_BASIS_WEDGE) == exp, name


def cocktail_party(k):
    # K_{2,2,...,2} with k parts: a 4-set holding 2 antipodal pairs is a
    # 4-cycle, 1 pair a diamond, none a 4-clique
    n = 2 * k
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if b != a + k]
    return G.csr(n, edges), (0, 0, 0, comb(k, 2), 4 * k * comb(k - 1, 2), 16 * comb(k, 4))


def test_dense_out_lists_global_bitmap(ctx):
    # out-degrees above 1024 take the bitmap-in-global-memory owners
    g, exp = cocktail_party(560)
    assert ctx.count(*g) == exp
    assert ctx.count(*G.complete(1050)) == (0, 0, 0, 0, 0, comb(1050, 4))


def test_hub_rows_and_window_counters(ctx):
    # a 40000-spoke wheel: the hub row is sorted by the bitmap kernel and the
    # hub's 4-cycle owner uses the windowed counters
    k = 40000
    assert ctx.count(*G.wheel(k)) == cf_wheel(k)
    assert ctx.count(*G.star(40000)) == (comb(40000, 3), 0, 0, 0, 0, 0)
    g = G.complete_bipartite(3, 70000)
    assert ctx.count(*g) == (3 * comb(70000, 3) + 70000 * comb(3, 3), 0, 0,
                             comb(3, 2) * comb(70000, 2), 0, 0)


def test_every_row_sort_class(ctx):
    # rows of 3000, 6000, 12000 and 20000 entries (bitonic sorts of 4096,
    # 8192 and 16384 slots, then the bitmap windows) beside short ones: the
    # per-edge triangle counts come back in the input layout, so every
    # sorted row is checked entry by entry, and the counts are the oracle's
    parts = [G.wheel(3000), G.wheel(6000), G.star(12000), G.wheel(20000), gg.gnm(2000, 9000, 5)]
    g = parts[0]
    for h in parts[1:]:
        g = G.disjoint_union(g, h)
    ref, t_ref = oracle.closure(*g, want_t=True)
    assert ctx.count(*g) == ref
    assert (ctx.edge_triangles(*g) == t_ref).all()


def test_multi_window_long_segments(ctx):
    # A 300000-cycle below K_{50,200}: the cycle's degree-2 ranks fill more
    # than one window of 4-bit counters (262144 per window), so the 4-cycle
    # owners (the 50 side) see their lower neighbours' rows only in the
    # second window, and every such visit is longer than 8 entries; the
    # relabelled copy mixes the two parts in the input ids (not in the
    # degree order).
    cyc, bip = G.cycle(300000), G.complete_bipartite(50, 200)
    exp = tuple(a + b for a, b in zip(
        (0, 300000, 0, 0, 0, 0),
        (50 * comb(200, 3) + 200 * comb(50, 3), 0, 0, comb(50, 2) * comb(200, 2), 0, 0)))
    g = G.disjoint_union(cyc, bip)
    assert ctx.count(*g) == exp
    perm = np.random.default_rng(3).permutation(len(g[0]) - 1)
    assert ctx.count(*G.relabel(g, perm)) == exp
    # hubs whose windows hold both short and long visits, against the oracle
    h = G.disjoint_union(G.disjoint_union(cyc, bip), gg.ba(3000, 12, 7))
    assert ctx.count(*h) == oracle.closure(*h)


def _random_cases():
    out = []
    for s in range(30):
        n = 10 + (s * 37) % 300
        p = 0.02 + 0.25 * ((s * 13) % 10) / 10
        out.append(G.gnp(n, p, 100 + s))
    for s in range(8):
        out.append(gg.ba(200 + 50 * s, 2 + s, s))
    for s in range(6):
        out.append(G.planted_cliques(400, 2000, [30 + 10 * s, 12], s))
    out.append(gg.rmat(12, 8, 0.57, 0.19, 0.19, 3))
    out.append(gg.chunglu(5000, 2.2, 10.0, 4))
    out.append(gg.rgg(5000, 10.0, 5))
    return out


def test_random_graphs_vs_oracle(ctx):
    import paper_2607_12074_amd as m4
    for i, g in enumerate(_random_cases()):
        ref = oracle.closure(*g)
        assert ctx.count(*g) == ref, i
        assert ctx.count(*g, flags=m4.M4_BASIS_WEDGE) == ref, i


def test_small_graphs_vs_brute_force(ctx):
    for s in range(20):
        g = G.gnp(9 + s % 12, 0.3, 900 + s)
        ref = oracle.brute(*g)
        assert ctx.count(*g) == ref, s
        assert ctx.count(*g, flags=__import__("paper_2607_12074_amd").M4_BASIS_WEDGE) == ref, s


def test_er_workload_golden(ctx):
    gold = json.load(open(os.path.join(HERE, "golden", "er_2000_20000.json")))
    g = gg.er_c1(seed=1)
    import paper_2607_12074_amd as m4
    for fl in (0, m4.M4_BASIS_WEDGE, m4.M4_BASIS_EDGE):
        counts, st = ctx.count(*g, flags=fl, stats=True)
        assert list(counts) == gold["counts"], fl
        for k, v in gold["basis"].items():
            assert st[k] == v, (fl, k)


def test_batch_golden_graphs_single(ctx):
    gold = json.load(open(os.path.join(HERE, "golden", "batch_first64.json")))
    for rec in gold["graphs"][:24]:
        g = gg.batch_graph(rec["index"])
        assert list(ctx.count(*g)) == rec["counts"], rec["index"]


def test_edge_triangles_elementwise(ctx):
    for g in (gg.er_c1(seed=1), gg.rmat(13, 10, 0.57, 0.19, 0.19, 7),
              G.planted_cliques(600, 3000, [70, 25], 9)):
        _, t_ref = oracle.closure(*g, want_t=True)
        t = ctx.edge_triangles(*g)
        assert np.array_equal(t, t_ref)


def test_cache_modes_identical(ctx):
    import paper_2607_12074_amd as m4
    for g in (G.planted_cliques(500, 2500, [90, 40, 20], 3),
              gg.rmat(13, 12, 0.57, 0.19, 0.19, 11)):
        ref = oracle.closure(*g)
        on, st_on = ctx.count(*g, stats=True)
        off, st_off = ctx.count(*g, flags=m4.M4_NO_CACHE, stats=True)
        tiny, st_tiny = ctx.count(*g, cache_rows=3, stats=True)
        assert on == off == tiny == ref
        assert st_on["cache_lookups"] == st_off["cache_lookups"] == st_tiny["cache_lookups"]
        assert st_on["cache_hits"] == st_on["cache_lookups"] > 0
        assert st_off["cache_hits"] == 0
        assert 0 < st_tiny["cache_hits"] < st_tiny["cache_lookups"]


def test_threshold_sweep_identical(ctx):
    g = gg.rmat(14, 10, 0.57, 0.19, 0.19, 5)
    ref = oracle.closure(*g)
    for tw in (2, 5, 16, 64):
        for cl in (1, 64, 2048):
            assert ctx.count(*g, tri_wave_max=tw, c4_light_max=cl) == ref, (tw, cl)
    # medium 4-cycle bucket: none, below the light bound (empty), partial, full
    for cl, md in ((64, -1), (2048, 1000), (64, 3000), (1, 12288)):
        got, st = ctx.count(*g, c4_light_max=cl, c4_med_max=md, stats=True)
        assert got == ref, (cl, md)


def test_medium_bucket_rank_ranges(ctx):
    # owners with wedge bounds above 3/4 of the medium table are counted over
    # rank ranges: K_{30,2000} (several endpoints per range), K_{8,9000} (one
    # endpoint bin above the range capacity), and an R-MAT graph whose owners
    # span more ranks than the table has bins; c4_med_win=1 sends every
    # owner with a bound up to 65536 there, whatever its window count
    import paper_2607_12074_amd as m4
    med = m4.KERNELS.index("c4_med")
    saved = ctx.get_tuning()
    try:
        for g in (G.complete_bipartite(30, 2000), G.complete_bipartite(8, 9000),
                  gg.rmat(16, 12, 0.57, 0.19, 0.19, 21)):
            ref = oracle.closure(*g)
            seen = []
            for md, mw in ((-1, 0), (12288, 0), (12288, 1)):
                ctx.set_tuning(c4_med_win=mw)
                got, st = ctx.count(*g, c4_med_max=md, flags=m4.M4_BASIS_WEDGE, stats=True)
                assert got == ref, (md, mw)
                seen.append(st["k_rows"][med])
            assert seen[0] == 0 and seen[2] > seen[1]
    finally:
        ctx.set_tuning(**saved)


def test_serial_and_overlapped_stages_agree(ctx):
    # the triangle and 4-cycle stages overlap on two streams by default;
    # M4_SERIAL runs them on one: counts, basis and work counters agree
    import paper_2607_12074_amd as m4
    g = gg.rmat(16, 12, 0.57, 0.19, 0.19, 23)
    ref = oracle.closure(*g)
    b, sb = ctx.count(*g, flags=m4.M4_SERIAL | m4.M4_BASIS_WEDGE, stats=True)
    assert b == ref
    for _ in range(3):
        a, sa = ctx.count(*g, flags=m4.M4_BASIS_WEDGE, stats=True)
        assert a == ref
        for k in ("T", "K4", "C4_ni", "S", "P_ni", "Paw_ni", "D_ni", "sum_t", "wedges",
                  "intersect_steps", "cache_lookups"):
            assert sa[k] == sb[k], k


def test_caller_stream_and_tuning_bounds(ctx):
    # device tensors on a side torch stream: the count is ordered on that
    # stream (the 4-cycle stage forks from it and joins back into it)
    import torch
    import paper_2607_12074_amd as m4
    g = gg.rmat(15, 10, 0.57, 0.19, 0.19, 31)
    ref = oracle.closure(*g)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        rp = torch.from_numpy(g[0]).cuda()
        col = torch.from_numpy(g[1]).cuda()
        for _ in range(2):
            assert ctx.count(rp, col) == ref
    side.synchronize()
    # out-of-range thresholds are rejected and leave the tuning unchanged
    before = ctx.get_tuning()
    for bad in ({"c4_med_max": 20000}, {"c4_med_win": -1}, {"probe_w": 0},
                {"tri_wave_max": 65}, {"hub_min": 2}, {"tri_wave_far": 1}, {"probe_w_far": 300},
                {"c4_bin_dense": 32}):
        with pytest.raises(m4.M4Error) as e:
            ctx.set_tuning(**bad)
        assert e.value.code == m4.M4_EINVAL
    assert ctx.get_tuning() == before


def test_device_tensor_input(ctx):
    import torch
    g = gg.rmat(12, 10, 0.57, 0.19, 0.19, 8)
    rp = torch.from_numpy(g[0]).cuda()
    col = torch.from_numpy(g[1]).cuda()
    assert ctx.count(rp, col) == ctx.count(*g) == oracle.closure(*g)
    t_dev = ctx.edge_triangles(rp, col).cpu().numpy().view(np.uint32)
    assert np.array_equal(t_dev, ctx.edge_triangles(*g))


def test_validation_rejects_malformed(ctx):
    import paper_2607_12074_amd as m4
    rp, col = G.gnp(40, 0.2, 1)
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]  # unsorted row
    with pytest.raises(m4.M4Error) as e:
        ctx.count(rp, bad, flags=m4.M4_VALIDATE)
    assert e.value.code == m4.M4_EINVAL
    # asymmetric: drop one direction of an edge
    rp2, col2 = G.csr(4, [(0, 1), (1, 2), (2, 3)])
    col3 = col2.copy()
    col3[0] = 2  # 0 -> 2 without 2 -> 0
    with pytest.raises(m4.M4Error):
        ctx.count(rp2, col3, flags=m4.M4_VALIDATE)
    assert ctx.count(rp, col, flags=m4.M4_VALIDATE) == oracle.closure(rp, col)
    with pytest.raises(m4.M4Error) as e:
        ctx.count(rp, col[:-2])
    assert e.value.code == m4.M4_ERANGE


def test_empty_and_tiny(ctx):
    assert ctx.count(*G.csr(0, [])) == (0,) * 6
    assert ctx.count(*G.csr(3, [(0, 1), (1, 2)])) == (0,) * 6
    assert ctx.count(*G.csr(100, [])) == (0,) * 6
    assert ctx.count(*G.csr(5, [(0, 1), (1, 2), (2, 3)])) == (0, 1, 0, 0, 0, 0)


def test_repeat_is_deterministic(ctx):
    g = gg.rmat(14, 12, 0.57, 0.19, 0.19, 13)
    a = ctx.count(*g)
    b = ctx.count(*g)
    assert a == b == oracle.closure(*g)


def test_overflow_boundary_of_the_star(ctx):
    # C(n, 3) induced 3-stars: 4 801 000 leaves fit in 64 bits, 4 801 500 do
    # not (the oracle reports status 3 for the same graph)
    import paper_2607_12074_amd as m4
    assert ctx.count(*G.star(4_801_000)) == (comb(4_801_000, 3), 0, 0, 0, 0, 0)
    with pytest.raises(m4.M4Error) as e:
        ctx.count(*G.star(4_801_500))
    assert e.value.code == m4.M4_EOVERFLOW


def test_web_scale24_matches_oracle_golden(ctx):
    # the headline workload at its full size (268 M edges, CSR on the device
    # as in the bench): counts and basis equal the oracle's stored values
    import torch
    gold = json.load(open(os.path.join(HERE, "golden", "rmat_web_s24.json")))
    rp, col = gg.rmat_web(scale=24, edge_factor=16, seed=4)
    assert (len(rp) - 1, len(col) // 2) == (gold["n"], gold["m"])
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    del rp, col
    counts, st = ctx.count(rp_d, col_d, stats=True)
    assert list(counts) == gold["counts"]
    for k, v in gold["basis"].items():
        assert st[k] == v, k


def test_binned_four_cycle_owners(ctx):
    # every owner above the one-pass table bound binned by counter window
    # (c4_bin_win = 1), or only those spanning several windows, or none; the
    # binning scratch shrunk to 1000 endpoints (owners scattered in several
    # rank ranges) or to 64 (buckets alone beyond it, counted straight from
    # the rows); owners dense over their windows (c4_bin_dense) kept on the
    # window kernel beside binned ones in the same count: the counts never
    # change; the 300000-cycle graph spans two windows
    import paper_2607_12074_amd as m4
    cyc, bip = G.cycle(300000), G.complete_bipartite(50, 200)
    graphs = [gg.rmat(14, 10, 0.57, 0.19, 0.19, 5), gg.rmat(15, 16, 0.45, 0.22, 0.22, 6),
              gg.ba(6000, 9, 2), G.complete_bipartite(7, 900), G.complete_bipartite(60, 3000),
              G.disjoint_union(G.disjoint_union(cyc, bip), gg.ba(3000, 12, 7))]
    base = ctx.get_tuning()
    slot = m4.KERNELS.index("c4_bin")
    wslot = m4.KERNELS.index("c4_window")
    binned = split = 0
    try:
        for g in graphs:
            ref = oracle.closure(*g)
            # (bin_win, bin_cap, bin_dense, light_max, med_max); the last two
            # bin owners from 256 endpoints so that a dense bound of 512 or
            # 2048 per window splits them between the two kernels
            for bw, cap, bd, lm, mm in ((1, 0, 0, 2048, 6144), (1, 1000, 0, 2048, 6144),
                                        (1, 64, 0, 2048, 6144), (2, 0, 0, 2048, 6144),
                                        (0, 0, 0, 2048, 6144), (1, 0, 512, 256, 0),
                                        (1, 1000, 2048, 256, 0)):
                ctx.set_tuning(c4_bin_win=bw, c4_bin_cap=cap, c4_bin_dense=bd, c4_light_max=lm,
                               c4_med_max=mm)
                got, st = ctx.count(*g, flags=m4.M4_BASIS_WEDGE, stats=True)
                assert got == ref, (bw, cap, bd, lm, mm)
                if bw == 0:
                    assert st["k_rows"][slot] == 0
                else:
                    binned += st["k_rows"][slot]
                    # every wedge endpoint of a binned owner is counted once
                    assert st["k_elems"][slot] <= st["wedges"]
                    if bd and st["k_rows"][slot] and st["k_rows"][wslot]:
                        split += 1
    finally:
        ctx.set_tuning(**base)
    assert binned > 0 and split > 0
