"""Halo-partitioned path (ownership-preserving derivation, Section III-E):
under a device budget that forces many owner ranges the counts, the closure
basis and the anchor work must equal the resident run bit for bit."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2607_12074_amd as m4
    c = m4.Context(0)
    yield c
    c.close()


def budget_for(g, parts):
    """A device budget that holds the n-sized arrays, the per-edge triangle
    counts and about 1/parts of the rows with their halos."""
    n, nnz = len(g[0]) - 1, len(g[1])
    fixed = 96 * n + 2 * nnz + (1 << 17)
    return fixed + (8 * nnz + 40 * n) // parts


CASES = [
    ("rmat12", lambda: gg.rmat(12, 8, 0.57, 0.19, 0.19, 5)),
    ("gnm", lambda: gg.gnm(3000, 24000, 9)),
    ("ba", lambda: gg.ba(3000, 5, 4)),
    ("wheel", lambda: G.wheel(4000)),
    ("bipartite", lambda: G.complete_bipartite(3, 3000)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_partition_equals_resident(ctx, name, make):
    import paper_2607_12074_amd as m4
    g = make()
    # halo partitions count 4-cycles with wedges: the resident reference too
    ref, rst = ctx.count(*g, flags=m4.M4_BASIS_WEDGE, stats=True)
    assert ref == oracle.closure(*g)
    for parts in (2, 6):
        got, st = ctx.count(*g, flags=m4.M4_FORCE_PARTITION | m4.M4_STATS,
                            budget=budget_for(g, parts), stats=True)
        assert got == ref, (name, parts)
        for k in ("T", "K4", "C4_ni", "S", "P_ni", "Paw_ni", "D_ni", "sum_t"):
            assert st[k] == rst[k], (name, parts, k)
        # every anchor is counted by exactly one owner range
        assert st["cache_lookups"] == rst["cache_lookups"]
        assert st["wedges"] == rst["wedges"]
        assert st["partitions"] >= 3


def test_partition_budget_sweep_and_device_input(ctx):
    import torch
    import paper_2607_12074_amd as m4
    g = gg.rmat(13, 6, 0.57, 0.19, 0.19, 11)
    ref = ctx.count(*g)
    seen = set()
    for parts in (1, 3, 12):
        got, st = ctx.count(*g, flags=m4.M4_FORCE_PARTITION, budget=budget_for(g, parts),
                            stats=True)
        assert got == ref, parts
        seen.add(st["partitions"])
    assert len(seen) >= 2
    rp, col = (torch.from_numpy(np.asarray(a)).cuda() for a in g)
    assert ctx.count(rp, col, flags=m4.M4_FORCE_PARTITION, budget=budget_for(g, 4)) == ref


def test_partition_budget_too_small_is_an_error(ctx):
    import paper_2607_12074_amd as m4
    g = gg.gnm(2000, 10000, 3)
    with pytest.raises(m4.M4Error) as e:
        ctx.count(*g, flags=m4.M4_FORCE_PARTITION, budget=4096)
    assert e.value.code == m4.M4_ENOMEM


def test_web_rmat_under_budget(ctx):
    # web-like R-MAT (the skew of the scale-24 web workload at scale 19),
    # resident and under a budget that holds about a third of the rows
    g = gg.rmat(19, 16, 0.45, 0.22, 0.22, 4)
    ref, rst = ctx.count(*g, stats=True)
    got, st = ctx.count(*g, budget=budget_for(g, 3), stats=True)
    assert got == ref
    assert st["partitions"] >= 3 and st["h2d_bytes"] > 0
    for k in ("T", "K4", "C4_ni", "D_ni"):
        assert st[k] == rst[k], k


def test_partition_with_ranged_medium_table(ctx):
    # owners with wedge bounds in (12288, 65536] counted over rank ranges of
    # the medium table (c4_med_win=1 sends all of them there), on stored row
    # prefixes of a partition
    import paper_2607_12074_amd as m4
    g = gg.rmat(16, 12, 0.57, 0.19, 0.19, 21)
    saved = ctx.get_tuning()
    try:
        ctx.set_tuning(c4_med_win=1)
        ref, rst = ctx.count(*g, flags=m4.M4_BASIS_WEDGE, stats=True)
        assert ref == oracle.closure(*g)
        got, st = ctx.count(*g, flags=m4.M4_FORCE_PARTITION | m4.M4_STATS,
                            budget=budget_for(g, 4), stats=True)
        assert got == ref
        assert st["partitions"] >= 3
        for k in ("C4_ni", "wedges"):
            assert st[k] == rst[k], k
    finally:
        ctx.set_tuning(**saved)


def test_budget_caps_the_device_footprint():
    # A budgeted call frees the workspaces of earlier resident calls and
    # holds no more than the budget: measured from the device's free memory
    # (the library allocates with hipMalloc, outside torch's cache).
    import torch
    import paper_2607_12074_amd as m4
    g = gg.rmat(15, 12, 0.57, 0.19, 0.19, 21)
    ref = oracle.closure(*g)
    budget = budget_for(g, 4)
    # the runtime's own device memory (code objects loaded at a kernel's
    # first launch, private-segment scratch) comes from a first pair of calls
    # on a throw-away context, so that it is not charged to the one measured
    warm = m4.Context(0)
    try:
        warm.count(*g)
        warm.count(*g, budget=budget)
    finally:
        warm.close()
    c = m4.Context(0)
    try:
        free0, _ = torch.cuda.mem_get_info(0)
        got, st = c.count(*g, stats=True)  # resident: grows the workspaces
        assert got == ref
        free1, _ = torch.cuda.mem_get_info(0)
        assert free0 - free1 >= st["device_bytes"] // 2
        # below the resident footprint: the call must partition by itself
        assert budget < st["device_bytes"]
        got, st = c.count(*g, budget=budget, stats=True)
        assert got == ref and st["partitions"] >= 3
        assert st["device_bytes"] <= budget
        free2, _ = torch.cuda.mem_get_info(0)
        # allocation granularity aside, the context now holds <= the budget
        assert free0 - free2 <= budget + (4 << 20), (free0 - free2, budget)
    finally:
        c.close()
