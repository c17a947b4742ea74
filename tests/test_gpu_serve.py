"""Serving loop: each request's counts are identical alone and in the mix
(tolerance 0: the counts are integers), the admitted device footprint never
exceeds the budget, and oversize requests and a full queue are reported."""
import time

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


def _collect(srv, want, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < want:
        for r in srv.poll(256):
            out[r["id"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(out)} of {want} results")
        time.sleep(0.001)
    return out


def test_mix_equals_alone(ctx):
    import paper_2607_12074_amd as m4
    graphs = [gg.serve_graph(i, seed=21) for i in range(48)]
    graphs += [gg.rmat(14, 8, 0.57, 0.19, 0.19, 1), G.wheel(20000)]  # beyond one workgroup
    import torch
    budget = 512 << 20
    free0, _ = torch.cuda.mem_get_info(0)
    srv = m4.Server(ctx, budget)
    ids = {}
    for i, g in enumerate(graphs):
        ids[srv.submit(*g, tag=i)] = i
    res = _collect(srv, len(graphs))
    st = srv.stats()
    # lane arenas and the worker's workspaces are kept after the work: device
    # memory really allocated (hipMalloc, outside torch's cache)
    free1, _ = torch.cuda.mem_get_info(0)
    srv.close()
    assert st["max_inflight_bytes"] <= budget and st["launches"] >= 1
    assert free0 - free1 <= budget + (2 << 20), (free0 - free1, budget)
    for rid, r in res.items():
        i = ids[rid]
        assert r["tag"] == i and r["status"] == 0
        assert r["counts"] == ctx.count(*graphs[i]), i
        assert r["t_submit_ms"] <= r["t_admit_ms"] <= r["t_done_ms"]
    for i in range(0, len(graphs), 9):
        assert res[[k for k, v in ids.items() if v == i][0]]["counts"] == oracle.closure(*graphs[i])


def test_tight_budget_serialises_and_rejects(ctx):
    import paper_2607_12074_amd as m4
    import torch
    graphs = [gg.batch_graph(i, seed=4) for i in range(40)]
    budget = 16 << 20
    free0, _ = torch.cuda.mem_get_info(0)
    srv = m4.Server(ctx, budget)
    ids = [srv.submit(*g, tag=i) for i, g in enumerate(graphs)]
    big = gg.rmat(16, 16, 0.57, 0.19, 0.19, 2)  # needs more than the budget
    big_id = srv.submit(*big, tag=999)
    res = _collect(srv, len(ids) + 1)
    st = srv.stats()
    # what the server keeps after the work (lane arenas, worker workspaces)
    # is device memory really allocated (hipMalloc, outside torch's cache)
    free1, _ = torch.cuda.mem_get_info(0)
    srv.close()
    assert st["max_inflight_bytes"] <= budget
    assert free0 - free1 <= budget + (2 << 20), (free0 - free1, budget)
    assert res[big_id]["status"] == m4.M4_ENOMEM
    for rid, g in zip(ids, graphs):
        assert res[rid]["status"] == 0 and res[rid]["counts"] == ctx.count(*g)


def test_queue_limit(ctx):
    import paper_2607_12074_amd as m4
    srv = m4.Server(ctx, 1 << 30, max_queue=1)
    g = G.complete(6)
    accepted, busy = 0, 0
    for _ in range(200):
        try:
            srv.submit(*g)
            accepted += 1
        except m4.M4Error as e:
            assert e.code == m4.M4_EBUSY
            busy += 1
    srv.drain()
    res = srv.poll(1024)
    srv.close()
    assert len(res) == accepted and accepted >= 1
    assert all(r["counts"] == (0, 0, 0, 0, 0, 15) for r in res)
