"""Allocation-free entry point m4_count_motifs4_noalloc (for callers that
cannot allocate device memory) against m4_count_motifs4_ex on the same
device CSR: two calls in a row, the second with a smaller graph, with no
change in the device's free memory across a call; the errors it reports for
host input, a device budget and a graph beyond its fixed scratch."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _dev(g):
    import torch
    return torch.from_numpy(g[0]).cuda(), torch.from_numpy(g[1]).cuda()


@pytest.fixture(scope="module")
def ctx():
    import paper_2607_12074_amd as m4
    c = m4.Context(0)
    yield c
    c.close()


def test_matches_the_allocating_count_twice_second_smaller(ctx):
    import torch
    big = _dev(gg.rmat(16, 10, 0.57, 0.19, 0.19, 3))
    small = _dev(gg.gnm(2000, 20000, 1))
    want_big, want_small = ctx.count(*big), ctx.count(*small)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got_big = ctx.count_noalloc(*big)
    got_small = ctx.count_noalloc(*small)
    torch.cuda.synchronize()
    assert got_big == want_big and got_small == want_small
    assert torch.cuda.mem_get_info()[0] == free0
    # the context's own workspaces are untouched: an allocating count after
    # it gives the same result
    assert ctx.count(*big) == want_big


def test_errors(ctx):
    import paper_2607_12074_amd as m4
    g = gg.gnm(500, 3000, 2)
    with pytest.raises(m4.M4Error) as e:
        ctx.count_noalloc(*g)  # host arrays
    assert e.value.code == m4.M4_EINVAL
    d = _dev(g)
    with pytest.raises(m4.M4Error) as e:
        ctx.count_noalloc(*d, budget=1 << 30)
    assert e.value.code == m4.M4_EINVAL
    # a path on 8 M vertices needs more workspace than the fixed array
    n = 8_000_000
    src = np.arange(n - 1, dtype=np.int32)
    big = _dev(gg.from_edges(n, src, src + 1))
    with pytest.raises(m4.M4Error) as e:
        ctx.count_noalloc(*big)
    assert e.value.code == m4.M4_ENOMEM
    # and the small graph still counts afterwards
    assert ctx.count_noalloc(*d) == ctx.count(*d)
