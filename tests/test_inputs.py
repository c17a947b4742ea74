"""Seeded input generators: determinism and simplicity of the CSR they emit."""
import numpy as np
import pytest

import graphgen as gg
import oracle


def _simple(rp, col):
    return oracle.validate(rp, col)


@pytest.mark.parametrize("make", [
    lambda s: gg.gnm(300, 2000, s),
    lambda s: gg.rmat(12, 8, 0.57, 0.19, 0.19, s),
    lambda s: gg.ba(500, 4, s),
    lambda s: gg.chunglu(3000, 2.3, 8.0, s),
    lambda s: gg.rgg(3000, 9.0, s),
])
def test_deterministic_and_simple(make):
    a = make(5)
    b = make(5)
    c = make(6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not (len(a[1]) == len(c[1]) and np.array_equal(a[1], c[1]))
    assert _simple(*a)


def test_gnm_exact_edge_count():
    rp, col = gg.gnm(2000, 20000, 1)
    assert len(rp) == 2001 and len(col) == 40000
    rp, col = gg.gnm(20, 1000, 1)  # clipped to the complete graph
    assert len(col) == 20 * 19


def test_ba_edge_count():
    n, m = 300, 3
    rp, col = gg.ba(n, m, 2)
    assert len(col) // 2 == m + (n - m - 1) * m


def test_rmat_thread_count_independent():
    import os
    import subprocess
    import sys
    code = ("import graphgen as gg, hashlib;"
            "rp,c=gg.rmat(14,10,0.57,0.19,0.19,9);"
            "print(hashlib.sha1(c.tobytes()).hexdigest())")
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                           text=True, cwd=os.path.dirname(os.path.dirname(__file__)))
        outs.append(r.stdout.strip())
    assert outs[0] == outs[1] and len(outs[0]) == 40


def test_batch_and_serve_specs():
    ns = [gg.batch_spec(i)[1] for i in range(2000)]
    assert min(ns) >= 20 and max(ns) <= 5000
    kinds = {gg.batch_spec(i)[0] for i in range(10)}
    assert kinds == {"gnm", "ba"}
    sn = [gg.serve_spec(i)[1] for i in range(2000)]
    assert max(sn) <= 2_000_000
    assert 3000 < float(np.median(sn)) < 8000
