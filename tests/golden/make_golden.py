"""Writes the stored expected values under tests/golden/.

Calls only the CPU oracle (and the seeded input generators): no value here
comes from the GPU path.  Re-run after changing a generator:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def er_workload():
    rp, col = gg.er_c1(seed=1)
    esu = oracle.esu(rp, col)
    paper = oracle.paper(rp, col)
    cnt, basis = oracle.closure(rp, col, want_basis=True)
    assert esu == paper == cnt
    return {
        "workload": "G(n=2000, m=20000), generator seed 1",
        "source": "oracle: ESU enumeration of connected 4-sets (= printed closure "
                  "equations = plain closure counter)",
        "n": int(len(rp) - 1), "m": int(len(col) // 2),
        "counts": list(esu), "basis": basis,
    }


def batch_workload(count=64):
    out = []
    for i in range(count):
        kind, n, p, s = gg.batch_spec(i)
        rp, col = gg.batch_graph(i)
        c = oracle.closure(rp, col)
        if n <= 1200:
            assert oracle.esu(rp, col) == c
        out.append({"index": i, "kind": kind, "n": n, "param": p, "seed": s,
                    "m": int(len(col) // 2), "counts": list(c)})
    return {"workload": "first graphs of the uneven batch, generator seed 3",
            "source": "oracle: plain closure counter (ESU agrees where n <= 1200)",
            "graphs": out}


def web_workload():
    """The web-like R-MAT graph of the headline benchmark (scale 24, edge
    factor 16, (0.45, 0.22, 0.22, 0.11), seed 4): minutes of CPU time."""
    rp, col = gg.rmat_web(scale=24, edge_factor=16, seed=4)
    cnt, basis = oracle.closure(rp, col, want_basis=True)
    return {
        "workload": "R-MAT scale 24, edge factor 16, (a,b,c,d) = (0.45, 0.22, 0.22, 0.11), "
                    "generator seed 4, random id permutation, symmetrised and deduplicated",
        "source": "oracle: plain closure counter",
        "n": int(len(rp) - 1), "m": int(len(col) // 2),
        "counts": list(cnt), "basis": basis,
    }


if __name__ == "__main__":
    # python tests/golden/make_golden.py        -- the small workloads
    # python tests/golden/make_golden.py web24  -- the scale-24 web graph
    if sys.argv[1:] == ["web24"]:
        with open(os.path.join(HERE, "rmat_web_s24.json"), "w") as f:
            json.dump(web_workload(), f, indent=1)
    else:
        with open(os.path.join(HERE, "er_2000_20000.json"), "w") as f:
            json.dump(er_workload(), f, indent=1)
        with open(os.path.join(HERE, "batch_first64.json"), "w") as f:
            json.dump(batch_workload(), f, indent=1)
    print("written")
