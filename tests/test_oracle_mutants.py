"""The oracle pins have teeth: plausible mistakes planted in a copy of the
oracle source (compiled on the CPU into a temporary library) must each be
caught by the closed forms or by agreement with the all-subsets tier."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests import graphs as G
from tests.test_oracle_pins import CLOSED

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "m4ref.c")

# (tier entry point, exact source text, planted replacement)
MUTANTS = [
    ("m4ref_closure", "res[DIAMOND] = D - 6 * K4;", "res[DIAMOND] = D - 5 * K4;"),
    ("m4ref_closure", "if (te) Paw2 += te * (du + dv - 4);", "if (te) Paw2 += te * (du + dv - 2);"),
    ("m4ref_closure", "C4 += (u128)c * (c - 1) / 2;", "C4 += (u128)c * c / 2;"),
    ("m4ref_closure", "u128 Pni = P - 3 * T;", "u128 Pni = P - 2 * T;"),
    ("m4ref_closure", "if (inU[x] && inV[x]) K4++;", "if (inU[x]) K4++;"),
    ("m4ref_closure", "if (!before(rp, w, u)) continue;", "if (w == u) continue;"),
    ("m4ref_brute", "case 1223: return PAW;", "case 1223: return PATH;"),
    ("m4ref_brute", "int k = classify(ab + ac + ad, ab + bc + bd, ac + bc + cd, ad + bd + cd);",
     "int k = classify(ab + ac + ad, ab + bc + bd, ac + bc + bd, ad + bd + cd);"),
    ("m4ref_esu", "if (u > s->root && !touches_sub(s, k, u) && u != w) E2[len2++] = u;",
     "if (u > s->root && u != w) E2[len2++] = u;"),
    ("m4ref_paper", "if (x != a && x != b && x != c) X[mult]++;", "X[mult]++;"),
    ("m4ref_paper", "star += c3 - (mH2 / 2) * (d - 2) + sum_c2 - tau;",
     "star += c3 - (mH2 / 2) * (d - 2) + sum_c2 + tau;"),
    ("m4ref_paper", "res[CYCLE] = cycle_pairs / 4;", "res[CYCLE] = cycle_pairs / 2;"),
]


def _compile(tmp_path, i, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / f"mut{i}.c"
    path.write_text(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC), "m4ref.h")
    lib = tmp_path / f"libmut{i}.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-I",
                    os.path.dirname(hdr), str(path), "-o", str(lib)], check=True)
    return ctypes.CDLL(str(lib))


def _run(lib, fn, g):
    rp = np.ascontiguousarray(g[0], dtype=np.int64)
    col = np.ascontiguousarray(g[1], dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    out = np.zeros(6, dtype=np.uint64)
    f = getattr(lib, fn)
    if fn == "m4ref_closure":
        f.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 2 + [ctypes.c_int] + [ctypes.c_void_p] * 3
        rc = f(len(rp) - 1, rp.ctypes.data, col.ctypes.data, 1, out.ctypes.data, None, None)
    else:
        f.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 3
        rc = f(len(rp) - 1, rp.ctypes.data, col.ctypes.data, out.ctypes.data)
    return None if rc != 0 else tuple(int(x) for x in out)


@pytest.mark.parametrize("i", range(len(MUTANTS)))
def test_mutant_is_caught(tmp_path, i):
    import oracle
    fn, old, new = MUTANTS[i]
    lib = _compile(tmp_path, i, old, new)
    caught = False
    for _, make, exp in CLOSED:
        if _run(lib, fn, make()) != exp:
            caught = True
            break
    if not caught:
        for s in range(10):
            g = G.gnp(14, 0.35, 500 + s)
            if _run(lib, fn, g) != oracle.brute(*g):
                caught = True
                break
    assert caught, f"planted mistake not detected: {new}"
