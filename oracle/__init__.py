"""CPU oracle for connected induced 4-node motif counts -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product library never links, loads or
calls it, and it shares no code with the GPU path.

Counts are returned in the order
``(3-star, 4-path, tailed triangle, 4-cycle, diamond, 4-clique)``.

Tiers (all plain C in ``m4ref.c``, reached through ctypes):

* ``brute``   -- every 4-vertex subset classified by the degree sequence of its
  induced subgraph (the induced-occurrence definition, Section II).
* ``esu``     -- ESU enumeration (Wernicke 2006) of the connected 4-sets,
  classified the same way.
* ``paper``   -- the closure equations of Section III-F applied as printed.
* ``closure`` -- non-induced anchor counts (per-edge triangles, 4-cliques,
  4-cycles) plus the exact triangular inverse; also the CPU timing baseline.
* ``orbits_brute`` / ``orbits_esu`` -- per-vertex graphlet orbit counts
  (orbits 4..14) of the same induced 4-sets, from all subsets or ESU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "m4ref.c")
_LIB = os.path.join(_HERE, "libm4ref.so")
_lib = None

NAMES = ("star", "path", "paw", "cycle", "diamond", "clique")
BASIS = ("T", "K4", "C4_ni", "S", "P_ni", "Paw_ni", "D_ni", "sum_t")


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile libm4ref.so in place with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", _SRC,
               "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        for f in ("m4ref_brute", "m4ref_esu", "m4ref_paper"):
            getattr(lib, f).argtypes = [i64, p, p, p]
            getattr(lib, f).restype = ctypes.c_int
        lib.m4ref_closure.argtypes = [i64, p, p, ctypes.c_int, p, p, p]
        lib.m4ref_closure.restype = ctypes.c_int
        lib.m4ref_validate.argtypes = [i64, p, p]
        lib.m4ref_validate.restype = ctypes.c_int
        lib.m4ref_common.argtypes = [i64, p, p, i32, i32]
        lib.m4ref_common.restype = ctypes.c_int64
        for f in ("m4ref_orbits_brute", "m4ref_orbits_esu"):
            getattr(lib, f).argtypes = [i64, p, p, p]
            getattr(lib, f).restype = ctypes.c_int
        lib.m4ref_threads.argtypes = [ctypes.c_int]
        lib.m4ref_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, dtype=np.int32)
    return len(rp) - 1, rp, c


def _call(name, row_ptr, col):
    n, rp, c = _csr(row_ptr, col)
    out = np.zeros(6, dtype=np.uint64)
    rc = getattr(_load(), name)(n, rp.ctypes.data, c.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise OracleError(f"{name} failed with code {rc}")
    return tuple(int(x) for x in out)


def brute(row_ptr, col):
    return _call("m4ref_brute", row_ptr, col)


def esu(row_ptr, col):
    return _call("m4ref_esu", row_ptr, col)


def paper(row_ptr, col):
    return _call("m4ref_paper", row_ptr, col)


def closure(row_ptr, col, threads: int = 0, want_t: bool = False,
            want_basis: bool = False):
    """Plain closure counter.  Returns the six counts, plus the per-CSR-entry
    triangle counts and/or the non-induced basis dict when asked."""
    n, rp, c = _csr(row_ptr, col)
    out = np.zeros(6, dtype=np.uint64)
    t = np.zeros(max(int(rp[-1]), 1), dtype=np.uint32) if want_t else None
    basis = np.zeros(8, dtype=np.uint64)
    rc = _load().m4ref_closure(n, rp.ctypes.data, c.ctypes.data, threads,
                               out.ctypes.data,
                               t.ctypes.data if t is not None else None,
                               basis.ctypes.data)
    if rc != 0:
        raise OracleError(f"m4ref_closure failed with code {rc}")
    res = [tuple(int(x) for x in out)]
    if want_t:
        res.append(t[: int(rp[-1])])
    if want_basis:
        res.append({k: int(v) for k, v in zip(BASIS, basis)})
    return res[0] if len(res) == 1 else tuple(res)


ORBITS = tuple(range(4, 15))


def _orbits(name, row_ptr, col):
    n, rp, c = _csr(row_ptr, col)
    orb = np.zeros((max(n, 1), 11), dtype=np.uint64)
    rc = getattr(_load(), name)(n, rp.ctypes.data, c.ctypes.data, orb.ctypes.data)
    if rc != 0:
        raise OracleError(f"{name} failed with code {rc}")
    return orb[:n]


def orbits_brute(row_ptr, col):
    """uint64[n, 11]: column o - 4 holds, per vertex, the induced 4-sets in
    which it occupies graphlet orbit o (4..14), from every 4-vertex subset."""
    return _orbits("m4ref_orbits_brute", row_ptr, col)


def orbits_esu(row_ptr, col):
    """The same per-vertex orbit counts from the ESU enumeration of the
    connected 4-sets."""
    return _orbits("m4ref_orbits_esu", row_ptr, col)


def validate(row_ptr, col) -> bool:
    n, rp, c = _csr(row_ptr, col)
    return _load().m4ref_validate(n, rp.ctypes.data, c.ctypes.data) == 0


def common(row_ptr, col, u: int, v: int) -> int:
    n, rp, c = _csr(row_ptr, col)
    return int(_load().m4ref_common(n, rp.ctypes.data, c.ctypes.data, u, v))


def threads(req: int = 0) -> int:
    return int(_load().m4ref_threads(req))
