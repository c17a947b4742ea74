"""Seeded synthetic graph generators (inputs shared by the counter and its oracle).

The generators live in ``m4gen.c`` (plain C, OpenMP) and are reached through
ctypes.  Every function returns ``(row_ptr, col)``: a symmetric CSR with
``row_ptr`` int64[n+1] and ``col`` int32[nnz], rows strictly increasing, no
self-loops and no duplicate edges.  No motif arithmetic lives here.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "m4gen.c")
_LIB = os.path.join(_HERE, "libm4gen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libm4gen.so in place with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall", _SRC,
               "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32))]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        G = ctypes.POINTER(_Graph)
        i64, u64, dbl, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        lib.m4gen_uniform.argtypes = [u64, u64, u64]
        lib.m4gen_uniform.restype = dbl
        lib.m4gen_gnm.argtypes = [i64, i64, u64, G]
        lib.m4gen_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, i32, G]
        lib.m4gen_ba.argtypes = [i64, i32, u64, G]
        lib.m4gen_chunglu.argtypes = [i64, dbl, dbl, u64, G]
        lib.m4gen_rgg.argtypes = [i64, dbl, u64, G]
        lib.m4gen_from_edges.argtypes = [i64, i64, ctypes.c_void_p, ctypes.c_void_p, G]
        lib.m4gen_free.argtypes = [G]
        for f in ("m4gen_gnm", "m4gen_rmat", "m4gen_ba", "m4gen_chunglu",
                  "m4gen_rgg", "m4gen_from_edges"):
            getattr(lib, f).restype = ctypes.c_int
        lib.m4gen_free.restype = None
        _lib = lib
    return _lib


def _take(rc: int, g: _Graph):
    lib = _load()
    if rc != 0:
        raise ValueError(f"graph generator failed with code {rc}")
    try:
        n, nnz = g.n, g.nnz
        rp = np.ctypeslib.as_array(g.row_ptr, shape=(n + 1,)).copy()
        col = (np.ctypeslib.as_array(g.col, shape=(nnz,)).copy() if nnz > 0
               else np.zeros(0, dtype=np.int32))
    finally:
        lib.m4gen_free(ctypes.byref(g))
    return rp, col


def uniform(seed: int, stream: int, ctr: int) -> float:
    """Counter-based uniform draw in [0, 1)."""
    return _load().m4gen_uniform(seed & (2**64 - 1), stream & (2**64 - 1), ctr)


def gnm(n: int, m: int, seed: int):
    g = _Graph()
    return _take(_load().m4gen_gnm(n, m, seed, ctypes.byref(g)), g)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         permute: bool = True):
    g = _Graph()
    return _take(_load().m4gen_rmat(scale, edge_factor, a, b, c, seed,
                                    1 if permute else 0, ctypes.byref(g)), g)


def ba(n: int, m_ba: int, seed: int):
    g = _Graph()
    return _take(_load().m4gen_ba(n, m_ba, seed, ctypes.byref(g)), g)


def chunglu(n: int, beta: float, mean_deg: float, seed: int):
    g = _Graph()
    return _take(_load().m4gen_chunglu(n, beta, mean_deg, seed, ctypes.byref(g)), g)


def rgg(n: int, mean_deg: float, seed: int):
    g = _Graph()
    return _take(_load().m4gen_rgg(n, mean_deg, seed, ctypes.byref(g)), g)


def from_edges(n: int, src, dst):
    """Symmetric simple CSR from an edge list (loops and duplicates removed)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    g = _Graph()
    return _take(_load().m4gen_from_edges(n, src.size, src.ctypes.data,
                                          dst.ctypes.data, ctypes.byref(g)), g)


# ----------------------------------------------------------- workload recipes

def er_c1(seed: int = 1):
    """Uniform G(n=2000, m=20000)."""
    return gnm(2000, 20000, seed)


def rmat_social(scale: int = 20, edge_factor: int = 10, seed: int = 2):
    """Social-like R-MAT (a, b, c, d) = (0.57, 0.19, 0.19, 0.05)."""
    return rmat(scale, edge_factor, 0.57, 0.19, 0.19, seed, True)


def rmat_web(scale: int = 24, edge_factor: int = 16, seed: int = 4):
    """Web-like R-MAT (a, b, c, d) = (0.45, 0.22, 0.22, 0.11)."""
    return rmat(scale, edge_factor, 0.45, 0.22, 0.22, seed, True)


_STREAM_BATCH = 0x6261746368
_STREAM_SERVE = 0x7365727665


def batch_spec(index: int, seed: int = 3, n_lo: int = 20, n_hi: int = 5000):
    """Parameters of graph `index` of the uneven batch: n log-uniform in
    [n_lo, n_hi]; even indices G(n, round(n k / 2)) with k ~ U[3, 30], odd
    indices Barabasi-Albert with m ~ U{2..8}."""
    u0 = uniform(seed, _STREAM_BATCH, 4 * index)
    u1 = uniform(seed, _STREAM_BATCH, 4 * index + 1)
    n = int(round(math.exp(math.log(n_lo) + u0 * (math.log(n_hi) - math.log(n_lo)))))
    gseed = (seed * 1000003 + index) & (2**63 - 1)
    if index % 2 == 0:
        k = 3.0 + 27.0 * u1
        m = min(int(round(n * k / 2.0)), n * (n - 1) // 2)
        return ("gnm", n, m, gseed)
    m_ba = 2 + min(6, int(u1 * 7.0))
    return ("ba", n, m_ba, gseed)


def batch_graph(index: int, seed: int = 3, n_lo: int = 20, n_hi: int = 5000):
    kind, n, p, gseed = batch_spec(index, seed, n_lo, n_hi)
    return gnm(n, p, gseed) if kind == "gnm" else ba(n, p, gseed)


def serve_spec(index: int, seed: int = 5, median: float = 5000.0,
               sigma: float = 1.5, cap: int = 2_000_000):
    """Parameters of serving request `index`: n log-normal (median, sigma),
    capped; even indices Chung-Lu with exponent U[2.1, 2.8], odd indices a
    random geometric graph; mean degree U[6, 12]."""
    u0 = uniform(seed, _STREAM_SERVE, 4 * index)
    u1 = uniform(seed, _STREAM_SERVE, 4 * index + 1)
    u2 = uniform(seed, _STREAM_SERVE, 4 * index + 2)
    u3 = uniform(seed, _STREAM_SERVE, 4 * index + 3)
    # Box-Muller from two counter draws
    z = math.sqrt(-2.0 * math.log(max(u0, 1e-300))) * math.cos(2.0 * math.pi * u1)
    n = int(min(cap, max(8, round(median * math.exp(sigma * z)))))
    k = 6.0 + 6.0 * u2
    gseed = (seed * 1000033 + index) & (2**63 - 1)
    if index % 2 == 0:
        return ("chunglu", n, (2.1 + 0.7 * u3, k), gseed)
    return ("rgg", n, (k,), gseed)


def serve_graph(index: int, seed: int = 5, **kw):
    kind, n, p, gseed = serve_spec(index, seed, **kw)
    if kind == "chunglu":
        return chunglu(n, p[0], p[1], gseed)
    return rgg(n, p[0], gseed)
