"""Python binding of libm4 -- exact connected induced 4-node motif counts on
AMD MI355X (gfx950).

Argument marshalling only: every step of the count runs in the HIP kernels
of ``libm4.so`` (``csrc/``), reached through its C ABI (``include/m4.h``).
There is no CPU fallback: if the library is missing or no GPU is present the
calls raise.  torch is used for device memory and streams only.

Counts are returned as Python ints in the order
``(3-star, 4-path, tailed triangle, 4-cycle, diamond, 4-clique)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libm4.so")

M4_OK, M4_EINVAL, M4_ERANGE, M4_EOVERFLOW, M4_ENOMEM, M4_EDEVICE, M4_EBUSY, M4_EINTERNAL = range(8)
M4_VALIDATE, M4_NO_CACHE, M4_FORCE_PARTITION, M4_STATS, M4_TIMING = 0x1, 0x2, 0x4, 0x8, 0x10
M4_PLAIN_LOOP = 0x20
M4_SERIAL = 0x40
M4_BASIS_WEDGE, M4_BASIS_EDGE = 0x80, 0x100
M4_NK = 16
KERNELS = ("build", "tri_global", "tri_1024", "tri_512", "tri_256", "tri_128", "tri_wave",
           "c4_plan", "c4_window", "c4_med", "c4_hash", "closure", "tri_hubs", "c4_desc",
           "c4_bin", "edge")
NAMES = ("star", "path", "paw", "cycle", "diamond", "clique")
BASIS = ("T", "K4", "C4_ni", "S", "P_ni", "Paw_ni", "D_ni", "sum_t")


class M4Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"m4 error {code}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("device_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("cache_rows", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p),
                ("tri_wave_max", ctypes.c_int32), ("c4_light_max", ctypes.c_int32),
                ("c4_med_max", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("basis", ctypes.c_uint64 * 8), ("intersect_steps", ctypes.c_uint64),
                ("wedges", ctypes.c_uint64), ("cache_lookups", ctypes.c_uint64),
                ("cache_hits", ctypes.c_uint64), ("partitions", ctypes.c_uint64),
                ("h2d_bytes", ctypes.c_uint64), ("halo_rows", ctypes.c_uint64),
                ("k_elems", ctypes.c_uint64 * M4_NK), ("k_rows", ctypes.c_uint64 * M4_NK),
                ("k_aux", ctypes.c_uint64 * M4_NK), ("k_aux2", ctypes.c_uint64 * M4_NK),
                ("ms_kernel", ctypes.c_double * M4_NK),
                ("ms_total", ctypes.c_double), ("ms_build", ctypes.c_double),
                ("ms_tri", ctypes.c_double), ("ms_c4", ctypes.c_double),
                ("ms_closure", ctypes.c_double), ("ms_h2d", ctypes.c_double),
                ("device_bytes", ctypes.c_uint64), ("ms_host", ctypes.c_double),
                ("basis_used", ctypes.c_uint32), ("cost_wedge", ctypes.c_double),
                ("cost_edge", ctypes.c_double)]

    def to_dict(self):
        d = {k: int(v) for k, v in zip(BASIS, self.basis)}
        for f, _ in self._fields_[1:]:
            v = getattr(self, f)
            d[f] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class Batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int64), ("voff", ctypes.c_void_p),
                ("eoff", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tri_wave_max", ctypes.c_int32), ("c4_light_max", ctypes.c_int32),
                ("batch_variant", ctypes.c_int32), ("batch_light", ctypes.c_int32),
                ("hub_min", ctypes.c_int32), ("c4_med_max", ctypes.c_int32),
                ("probe_w", ctypes.c_int32), ("c4_med_win", ctypes.c_int32),
                ("c4_bin_win", ctypes.c_int32), ("c4_bin_cap", ctypes.c_int32),
                ("c4_bin_dense", ctypes.c_int32), ("probe_w_far", ctypes.c_int32),
                ("tri_wave_far", ctypes.c_int32)]

    def to_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("counts", ctypes.c_uint64 * 6), ("t_submit_ms", ctypes.c_double),
                ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


_lib = None


def lib():
    """The loaded libm4.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname; loading it
        # first makes libm4 bind to that one runtime, so device pointers and
        # streams from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise M4Error(M4_EDEVICE, f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        p, i, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        L.m4_ctx_create.argtypes = [i, ctypes.POINTER(p)]
        L.m4_ctx_destroy.argtypes = [p]
        L.m4_ctx_destroy.restype = None
        L.m4_last_error.argtypes = [p]
        L.m4_last_error.restype = ctypes.c_char_p
        L.m4_ctx_device.argtypes = [p]
        L.m4_ctx_device.restype = ctypes.c_char_p
        L.m4_strerror.argtypes = [i]
        L.m4_strerror.restype = ctypes.c_char_p
        L.m4_count_motifs4.argtypes = [ctypes.POINTER(Csr), p]
        L.m4_count_motifs4_ex.argtypes = [p, ctypes.POINTER(Csr), ctypes.POINTER(Opts), p,
                                          ctypes.POINTER(Stats)]
        L.m4_edge_triangles.argtypes = [p, ctypes.POINTER(Csr), ctypes.POINTER(Opts), p]
        L.m4_count_orbits4.argtypes = [p, ctypes.POINTER(Csr), ctypes.POINTER(Opts), p]
        L.m4_count_motifs4_noalloc.argtypes = [p, ctypes.POINTER(Csr), ctypes.POINTER(Opts), p]
        L.m4_count_batch.argtypes = [p, ctypes.POINTER(Batch), ctypes.POINTER(Opts), p,
                                     ctypes.POINTER(Stats)]
        L.m4_get_tuning.argtypes = [p, ctypes.POINTER(Tuning)]
        L.m4_set_tuning.argtypes = [p, ctypes.POINTER(Tuning)]
        L.m4_autotune.argtypes = [p, ctypes.POINTER(Csr), ctypes.POINTER(Batch), i,
                                  ctypes.POINTER(Tuning)]
        L.m4_server_create.argtypes = [p, u64, i, ctypes.POINTER(p)]
        L.m4_server_submit.argtypes = [p, ctypes.POINTER(Csr), u64, ctypes.POINTER(u64)]
        L.m4_server_poll.argtypes = [p, ctypes.POINTER(Result), i, ctypes.POINTER(i)]
        L.m4_server_drain.argtypes = [p]
        L.m4_server_destroy.argtypes = [p]
        L.m4_server_destroy.restype = None
        L.m4_server_now_ms.argtypes = [p]
        L.m4_server_now_ms.restype = ctypes.c_double
        L.m4_plan_partitions.argtypes = [i, ctypes.c_int64, p, p, p, p, ctypes.c_int64, u64,
                                         ctypes.c_int64, ctypes.c_int64, p, p, p, p, p, p]
        _lib = L
    return _lib


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Keep:
    """Holds converted arrays alive for the duration of a call."""

    def __init__(self):
        self.refs = []


def make_csr(row_ptr, col, keep: _Keep) -> Csr:
    """Csr view of (row_ptr int64[n+1], col int32[nnz]): numpy arrays (host)
    or torch tensors (device when they live on a GPU)."""
    if _is_torch(row_ptr):
        import torch
        rp = row_ptr.to(torch.int64).contiguous()
        c = col.to(torch.int32).contiguous()
        keep.refs += [rp, c]
        on_dev = 1 if rp.is_cuda else 0
        if rp.is_cuda != c.is_cuda:
            raise ValueError("row_ptr and col must live on the same device")
        return Csr(rp.numel() - 1, c.numel(), rp.data_ptr(),
                   c.data_ptr() if c.numel() else None, on_dev)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    keep.refs += [rp, c]
    return Csr(len(rp) - 1, c.size, rp.ctypes.data, c.ctypes.data if c.size else None, 0)


def make_opts(flags=0, budget=0, cache_rows=0, stream=None, tri_wave_max=0, c4_light_max=0,
              c4_med_max=0) -> Opts:
    o = Opts()
    o.device_budget_bytes = int(budget)
    o.flags = int(flags)
    o.cache_rows = int(cache_rows)
    o.hip_stream = stream
    o.tri_wave_max = int(tri_wave_max)
    o.c4_light_max = int(c4_light_max)
    o.c4_med_max = int(c4_med_max)
    return o


class Context:
    """One device, one stream, a growable workspace (reused across calls)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = lib().m4_ctx_create(device, ctypes.byref(h))
        if rc != M4_OK:
            raise M4Error(rc, "m4_ctx_create: " + lib().m4_strerror(rc).decode())
        self.h = h
        self.device = device
        self.arch = lib().m4_ctx_device(h).decode()

    def close(self):
        if getattr(self, "h", None):
            lib().m4_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != M4_OK:
            raise M4Error(rc, lib().m4_last_error(self.h).decode())

    @staticmethod
    def _stream_for(x, stream):
        if stream is not None:
            return stream
        if _is_torch(x) and x.is_cuda:
            import torch
            return torch.cuda.current_stream(x.device).cuda_stream
        return None

    def count(self, row_ptr, col, *, flags=0, budget=0, cache_rows=0, stream=None,
              tri_wave_max=0, c4_light_max=0, c4_med_max=0, stats=False, timing=False):
        """Six counts; with stats=True (work counters) or timing=True (per
        kernel HIP-event times) also the m4_stats dict.  Threshold arguments
        of 0 keep the context's tuning (c4_med_max=-1: no medium bucket)."""
        keep = _Keep()
        g = make_csr(row_ptr, col, keep)
        fl = flags | (M4_STATS if stats else 0) | (M4_TIMING if timing else 0)
        o = make_opts(fl, budget, cache_rows, self._stream_for(row_ptr, stream), tri_wave_max,
                      c4_light_max, c4_med_max)
        out = (ctypes.c_uint64 * 6)()
        st = Stats()
        self._check(lib().m4_count_motifs4_ex(self.h, ctypes.byref(g), ctypes.byref(o),
                                              out, ctypes.byref(st)))
        counts = tuple(int(x) for x in out)
        return (counts, st.to_dict()) if (stats or timing) else counts

    def count_noalloc(self, row_ptr, col, *, flags=0, budget=0, stream=None):
        """The six counts through the allocation-free entry point (CSR in
        device memory, workspaces from the library's fixed device array)."""
        keep = _Keep()
        g = make_csr(row_ptr, col, keep)
        o = make_opts(flags, budget, 0, self._stream_for(row_ptr, stream))
        out = (ctypes.c_uint64 * 6)()
        self._check(lib().m4_count_motifs4_noalloc(self.h, ctypes.byref(g), ctypes.byref(o), out))
        return tuple(int(x) for x in out)

    def edge_triangles(self, row_ptr, col, *, flags=0, stream=None, tri_wave_max=0):
        """t_e for every CSR entry, in the input layout (numpy uint32 for host
        inputs, a torch int32 tensor holding uint32 bits for device inputs)."""
        keep = _Keep()
        g = make_csr(row_ptr, col, keep)
        o = make_opts(flags, 0, 0, self._stream_for(row_ptr, stream), tri_wave_max, 0)
        if g.on_device:
            import torch
            t = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=row_ptr.device)
            ptr = t.data_ptr()
        else:
            t = np.zeros(max(g.nnz, 1), dtype=np.uint32)
            ptr = t.ctypes.data
        self._check(lib().m4_edge_triangles(self.h, ctypes.byref(g), ctypes.byref(o), ptr))
        return t[: g.nnz]

    def orbits(self, row_ptr, col, *, flags=0, budget=0, stream=None):
        """Per-vertex graphlet orbit counts (orbits 4..14, column o - 4): numpy
        uint64 (n, 11) for host inputs, a torch int64 (n, 11) tensor holding
        uint64 bits for device inputs.  A device budget is rejected."""
        keep = _Keep()
        g = make_csr(row_ptr, col, keep)
        o = make_opts(flags, budget, 0, self._stream_for(row_ptr, stream))
        n = g.n
        if g.on_device:
            import torch
            out = torch.empty((max(n, 1), 11), dtype=torch.int64, device=row_ptr.device)
            ptr = out.data_ptr()
        else:
            out = np.zeros((max(n, 1), 11), dtype=np.uint64)
            ptr = out.ctypes.data
        self._check(lib().m4_count_orbits4(self.h, ctypes.byref(g), ctypes.byref(o), ptr))
        return out[:n]

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib().m4_get_tuning(self.h, ctypes.byref(t)))
        return t.to_dict()

    def set_tuning(self, **kw):
        t = Tuning()
        self._check(lib().m4_get_tuning(self.h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        self._check(lib().m4_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, graph=None, batch=None, reps=3, cache=None) -> dict:
        """Times the threshold candidates on a sample graph (row_ptr, col)
        and/or a packed arena (voff, eoff, row_ptr, col) and keeps the fastest
        in this context.  With cache (a JSON path) a result stored for the
        same device and sample size class is reused instead of re-timing."""
        import json
        key = None
        if cache is not None:
            key = self._tune_key(graph, batch)
            try:
                store = json.load(open(cache))
            except (OSError, ValueError):
                store = {}
            if key in store:
                self.set_tuning(**store[key])
                return dict(store[key], cached=True)
        keep = _Keep()
        g = make_csr(*graph, keep) if graph is not None else None
        b = self._make_batch(*batch, keep=keep) if batch is not None else None
        t = Tuning()
        self._check(lib().m4_autotune(self.h, ctypes.byref(g) if g is not None else None,
                                      ctypes.byref(b) if b is not None else None, int(reps),
                                      ctypes.byref(t)))
        res = t.to_dict()
        if cache is not None:
            try:
                store = json.load(open(cache))
            except (OSError, ValueError):
                store = {}
            store[key] = res
            with open(cache, "w") as fh:
                json.dump(store, fh, indent=1, sort_keys=True)
        return dict(res, cached=False)

    def _tune_key(self, graph, batch):
        import math
        parts = [self.arch]
        if graph is not None:
            n, nnz = len(graph[0]) - 1, len(graph[1])
            parts.append(f"g{int(math.log2(max(n, 1)))}.{int(math.log2(max(nnz, 1)))}")
        if batch is not None:
            G, nnz = len(batch[0]) - 1, int(batch[1][-1])
            parts.append(f"b{int(math.log2(max(G, 1)))}.{int(math.log2(max(nnz, 1)))}")
        return "/".join(parts)

    def _make_batch(self, voff, eoff, row_ptr, col, keep):
        if _is_torch(row_ptr):
            import torch
            arrs = [voff.to(torch.int64).contiguous(), eoff.to(torch.int64).contiguous(),
                    row_ptr.to(torch.int64).contiguous(), col.to(torch.int32).contiguous()]
            keep.refs += arrs
            return Batch(len(voff) - 1, *[a.data_ptr() for a in arrs],
                         1 if row_ptr.is_cuda else 0)
        arrs = [np.ascontiguousarray(voff, dtype=np.int64),
                np.ascontiguousarray(eoff, dtype=np.int64),
                np.ascontiguousarray(row_ptr, dtype=np.int64),
                np.ascontiguousarray(col, dtype=np.int32)]
        if arrs[3].size == 0:
            arrs[3] = np.zeros(1, dtype=np.int32)
        keep.refs += arrs
        return Batch(len(voff) - 1, *[a.ctypes.data for a in arrs], 0)

    def count_batch(self, voff, eoff, row_ptr, col, *, flags=0, stream=None, stats=False,
                    tri_wave_max=0, c4_light_max=0, plain=False):
        """Counts of every graph of a packed arena (see m4_batch in m4.h);
        returns a (G, 6) uint64 numpy array."""
        keep = _Keep()
        G = len(voff) - 1
        b = self._make_batch(voff, eoff, row_ptr, col, keep)
        if plain:
            flags |= M4_PLAIN_LOOP
        o = make_opts(flags | (M4_STATS if stats else 0), 0, 0,
                      self._stream_for(row_ptr, stream), tri_wave_max, c4_light_max)
        out = np.zeros((max(G, 1), 6), dtype=np.uint64)
        st = Stats()
        self._check(lib().m4_count_batch(self.h, ctypes.byref(b), ctypes.byref(o),
                                         out.ctypes.data, ctypes.byref(st)))
        return (out[:G], st.to_dict()) if stats else out[:G]


_default = None


def plan_partitions(kind, nptr, col, dlo, dplus, r1, cap_bytes, max_ranges=None,
                    max_rows=None):
    """Owner ranges of the host partition planner (``m4_plan_partitions``) on
    a rank-space CSR in host memory: kind 0 triangle ranges, 1 4-cycle
    ranges.  Returns (status, ends, rows) with rows[k] a list of (v, first,
    len) for range k."""
    n = len(nptr) - 1
    nptr = np.ascontiguousarray(nptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    dlo = np.ascontiguousarray(dlo, dtype=np.int32)
    dplus = np.ascontiguousarray(dplus, dtype=np.int32)
    mr = max_ranges if max_ranges is not None else n + 1
    mw = max_rows if max_rows is not None else (n + 1) * (n + 1)
    ends = np.zeros(max(mr, 1), np.int64)
    rr = np.zeros(max(mr, 1), np.int64)
    rv = np.zeros(max(mw, 1), np.int32)
    rf = np.zeros(max(mw, 1), np.int64)
    rl = np.zeros(max(mw, 1), np.int32)
    k = ctypes.c_int64(0)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib().m4_plan_partitions(int(kind), n, ptr(nptr), ptr(col), ptr(dlo), ptr(dplus),
                                  int(r1), int(cap_bytes), mr, mw, ptr(ends), ptr(rr), ptr(rv),
                                  ptr(rf), ptr(rl), ctypes.byref(k))
    rows, b = [], 0
    for j in range(k.value):
        e = int(rr[j])
        rows.append(list(zip(rv[b:e].tolist(), rf[b:e].tolist(), rl[b:e].tolist())))
        b = e
    return rc, ends[:k.value].tolist(), rows


def default_context() -> Context:
    global _default
    if _default is None:
        _default = Context(0)
    return _default


def count_motifs4(row_ptr, col, **kw):
    """Six induced 4-node motif counts of one graph on GPU 0."""
    return default_context().count(row_ptr, col, **kw)


def pack_batch(graphs):
    """Arena layout of m4_batch from a list of (row_ptr, col) host CSRs."""
    G = len(graphs)
    ns = np.array([len(rp) - 1 for rp, _ in graphs], dtype=np.int64)
    ms = np.array([len(c) for _, c in graphs], dtype=np.int64)
    voff = np.zeros(G + 1, dtype=np.int64)
    eoff = np.zeros(G + 1, dtype=np.int64)
    voff[1:] = np.cumsum(ns)
    eoff[1:] = np.cumsum(ms)
    row_ptr = np.concatenate([np.asarray(rp, dtype=np.int64) for rp, _ in graphs]) if G else \
        np.zeros(0, dtype=np.int64)
    col = np.concatenate([np.asarray(c, dtype=np.int32) for _, c in graphs]) if G else \
        np.zeros(0, dtype=np.int32)
    return voff, eoff, row_ptr, col


class Server:
    """Continuous-batching request loop on one device (m4_server_* C ABI).

    submit() copies a host CSR into the server and returns its id at once;
    poll() returns finished requests as dicts with the six counts and the
    submit / admit / done times (ms on the server clock)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_queue: int = 0):
        L = lib()
        L.m4_server_stats.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_uint64)] * 3
        h = ctypes.c_void_p()
        rc = L.m4_server_create(ctx.h, int(hbm_budget_bytes), int(max_queue), ctypes.byref(h))
        if rc != M4_OK:
            raise M4Error(rc, "m4_server_create: " + L.m4_strerror(rc).decode())
        self.h = h
        self.ctx = ctx

    def submit(self, row_ptr, col, tag: int = 0) -> int:
        keep = _Keep()
        g = make_csr(row_ptr, col, keep)
        rid = ctypes.c_uint64()
        rc = lib().m4_server_submit(self.h, ctypes.byref(g), int(tag), ctypes.byref(rid))
        if rc != M4_OK:
            raise M4Error(rc, "m4_server_submit: " + lib().m4_strerror(rc).decode())
        return rid.value

    def poll(self, max_results: int = 1024):
        res = (Result * max(max_results, 1))()
        got = ctypes.c_int()
        rc = lib().m4_server_poll(self.h, res, int(max_results), ctypes.byref(got))
        if rc != M4_OK:
            raise M4Error(rc, "m4_server_poll")
        return [{"id": r.id, "tag": r.tag, "status": r.status,
                 "counts": tuple(int(x) for x in r.counts), "t_submit_ms": r.t_submit_ms,
                 "t_admit_ms": r.t_admit_ms, "t_done_ms": r.t_done_ms}
                for r in res[: got.value]]

    def drain(self):
        lib().m4_server_drain(self.h)

    def now_ms(self) -> float:
        return lib().m4_server_now_ms(self.h)

    def stats(self):
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        lib().m4_server_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return {"max_inflight_bytes": a.value, "launches": b.value, "completed": c.value}

    def close(self):
        if getattr(self, "h", None):
            lib().m4_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
