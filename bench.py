#!/usr/bin/env python3
"""Benchmark of exact connected induced 4-node motif counting on one MI355X.

One step = one full count of the workload graph (CSR builder, triangle and
4-clique anchors, 4-cycle anchor, closure and exact inverse, 48-byte result
back to the host), with the input CSR already resident in HBM.  The headline
workload is the largest single-GPU configuration: a web-like R-MAT graph
(scale 24, edge factor 16, a,b,c,d = 0.45, 0.22, 0.22, 0.11, symmetrised and
deduplicated, 268 M undirected edges) generated from a fixed seed; its counts
are checked against values the CPU oracle computed for the same graph.

Prints ONE JSON line: throughput in edges/s (undirected edges / step time,
the triangle and 4-cycle stages overlapping on two streams), the roofline of
the dominant kernel (algorithmic bytes per launch over its HIP-event duration,
taken from further steps that run the stages one after the other so that a
kernel's events time it alone), the same graph under a 4 GB device budget
(halo partitions streamed from pinned host memory), the CPU oracle timed on
this host's cores, and secondary blocks: the per-vertex orbit counts of the
graph, the social R-MAT scale-20 graph (with its orbit counts), the batched
launch of 4096 uneven graphs and the serving loop.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edges/s for exact induced 4-motif counts; batched graphs/s vs plain; p99 ms"

# Workloads: (generator args, description)
WORKLOADS = {
    "web": dict(scale=24, edge_factor=16, abc=(0.45, 0.22, 0.22), seed=4,
                name="rmat-web", golden="rmat_web_s24.json"),
    "social": dict(scale=20, edge_factor=10, abc=(0.57, 0.19, 0.19), seed=2,
                   name="rmat-social", golden=None),
}

# Algorithmic bytes of one launch of each kernel slot: what the method must
# stream from HBM per unit of work, a function of the graph and the degree
# order only (not of this implementation), times the units that launch
# processed (work counters of m4_stats, include/m4.h):
#   triangle + 4-clique slots  4 E + 4 K + 8 R
#       E  out-list elements of the owners' out-neighbours (each oriented
#          edge u->v streams N+(v)), K  the owners' own out-list entries,
#       R  owners (one 8-byte row offset each); the 4-clique step works on
#          the frontier bitmaps the triangle step left in LDS and streams
#          nothing more
#   4-cycle slots (window, hash)  4 X + 8 S + 8 R
#       X  wedge endpoints (the prefix below the owner of each lower
#          neighbour's row), S  lower neighbours (row offset), R  owners
#   closure  12 m + 4 n  (per oriented edge its head, t_e and the head's
#          degree; per vertex its degree)
# Beside them each triangle slot reports the bytes it actually read from
# the lists and hub tables (k_aux2 4-byte words: hub-table probes replace
# longer scans, so a kernel may read fewer bytes than the algorithm streams).
TRI_SLOTS = {1: "tri_global", 2: "tri_1024", 3: "tri_512", 4: "tri_256", 5: "tri_128",
             6: "tri_wave"}
KERNEL_SYMBOL = {
    "tri_global": "k_tri_global", "tri_1024": "k_tri_lds<1024, 256>",
    "tri_512": "k_tri_lds<512, 256>", "tri_256": "k_tri_lds<256, 256>",
    "tri_128": "k_tri_lds<128, 256>", "tri_wave": "k_tri_lds<64, 64>",
    "c4_window": "k_c4_window", "c4_med": "k_c4_hash<1024, 16384, 4>",
    "c4_hash": "k_c4_hash<256, 4096, 4>", "closure": "k_closure", "c4_plan": "k_c4_plan",
    "build": "(CSR builder kernels)", "tri_hubs": "k_hub_insert", "c4_desc": "k_c4_desc",
    "c4_bin": "k_c4_bin",
}


def alg_bytes(slot: int, st: dict, n: int, m: int) -> float:
    E, R, A = st["k_elems"][slot], st["k_rows"][slot], st["k_aux"][slot]
    if slot in TRI_SLOTS:
        return 4.0 * E + 4.0 * A + 8.0 * R
    if slot in (8, 9, 10, 14):
        return 4.0 * E + 8.0 * A + 8.0 * R
    if slot == 11:
        return 12.0 * m + 4.0 * n
    return float("nan")


def read_bytes(slot: int, st: dict, n: int, m: int) -> float:
    """Bytes a triangle slot read from the lists and tables (plus its owners'
    own lists and offsets); the algorithmic bytes for every other slot."""
    if slot in TRI_SLOTS:
        return 4.0 * st["k_aux2"][slot] + 4.0 * st["k_aux"][slot] + 8.0 * st["k_rows"][slot]
    return alg_bytes(slot, st, n, m)


def source_digest() -> str:
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2607_12074_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:12]


def traffic_for(kernel: str, digest: str):
    """HBM bytes per launch measured with rocprofv3 PMC counters for this
    exact source (profiles/traffic.json); None if stale or absent."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(kernel)
    if not ent or rec.get("source_digest") != digest:
        return None
    return ent.get("bytes_per_launch")


def short_kernel_name(full: str) -> str:
    """'void m4::(anonymous namespace)::k_x<1, 2>(args)' -> 'k_x<1, 2>'."""
    s = full[5:] if full.startswith("void ") else full
    for pre in ("m4::(anonymous namespace)::", "m4::"):
        if s.startswith(pre):
            s = s[len(pre):]
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return s[:i]
    return s


def report_stats(path: str, top: int = 24) -> str:
    """Markdown table of a rocprofv3 --stats kernel summary (CSV)."""
    import csv
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short_kernel_name(r['Name'])}` | {r['Calls']} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def report_traffic(fetch_csv: str, write_csv: str, out_json: str) -> str:
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of `bench.py --copy-calib`, each scaled by
    the counter's reading for the 1 GiB device copy of that run; writes the
    record that traffic_for() reads and returns a markdown table."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                vals[short_kernel_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return vals

    f, w = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_kib = 1 << 20  # the calibration copy moves 1 GiB each way
    cf = [v for v in f.get("__amd_rocclr_copyBuffer", []) if v > copy_kib / 8]
    cw = [v for v in w.get("__amd_rocclr_copyBuffer", []) if v > copy_kib / 8]
    if not cf or not cw:
        raise SystemExit("no 1 GiB calibration copy in the PMC runs (run with --copy-calib)")
    ff, wf = copy_kib / (sum(cf) / len(cf)), copy_kib / (sum(cw) / len(cw))
    kernels = {}
    for k in sorted(set(f) & set(w)):
        if k == "__amd_rocclr_copyBuffer":
            continue
        fk, wk = sum(f[k]) / len(f[k]), sum(w[k]) / len(w[k])
        kernels[k] = {"dispatches": len(f[k]), "fetch_kib": fk, "write_kib": wk,
                      "bytes_per_launch": 1024.0 * (fk * ff + wk * wf)}
    rec = {"source_digest": source_digest(),
           "calibration": {"copy_bytes": 1 << 30, "fetch_factor": ff, "write_factor": wf},
           "kernels": kernels}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
        fh.write("\n")
    out = [f"Calibration: a 1 GiB device copy reads FETCH_SIZE x {ff:.3f} and "
           f"WRITE_SIZE x {wf:.3f} of its true bytes; source digest {rec['source_digest']}.", "",
           "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM bytes / launch (scaled) |",
           "|---|---|---|---|---|"]
    for k, e in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"])[:16]:
        out.append(f"| `{k}` | {e['dispatches']} | {e['fetch_kib']:.0f} | {e['write_kib']:.0f} | "
                   f"{e['bytes_per_launch']:.4g} |")
    return "\n".join(out)


def run_batch_leg(ctx, args):
    """Uneven batch: graphs/s of the persistent fused launch (hipGraph replay)
    against the plain one-graph-per-call loop, both on device-resident arenas
    and on the same stream; every graph's counts must agree."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_2607_12074_amd as m4

    G = args.batch_graphs
    t0 = time.perf_counter()
    graphs = [gg.batch_graph(i) for i in range(G)]
    arena = m4.pack_batch(graphs)
    gen_s = time.perf_counter() - t0
    dev = [torch.from_numpy(a).cuda() for a in arena]
    sum_m = int(arena[1][-1]) // 2
    # thresholds of the fused launch picked by the autotuner on a sample of
    # the same distribution (other seed), outside the timed region
    sample = m4.pack_batch([gg.batch_graph(i, seed=13) for i in range(512)])
    t0 = time.perf_counter()
    tuning = ctx.autotune(batch=sample, reps=2)
    tune_s = time.perf_counter() - t0
    out = ctx.count_batch(*dev)  # plan + capture
    for _ in range(2):
        ctx.count_batch(*dev)
    torch.cuda.synchronize()
    steps = max(args.steps, 1)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.count_batch(*dev)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = ctx.count_batch(*dev, plain=True)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) * 1e3
    return {"workload": f"{G} graphs, n log-uniform in [20, 5000], even G(n, m) with mean "
                        "degree U[3, 30], odd Barabasi-Albert m U{2..8}, seed 3",
            "graphs": G, "sum_m": sum_m, "ms_per_batch": ms_batch,
            "graphs_per_s": G / (ms_batch * 1e-3), "edges_per_s": sum_m / (ms_batch * 1e-3),
            "plain_ms": ms_plain, "plain_graphs_per_s": G / (ms_plain * 1e-3),
            "speedup_vs_plain": ms_plain / ms_batch,
            "plain_equal": bool(np.array_equal(plain, out)), "gen_s": round(gen_s, 2),
            "tuning": {k: tuning[k] for k in ("batch_variant", "batch_light")},
            "tune_s": round(tune_s, 2)}


def run_serve_leg(ctx, args):
    """Serving: requests with n log-normal (median 5000, sigma 1.5, cap 2M),
    half Chung-Lu power law, half random geometric.  After W warm-up requests
    a closed loop (all R measured requests submitted at once) gives the
    saturation rate; then a Poisson stream of the same R requests at 0.7 of
    it is replayed and p50/p99 latency (done - submit) and graphs/s are
    reported.  Both runs must return identical counts."""
    import numpy as np
    import graphgen as gg
    import paper_2607_12074_amd as m4

    W, R = args.serve_warmup, args.serve_requests
    t0 = time.perf_counter()
    graphs = [gg.serve_graph(i) for i in range(W + R)]
    gen_s = time.perf_counter() - t0
    warm, graphs = graphs[:W], graphs[W:]
    budget = int(args.serve_budget_gb * (1 << 30))

    def collect(srv, ids, limit_s=300.0):
        got = {}
        t_end = time.perf_counter() + limit_s
        while len(got) < len(ids):
            for r in srv.poll(4096):
                got[r["id"]] = r
            if time.perf_counter() > t_end:
                raise TimeoutError(f"serving leg: {len(got)} of {len(ids)} results")
            time.sleep(0.0002)
        return [got[i] for i in ids]

    srv = m4.Server(ctx, budget)
    for g in warm:
        srv.submit(*g)
    srv.drain()
    srv.poll(1 << 16)
    t0 = time.perf_counter()
    ids = [srv.submit(*g, tag=i) for i, g in enumerate(graphs)]
    closed = collect(srv, ids)
    sat = R / (time.perf_counter() - t0)
    note(f"serving closed loop: {sat:.1f} graphs/s")
    rate = 0.7 * sat
    gaps = np.random.default_rng(7).exponential(1.0 / rate, R)
    ids = []
    t_next = time.perf_counter()
    for i, g in enumerate(graphs):
        t_next += gaps[i]
        while time.perf_counter() < t_next:
            pass
        ids.append(srv.submit(*g, tag=i))
    opened = collect(srv, ids)
    st = srv.stats()
    srv.close()
    lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in opened])
    span = max(r["t_done_ms"] for r in opened) - min(r["t_submit_ms"] for r in opened)
    same = all(a["counts"] == b["counts"] and a["status"] == 0 == b["status"]
               for a, b in zip(closed, opened))
    ns = np.array([len(g[0]) - 1 for g in graphs])
    out = {"workload": f"{W} warm-up + {R} measured requests, n log-normal median 5000 sigma "
                       "1.5 cap 2M, even Chung-Lu exponent U[2.1,2.8], odd random geometric, "
                       "mean degree U[6,12], seed 5",
           "requests": R, "warmup_requests": W, "n_p50": int(np.median(ns)),
           "n_max": int(ns.max()), "saturation_graphs_per_s": sat, "offered_rate": rate,
           "graphs_per_s": R / (span * 1e-3), "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "budget_bytes": budget,
           "mix_equals_closed_loop": bool(same), "gen_s": round(gen_s, 2)}
    out.update({k: v for k, v in st.items()})
    return out


def note(msg):
    """One progress line per finished stage, on stderr."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def workload_desc(w: dict) -> str:
    a, b, c = w["abc"]
    return (f"{w['name']} scale {w['scale']} edge-factor {w['edge_factor']} "
            f"(a,b,c,d)=({a},{b},{c},{round(1 - a - b - c, 2)}) seed {w['seed']}, "
            "symmetrised and deduplicated")


def make_graph(w: dict):
    import graphgen as gg
    t0 = time.perf_counter()
    rp, col = gg.rmat(w["scale"], w["edge_factor"], *w["abc"], w["seed"], True)
    return rp, col, time.perf_counter() - t0


def golden_counts(w: dict, n: int, m: int):
    """Counts the CPU oracle computed for this exact graph (tests/golden/,
    written by tests/golden/make_golden.py), or None."""
    if not w.get("golden"):
        return None
    try:
        rec = json.load(open(os.path.join(ROOT, "tests", "golden", w["golden"])))
    except (OSError, ValueError):
        return None
    if rec.get("n") != n or rec.get("m") != m:
        return None
    return tuple(rec["counts"]), rec.get("basis")


def copy_rate_gbps(dev) -> float:
    """Achievable HBM rate on this machine: a plain 1 GiB device copy, HIP events."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9


def run_graph_leg(ctx, rp, col, args, steps, warmup, serial_flag):
    """Timed steps on a device-resident CSR, per-kernel HIP-event times from
    steps with the stages serial, work counters and the roofline of the
    dominant kernel."""
    import numpy as np
    import torch
    import paper_2607_12074_amd as m4

    n, m = len(rp) - 1, len(col) // 2
    dev = torch.device("cuda:0")
    rp_d = torch.from_numpy(rp).to(dev)
    col_d = torch.from_numpy(col).to(dev)
    torch.cuda.synchronize()
    step_flags = m4.M4_SERIAL if serial_flag else 0
    counts = None
    for _ in range(warmup):
        counts = ctx.count(rp_d, col_d, flags=step_flags)
    torch.cuda.synchronize()
    # timed region: K full counts (each ends with its 48-byte result on the
    # host, so the per-step wall times are complete counts)
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        counts = ctx.count(rp_d, col_d, flags=step_flags)
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    note(f"timed {steps} steps: {ms_step:.3f} ms/step")
    # kernel durations: more counts with the stages on one stream, so that
    # each kernel's HIP events (recorded on its launch stream) time it alone
    ms_k = np.zeros(m4.M4_NK)
    t0 = time.perf_counter()
    ksteps = max(1, min(steps, 5))
    for _ in range(ksteps):
        c_k, tst = ctx.count(rp_d, col_d, flags=m4.M4_SERIAL, timing=True)
        assert c_k == counts
        ms_k += np.array(tst["ms_kernel"])
    torch.cuda.synchronize()
    ms_step_serial = (time.perf_counter() - t0) * 1e3 / ksteps
    ms_k /= ksteps
    note(f"kernel timing steps (stages serial, HIP events): {ms_step_serial:.3f} ms/step")
    counts2, st = ctx.count(rp_d, col_d, flags=step_flags, stats=True)
    assert counts2 == counts
    del rp_d, col_d
    torch.cuda.empty_cache()
    names = m4.KERNELS
    dom = int(np.argmax(ms_k[1:len(names)])) + 1  # dominant kernel (not the builder group)
    dname = names[dom]
    B = alg_bytes(dom, st, n, m)
    achieved = B / (ms_k[dom] * 1e-3) / 1e9 if ms_k[dom] > 0 else 0.0
    kernels = {}
    for i in range(len(names)):
        if ms_k[i] <= 0:
            continue
        ab, rb = alg_bytes(i, st, n, m), read_bytes(i, st, n, m)
        kernels[names[i]] = {
            "ms": round(float(ms_k[i]), 4), "elems": st["k_elems"][i], "rows": st["k_rows"][i],
            "aux": st["k_aux"][i], "aux2": st["k_aux2"][i],
            "alg_GBps": round(ab / (ms_k[i] * 1e6), 1) if i > 0 and ab == ab else None,
            "read_GBps": round(rb / (ms_k[i] * 1e6), 1) if i > 0 and rb == rb else None}
    return {
        "n": n, "m": m, "counts": tuple(counts), "ms_step": ms_step,
        "ms_median": float(np.median(step_ms)), "ms_min": float(np.min(step_ms)),
        "ms_serial": ms_step_serial, "stats": st, "ms_k": ms_k, "dom": dom, "dname": dname,
        "alg_bytes": B, "achieved": achieved, "kernels": kernels,
        "work": {"intersect_steps": st["intersect_steps"], "wedges": st["wedges"],
                 "cache_lookups": st["cache_lookups"], "cache_hits": st["cache_hits"],
                 "intersection_work_per_edge": (st["intersect_steps"] + st["wedges"]) / m},
        "device_bytes": st["device_bytes"],
    }


def run_budget_leg(ctx, rp, col, budget_gb, resident_counts):
    """The same graph under a device budget: halo partitions streamed from
    pinned host memory.  Counts must equal the resident run bit for bit."""
    import paper_2607_12074_amd as m4
    budget = int(budget_gb * (1 << 30))
    t0 = time.perf_counter()
    counts, st = ctx.count(rp, col, budget=budget, stats=True)
    wall = time.perf_counter() - t0
    n, m = len(rp) - 1, len(col) // 2
    ms = st["ms_total"]
    return {"budget_bytes": budget, "ms": ms, "wall_s": round(wall, 3),
            "edges_per_s": m / (ms * 1e-3), "partitions": st["partitions"],
            "h2d_bytes": st["h2d_bytes"], "ms_h2d": st["ms_h2d"],
            "transfer_fraction": st["ms_h2d"] / ms if ms > 0 else None,
            "halo_rows": st["halo_rows"],
            "halo_amplification": st["halo_rows"] / n,
            "h2d_over_csr": st["h2d_bytes"] / (8.0 * (n + 1) + 8.0 * m),
            "device_bytes": st["device_bytes"],
            "ms_phases": {"order_and_rows": st["ms_build"], "triangles": st["ms_tri"],
                          "four_cycles": st["ms_c4"], "closure": st["ms_closure"],
                          "host_planning_and_gathers": st["ms_host"]},
            "equal_to_resident": tuple(counts) == tuple(resident_counts),
            "note": "host CSR in, counts out; the partition plan, halo gathers and "
                    "uploads are inside the time"}


def run_orbits_leg(ctx, rp, col, counts, reps: int):
    """Per-vertex orbit counts (orbits 4..14) of the resident graph: one
    untimed call, then reps timed calls; the orbit totals must give the six
    counts of the resident count."""
    import numpy as np
    import torch
    rpd, cold = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    out = ctx.orbits(rpd, cold)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = ctx.orbits(rpd, cold)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    c = out.sum(dim=0).cpu().numpy().view(np.uint64)
    tot = (int(c[3]), int(c[1]) // 2, int(c[7]), int(c[4]) // 4, int(c[9]) // 2, int(c[10]) // 4)
    m = len(col) // 2
    ms = float(np.median(ts))
    del rpd, cold, out
    torch.cuda.empty_cache()
    return {"ms": ms, "ms_min": min(ts), "reps": reps, "edges_per_s": m / (ms * 1e-3),
            "totals_equal_counts": tot == tuple(counts),
            "note": "uint64[n][11] per-vertex orbit counts, CSR resident, output on the device"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def run_cpu_leg(w: dict, args):
    """The CPU oracle (plain closure counter) on a bounded sample of the
    headline workload: the same generator and parameters at a smaller scale,
    on every host thread and on one; and the ESU enumeration on the
    2000-vertex ER graph, single-threaded."""
    import graphgen as gg
    import oracle
    a, b, c = w["abc"]
    out = {}
    sc = args.cpu_scale
    rp, col = gg.rmat(sc, w["edge_factor"], a, b, c, w["seed"], True)
    m = len(col) // 2
    t0 = time.perf_counter()
    oracle.closure(rp, col, threads=0)
    t_all = time.perf_counter() - t0
    threads = oracle.threads(0)
    sc1 = sc - 3
    rp1, col1 = gg.rmat(sc1, w["edge_factor"], a, b, c, w["seed"], True)
    m1 = len(col1) // 2
    t0 = time.perf_counter()
    oracle.closure(rp1, col1, threads=1)
    t_one = time.perf_counter() - t0
    rpe, cole = gg.er_c1(seed=1)
    t0 = time.perf_counter()
    oracle.esu(rpe, cole)
    t_esu = time.perf_counter() - t0
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    out = {"value": m / t_all, "unit": "edges/s", "cores": threads, "kind": "oracle",
           "sample": f"{w['name']} scale {sc} edge-factor {w['edge_factor']} (same generator, "
                     f"parameters and seed as the workload, m={m}), plain closure counter on "
                     f"{threads} threads, {t_all:.1f} s",
           "nproc": nproc, "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
           "one_core": {"value": m1 / t_one, "unit": "edges/s",
                        "sample": f"scale {sc1} (m={m1}), 1 thread, {t_one:.1f} s"},
           "esu_c1": {"seconds": round(t_esu, 3), "threads": 1,
                      "sample": "ESU enumeration of the connected 4-sets of G(n=2000, "
                                "m=20000), seed 1"}}
    note(f"cpu oracle: {threads} threads {t_all:.1f} s (scale {sc}), 1 thread {t_one:.1f} s, "
         f"ESU {t_esu:.1f} s")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="web")
    ap.add_argument("--scale", type=int, default=0, help="override the workload's scale")
    ap.add_argument("--budget-gb", type=float, default=4.0,
                    help="device budget of the partitioned leg (0 = skip it)")
    ap.add_argument("--no-social", action="store_true",
                    help="skip the secondary social R-MAT scale-20 block")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--orbit-reps", type=int, default=2,
                    help="timed per-vertex orbit calls on each graph (0: skip that leg)")
    ap.add_argument("--cpu-scale", type=int, default=21,
                    help="scale of the CPU oracle's sample of the workload family")
    ap.add_argument("--batch-graphs", type=int, default=4096,
                    help="graphs of the uneven batch (0 = skip the batched leg)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="measured requests of the serving leg (0 = skip it)")
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-budget-gb", type=float, default=2.0)
    ap.add_argument("--serial", action="store_true",
                    help="timed steps with the anchor stages on one stream (no overlap)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the single-graph thresholds on the workload first")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (PMC calibration)")
    ap.add_argument("--report-stats", metavar="CSV",
                    help="print a markdown table of a rocprofv3 kernel-stats CSV and exit")
    ap.add_argument("--report-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two PMC runs and exit")
    args = ap.parse_args()
    if args.report_stats:
        print(report_stats(args.report_stats))
        return
    if args.report_traffic:
        print(report_traffic(*args.report_traffic, os.path.join(ROOT, "profiles", "traffic.json")))
        return
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (--gpus 1); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_12074_amd as m4

    w = dict(WORKLOADS[args.workload])
    if args.scale:
        w["scale"] = args.scale
    rp, col, gen_s = make_graph(w)
    n, m = len(rp) - 1, len(col) // 2
    note(f"workload {w['name']} n={n} m={m} generated in {gen_s:.1f} s")
    dev = torch.device("cuda:0")
    ctx = m4.Context(0)

    # single-graph thresholds: the library defaults (picked from MI355X
    # sweeps), or with --tune the autotuner's choice on the workload graph,
    # outside the timed region
    if args.tune:
        t0 = time.perf_counter()
        tuned = ctx.autotune(graph=(rp, col), reps=2)
        note(f"single-graph tuning {tuned} in {time.perf_counter() - t0:.2f} s")
    graph_tuning = dict(ctx.get_tuning(), autotuned=bool(args.tune))

    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    main_leg = run_graph_leg(ctx, rp, col, args, args.steps, args.warmup, args.serial)
    counts = main_leg["counts"]
    gold = golden_counts(w, n, m)
    parity = None if gold is None else (tuple(gold[0]) == tuple(counts))
    note(f"parity vs the oracle's stored counts: {parity}")

    # outside the timed region: the same count from host arrays (the CSR
    # copied over PCIe in the call) and the achievable HBM rate on this machine
    ts = time.perf_counter()
    c_h = ctx.count(rp, col, flags=m4.M4_SERIAL if args.serial else 0)
    ms_host = (time.perf_counter() - ts) * 1e3
    assert c_h == counts
    copy_gbps = copy_rate_gbps(dev)

    budget = None
    if args.budget_gb > 0:
        budget = run_budget_leg(ctx, rp, col, args.budget_gb, counts)
        note(f"budget leg ({args.budget_gb} GB): {budget['ms'] / 1e3:.2f} s, "
             f"{budget['partitions']} partitions, equal {budget['equal_to_resident']}, "
             "phases ms " + ", ".join(f"{k} {v:.0f}" for k, v in budget["ms_phases"].items()))

    orbits = None
    if args.orbit_reps > 0:
        orbits = run_orbits_leg(ctx, rp, col, counts, args.orbit_reps)
        note(f"orbits leg: {orbits['ms']:.1f} ms, totals equal {orbits['totals_equal_counts']}")

    digest = source_digest()
    dname = main_leg["dname"]
    traffic = traffic_for(KERNEL_SYMBOL[dname], digest)

    cpu = None
    if not args.no_cpu:
        cpu = run_cpu_leg(w, args)

    social = None
    if not args.no_social and args.workload != "social":
        import oracle
        ws = WORKLOADS["social"]
        rps, cols, gs = make_graph(ws)
        leg = run_graph_leg(ctx, rps, cols, args, args.steps, args.warmup, args.serial)
        ref = None if args.no_cpu else oracle.closure(rps, cols, threads=0)
        social = {"workload": workload_desc(ws), "n": leg["n"], "m": leg["m"],
                  "value": leg["m"] / (leg["ms_step"] * 1e-3), "ms_per_step": leg["ms_step"],
                  "ms_per_step_median": leg["ms_median"], "ms_per_step_min": leg["ms_min"],
                  "ms_per_step_stages_serial": leg["ms_serial"], "counts": list(leg["counts"]),
                  "parity_vs_oracle": None if ref is None else tuple(ref) == leg["counts"],
                  "roofline": {"bound": "hbm", "kernel": KERNEL_SYMBOL[leg["dname"]],
                               "achieved": leg["achieved"], "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": leg["achieved"] / HBM_PEAK_GBS,
                               "alg_bytes": leg["alg_bytes"],
                               "ms": float(leg["ms_k"][leg["dom"]])},
                  "kernels": leg["kernels"], "work": leg["work"]}
        if args.orbit_reps > 0:
            social["orbits"] = run_orbits_leg(ctx, rps, cols, leg["counts"], args.orbit_reps)
        note(f"social block: {social['value']:.3g} edges/s, parity {social['parity_vs_oracle']}")

    batched = run_batch_leg(ctx, args) if args.batch_graphs > 0 else None
    if batched:
        note(f"batched leg: {batched['graphs_per_s']:.0f} graphs/s, "
             f"{batched['speedup_vs_plain']:.2f}x plain")
    serving = run_serve_leg(ctx, args) if args.serve_requests > 0 else None
    if serving:
        note(f"serving leg: p99 {serving['p99_ms']:.2f} ms")

    B, achieved = main_leg["alg_bytes"], main_leg["achieved"]
    line = {
        "metric": METRIC,
        "value": m / (main_leg["ms_step"] * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_step"],
        "ms_per_step_median": main_leg["ms_median"],
        "ms_per_step_min": main_leg["ms_min"],
        "ms_per_step_stages_serial": main_leg["ms_serial"],
        "pcie_inclusive": {"ms": ms_host, "edges_per_s": m / (ms_host * 1e-3),
                           "note": "host CSR copied to the device inside the call"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": workload_desc(w), "n": n, "m": m,
                   "parallelism": "single-gpu", "tuning": graph_tuning},
        "counts": list(counts),
        "parity_vs_oracle": parity,
        "parity_source": "tests/golden/" + w["golden"] if w.get("golden") else None,
        "roofline": {"bound": "hbm", "kernel": KERNEL_SYMBOL[dname], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes": B,
                     "ms": float(main_leg["ms_k"][main_leg["dom"]]),
                     "measured_copy_GBps": copy_gbps},
        "kernels": main_leg["kernels"],
        "work": main_leg["work"],
        "device_bytes": main_leg["device_bytes"],
        "budget": budget,
        "orbits": orbits,
        "cpu_baseline": cpu,
        "social": social,
        "batched": batched,
        "serving": serving,
        "source_digest": digest,
        "gen_s": round(gen_s, 2),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
