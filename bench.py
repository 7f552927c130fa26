"""Benchmark: edges/s to h-trussness on one MI355X.

A step is one full decomposition (every edge's h-trussness) of a synthetic
graph whose CSR is already resident in HBM.  Default workload: R-MAT scale 18
(262,144 vertices, edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05), seed 1),
symmetrised and deduplicated, h = 2.  `value` is m * K / wall time of the K
timed decompositions; the line also carries each decomposition's device time
(HIP events from its first kernel to its completion event) as median, min and
max.  Other single-graph workloads: chung_lu_100k_h2, rmat18_h3,
chung_lu_100k_h1, er200_h2.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Two more workloads measure the multi-graph forms:
  --workload batched   512 preferential-attachment graphs with planted
                       cliques (n ~ U[1000, 50000], h in {2, 3}) in one
                       batched call; graphs/s against a loop of single-graph
                       calls on one stream and on four streams, results
                       compared bit for bit
  --workload serve     a Poisson stream of Chung-Lu requests over size classes
                       through a session with a device-memory budget;
                       p50/p99 latency and graphs/s at fixed fractions of the
                       measured capacity

  --workload hindex    the H-index fixpoint method (Section 4) on the default
                       Chung-Lu graph: synchronous sweeps timed, asynchronous
                       and recompute-everything sweeps and the peeling method
                       once each, all outputs compared bit for bit
  --workload hindex_iterations
                       sweeps to convergence of the synchronous and the
                       asynchronous H-index iteration on several graphs

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

import numpy as np  # noqa: E402

from graphgen import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    "chung_lu_100k_h2": (lambda: W.d2(), 2,
                         "Chung-Lu n=100000 avg_deg=10 gamma=2.5 seed=1, h=2"),
    "rmat18_h2": (lambda: W.d3(), 2, "R-MAT scale 18 ef 16 (0.57,0.19,0.19,0.05) seed=1, h=2"),
    "rmat18_h3": (lambda: W.d3(), 3, "R-MAT scale 18 ef 16 (0.57,0.19,0.19,0.05) seed=1, h=3"),
    "er200_h2": (lambda: W.d1(0), 2, "Erdos-Renyi G(200,0.05) seed=0, h=2"),
    "chung_lu_100k_h1": (lambda: W.d2(), 1,
                         "Chung-Lu n=100000 avg_deg=10 gamma=2.5 seed=1, h=1 (classical truss)"),
}

CPU_SAMPLE_N = 6000  # Chung-Lu sample the oracle decomposes completely (about 10-30 s)

# Algorithmic bytes per unit of work of the two chunked round kernels (each
# access counted at its natural size, not as cache lines):
#   ball-change events: work item 16 B; examined slot 8 B (srem, col_idx);
#     tested pair 32 B (ball bit word, two row extents, (j-1)-ball word);
#     witness probe 16 B (srem, col_idx, ball word); dropped pair 48 B (two
#     ball-bit atomics, change-mark atomic, event record, follow-up items)
#   support update: work item 16 B; adjacency slot 20 B (the packed
#     neighbour and edge id word, the event target's ball word, and its
#     change-mark word for the half of the slots whose source is the smaller
#     endpoint); lost common neighbour 8 B (support atomic)
LEVEL_BYTES = {"level_items": 16, "level_slots": 8, "level_candidates": 32,
               "level_probes": 16, "level_drops": 48}
SUPPORT_BYTES = {"support_items": 16, "support_slots": 20, "support_hits": 8}
KERNEL_SYMBOL = {"level_events": "k_level", "support_update": "k_support"}
PROFILES = ROOT / "profiles"


def kernel_source_sha(kernel: str) -> str:
    from paper_2411_06405_amd.profsum import KERNEL_SOURCES, source_sha
    return source_sha(KERNEL_SOURCES[kernel])


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current source of that kernel."""
    tfile = PROFILES / f"traffic_{kernel}_{workload}.txt"
    if tfile.exists():
        t = json.loads(tfile.read_text())
        if t.get("source_sha") == kernel_source_sha(kernel):
            return t.get("bytes_per_launch")
    return None


def recorded_whole_traffic(workload: str):
    """HBM bytes of one whole decomposition (every library kernel, scaled
    counters) from the committed summary, if taken on the current kernels."""
    tfile = PROFILES / f"traffic_whole_{workload}.txt"
    if tfile.exists():
        t = json.loads(tfile.read_text())
        if t.get("source_sha") == kernel_source_sha("k_level"):
            return t.get("bytes_per_decomposition")
    return None


def whole_run(st: dict, workload: str, device_ms: float):
    """The whole decomposition against the HBM roofline and the method-level
    count: (i) counter bytes / device time / 8 TB/s, (ii) counter bytes /
    B_alg (below 1: the incremental kernels move less than re-evaluating the
    affected edges would), (iii) evaluations per second."""
    measured = recorded_whole_traffic(workload)
    alg = st.get("alg_bytes") or None
    evals = st.get("evaluations") or None
    out = {"evaluations": evals, "alg_bytes_method": alg, "counter_bytes": measured,
           "device_ms_median": device_ms}
    if measured and device_ms:
        out["counter_frac"] = measured / (device_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
    if measured and alg:
        out["traffic_efficiency"] = measured / alg
    if evals and device_ms:
        out["evaluations_per_s"] = evals / (device_ms * 1e-3)
    return out


def roofline_from_stats(st: dict, workload: str):
    """Roofline object of the dominant round kernel from a stats-mode run."""
    km, kl, work = st["kernel_ms"], st["kernel_launches"], st["work"]
    dom = max(("level_events", "support_update"), key=lambda k: km[k])
    table = LEVEL_BYTES if dom == "level_events" else SUPPORT_BYTES
    alg_bytes = sum(work[k] * b for k, b in table.items())
    launches = max(kl[dom], 1)
    avg_ms = km[dom] / launches
    per_launch = alg_bytes / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = recorded_traffic(KERNEL_SYMBOL[dom], workload)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": KERNEL_SYMBOL[dom], "launches": int(launches),
            "avg_launch_us": avg_ms * 1e3, "alg_bytes_per_launch": per_launch,
            "share_of_device_time": km[dom] / max(sum(km.values()), 1e-9)}


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it)."""
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(g, h, threads):
    import oracle
    t0 = time.perf_counter()
    _, _, info = oracle.decompose(g, h, threads=threads)
    return time.perf_counter() - t0, info


def cpu_baseline(workload: str):
    """Time the plain CPU oracle on bounded samples of the workload family:
    all host cores on the main sample, and one core next to all cores on a
    smaller one (the oracle's parallel speed-up on the same input)."""
    make, h, _ = WORKLOADS[workload]
    if workload.startswith("chung_lu"):
        g, g1 = W.d2(n=CPU_SAMPLE_N), W.d2(n=CPU_SAMPLE_N // 2)
        desc = f"Chung-Lu n={CPU_SAMPLE_N} (same avg_deg/gamma/seed)"
        desc1 = f"Chung-Lu n={CPU_SAMPLE_N // 2}"
    elif workload.startswith("rmat"):
        g, g1 = W.d3(scale=11), W.d3(scale=9)
        desc = "R-MAT scale 11 (same a,b,c,d, ef, seed)"
        desc1 = "R-MAT scale 9"
    else:
        g = g1 = make()
        desc = desc1 = "the workload itself"
    cores = len(os.sched_getaffinity(0))
    dt, info = _time_oracle(g, h, cores)
    dt1, info1 = _time_oracle(g1, h, 1)
    dtn, _ = _time_oracle(g1, h, cores)
    return {"value": g.m / dt, "unit": "edges/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"oracle full decomposition of {desc}: m={g.m}, {info['rounds']} rounds, "
                      f"{dt:.2f} s on {cores} threads; the oracle re-evaluates every live edge "
                      f"each round, so its rate falls as graphs grow",
            "one_core": {"value": g1.m / dt1, "unit": "edges/s", "cores": 1,
                         "sample": f"oracle full decomposition of {desc1}: m={g1.m}, "
                                   f"{info1['rounds']} rounds, {dt1:.2f} s on 1 thread"},
            "all_cores_same_sample": {"value": g1.m / dtn, "unit": "edges/s", "cores": cores,
                                      "seconds": dtn},
            }


# Algorithmic bytes of the H-index kernels, per unit of counted work:
#   edge updates: per edge and sweep its endpoints, H and the two drop masks
#     (28 B); the bytes the kernel counts for its passes over common
#     neighbourhoods (list walk: 12 B per member of the smaller ball -- its id,
#     key and the probed ball word -- plus 4 B per common member for the rank
#     word; bitset scan: 16 B per word pair plus 8 B of rank words per word
#     with common members); per common member the two path keys (8 B)
#   path-key rows: per row 12 B (offsets, flag); per row entry 4 B (zeroed);
#     per direct key 24 B (col_idx, edge id, H, rank word and ball word, key);
#     per relaxation 28 B (the same plus the atomic maximum)
HX_WORK_KINDS = ("edge_evaluations", "rows_built", "relaxations", "direct_keys",
                 "row_entries", "passes", "scan_bytes", "common_members")
HX_CPU_SAMPLE_N = 2000  # Chung-Lu sample the H-index oracle finishes in about 10-30 s


def _hx_roofline(st: dict, m: int) -> dict:
    km = list(st["kernel_ms"].values())
    kl = list(st["kernel_launches"].values())
    w = list(st["work"].values())
    edge_bytes = w[6] + w[7] * 8 + st["rounds"] * m * 28
    path_bytes = w[1] * 12 + w[4] * 4 + w[3] * 24 + w[2] * 28
    kinds = {"k_hx_paths": (km[1], kl[1], path_bytes), "k_hx_edges": (km[2], kl[2], edge_bytes)}
    dom = max(kinds, key=lambda k: kinds[k][0])
    ms, launches, alg = kinds[dom]
    launches = max(launches, 1)
    avg_ms = ms / launches
    per_launch = alg / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, "hindex"),
            "kernel": dom,
            "launches": int(launches), "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": per_launch,
            "share_of_device_time": ms / max(sum(km), 1e-9),
            "kernel_ms": {"init": km[0], "k_hx_paths": km[1], "k_hx_edges": km[2],
                          "tracking": km[3]}}


def run_hindex_iterations(args) -> dict:
    """Sweeps to convergence of the synchronous and asynchronous H-index
    iterations (the comparison of the paper's Fig. 6) on several synthetic
    graphs; both outputs are compared bit for bit."""
    import torch
    import paper_2411_06405_amd as ht
    cases = [(f"G(200,0.05) seed {s}", W.d1(s), 2) for s in range(3)]
    cases += [("Chung-Lu n=20000", W.d2(n=20_000), 1), ("Chung-Lu n=20000", W.d2(n=20_000), 2),
              ("Chung-Lu n=100000", W.d2(), 1), ("Chung-Lu n=100000", W.d2(), 2),
              ("R-MAT scale 12", W.d3(scale=12), 2), ("R-MAT scale 14", W.d3(scale=14), 1)]
    rows = []
    dev = torch.device("cuda:0")
    for name, g, h in cases:
        _log(f"{name} h={h} m={g.m}")
        rp = torch.from_numpy(g.row_ptr.view(np.int32)).to(dev)
        ci = torch.from_numpy(g.col_idx.view(np.int32)).to(dev)
        ws = ht.hindex_workspace(rp, ci, g.n, h, device=dev)
        row = {"graph": name, "n": g.n, "m": g.m, "h": h}
        outs = []
        for mode, asyn in (("sync", False), ("async", True)):
            ht.hindex(rp, ci, g.n, h, asynchronous=asyn, workspace=ws, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t, sw = ht.hindex(rp, ci, g.n, h, asynchronous=asyn, workspace=ws, device=dev)
            torch.cuda.synchronize()
            row[f"{mode}_sweeps"] = sw
            row[f"{mode}_ms"] = (time.perf_counter() - t0) * 1e3
            outs.append(t)
        row["identical"] = bool(torch.equal(outs[0], outs[1]))
        rows.append(row)
        del ws
        torch.cuda.empty_cache()
    return {"metric": "H-index sweeps to convergence, synchronous vs asynchronous",
            "unit": "sweeps", "n_gpus": 1, "data": "synthetic", "dtype": "u32",
            "higher_is_better": False, "rows": rows}


def _calibration_copy(torch, dev) -> None:
    """A 256 MiB device copy: the reference kernel for the HBM byte counters."""
    src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def run_hindex(args) -> dict:
    import torch
    import paper_2411_06405_amd as ht

    make, _, desc = WORKLOADS["chung_lu_100k_h2"]
    h = args.hx_h
    desc = desc.replace("h=2", f"h={h}")
    g = make()
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr.view(np.int32)).to(dev)
    ci = torch.from_numpy(g.col_idx.view(np.int32)).to(dev)
    ws = ht.hindex_workspace(rp, ci, g.n, h, pruning="keys", device=dev)  # fits every mode
    _log(f"H-index workspace {ws.numel() / 2**30:.2f} GiB")
    for _ in range(args.warmup):
        ht.hindex(rp, ci, g.n, h, workspace=ws, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t_sync, sweeps = ht.hindex(rp, ci, g.n, h, workspace=ws, device=dev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ref = t_sync.clone()
    modes = {}
    others = () if args.hx_sync_only else (
        ("async", dict(asynchronous=True)), ("sync_all", dict(track=False)),
        ("async_all", dict(asynchronous=True, track=False)),
        ("sync_keys", dict(pruning="keys")), ("async_keys", dict(asynchronous=True, pruning="keys")))
    for name, kw in others:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t_m, sw = ht.hindex(rp, ci, g.n, h, workspace=ws, device=dev, **kw)
        torch.cuda.synchronize()
        wk = list(ht.last_stats()["work"].values())
        modes[name] = {"ms": (time.perf_counter() - t1) * 1e3, "sweeps": sw,
                       "identical": bool(torch.equal(t_m, ref)),
                       "edge_evaluations": int(wk[0]), "rows_built": int(wk[1])}
        _log(f"{name}: {modes[name]}")
    identical, peel_ms = None, None
    if not args.hx_sync_only:
        pws = ht.alloc_workspace(g.n, g.m, h, device=dev)
        ht.decompose(rp, ci, g.n, h, workspace=pws, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t_peel, _ = ht.decompose(rp, ci, g.n, h, workspace=pws, device=dev)
        torch.cuda.synchronize()
        peel_ms = (time.perf_counter() - t1) * 1e3
        identical = bool(torch.equal(t_peel, ref))
        del pws
    os.environ["HOTRUSS_SWEEPS"] = "1"
    ht.hindex(rp, ci, g.n, h, workspace=ws, device=dev, stats=True)
    torch.cuda.synchronize()
    st = ht.last_stats()
    if args.calibrate:
        _calibration_copy(torch, dev)
    line = {
        "metric": f"edges/s to h-trussness (h={h})", "value": g.m * args.steps / dt,
        "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / max(args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc + "; H-index fixpoint method, synchronous sweeps",
                   "n": g.n, "m": g.m, "h": h, "sweeps": sweeps,
                   "identical_to_peeling": identical,
                   "peeling_ms": peel_ms, "other_modes": modes,
                   "value_changes": int(st["events"]),
                   "work": dict(zip(HX_WORK_KINDS, map(int, st["work"].values())))},
        "roofline": _hx_roofline(st, g.m),
    }
    if not args.no_cpu_baseline:
        from oracle.hindex import hindex_trussness  # the CPU-baseline leg only
        gs = W.d2(n=HX_CPU_SAMPLE_N)
        t1 = time.perf_counter()
        _, sw = hindex_trussness(gs, h)
        cdt = time.perf_counter() - t1
        line["cpu_baseline"] = {
            "value": gs.m / cdt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"H-index oracle (synchronous sweeps, numpy) on Chung-Lu "
                      f"n={HX_CPU_SAMPLE_N} (same avg_deg/gamma/seed): m={gs.m}, {sw} sweeps, "
                      f"{cdt:.2f} s"}
    return line


def _log(msg: str) -> None:
    """Progress of the long multi-graph runs, on stderr (the JSON line is stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _gen_pool(fn, specs, workers: int):
    """Generate graphs in worker processes (forked before any GPU use)."""
    import multiprocessing as mp
    if workers <= 1:
        return [fn(x) for x in specs]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(fn, specs, chunksize=1)


def _workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def run_batched(args) -> dict:
    """Batched call against loops of single-graph calls (one and four streams)."""
    from graphgen import concat
    specs = W.d4_specs()[:args.graphs]  # a prefix of the full 512-graph draw
    gs = _gen_pool(W.d4_graph, specs, _workers())
    _log(f"generated {len(gs)} graphs, sum m = {sum(g.m for g in gs)}")
    hs = np.array([s[2] for s in specs], dtype=np.uint32)
    b = concat(gs, hs)
    import threading
    import torch
    import paper_2411_06405_amd as ht
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(b.row_ptr_cat.view(np.int32)).to(dev)
    ci = torch.from_numpy(b.col_idx_cat.view(np.int32)).to(dev)
    vo, ao, eo = (b.vtx_off.astype(np.int64), b.adj_off.astype(np.int64),
                  b.edge_off.astype(np.int64))
    B, mt = b.B, int(eo[-1])
    # initial-pass knobs picked by the autotuner on the batch's largest graphs
    # (cached by shape); the plain loops below use the same setting
    tune = ht.autotune.autotune_batch(gs, hs, device=dev)
    _log(f"autotuned: {tune}")
    wsb = ht.batched_workspace_bytes(b.vtx_off, b.edge_off, b.h, tune=tune)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)

    def batched():
        return ht.decompose_batched(rp, ci, b.vtx_off, b.adj_off, b.edge_off, b.h,
                                    workspace=ws, tune=tune, device=dev)
    for i in range(args.warmup):
        batched()
        torch.cuda.synchronize()
        _log(f"batched warm-up {i + 1}/{args.warmup} done")
    t0 = time.perf_counter()
    for i in range(args.steps):
        tb, rb = batched()
        torch.cuda.synchronize()
        _log(f"batched step {i + 1}/{args.steps}: {time.perf_counter() - t0:.2f} s so far")
    t_batch = (time.perf_counter() - t0) / max(args.steps, 1)
    del ws
    torch.cuda.empty_cache()

    # single-graph calls, one graph after another on `nstreams` streams (one
    # host thread and one workspace per stream)
    n_ = [int(vo[g + 1] - vo[g]) for g in range(B)]
    wmax = max(ht.workspace_bytes(n_[g], int(eo[g + 1] - eo[g]), int(hs[g]), tune)
               for g in range(B))
    tp = torch.empty(max(mt, 1), dtype=torch.int32, device=dev)
    rp_out = torch.empty(max(mt, 1), dtype=torch.int32, device=dev)

    def plain_loop(nstreams: int) -> float:
        streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
        wss = [torch.empty(wmax, dtype=torch.uint8, device=dev) for _ in range(nstreams)]
        order = sorted(range(B), key=lambda g: -int(eo[g + 1] - eo[g]))
        errors = []

        def worker(i):
            try:
                with torch.cuda.stream(streams[i]):
                    for c, g in enumerate(order[i::nstreams]):
                        t, r = ht.decompose(rp[vo[g] + g:vo[g + 1] + g + 1], ci[ao[g]:ao[g + 1]],
                                            n_[g], int(hs[g]), workspace=wss[i], tune=tune,
                                            stream=streams[i], device=dev)
                        tp[eo[g]:eo[g + 1]].copy_(t)
                        rp_out[eo[g]:eo[g + 1]].copy_(r)
                        if i == 0 and c % 16 == 15:
                            streams[i].synchronize()
                            _log(f"plain x{nstreams}: stream 0 finished {c + 1} graphs")
                    streams[i].synchronize()
            except Exception as e:  # reported below
                errors.append(e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = [threading.Thread(target=worker, args=(i,)) for i in range(nstreams)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if errors:
            raise errors[0]
        return dt
    t_plain1 = plain_loop(1)
    _log(f"plain loop, 1 stream: {t_plain1:.2f} s")
    same1 = bool(torch.equal(tb, tp[:mt]) and torch.equal(rb, rp_out[:mt]))
    t_plain4 = plain_loop(4)
    _log(f"plain loop, 4 streams: {t_plain4:.2f} s")
    same4 = bool(torch.equal(tb, tp[:mt]) and torch.equal(rb, rp_out[:mt]))
    value = B / t_batch
    return {
        "metric": "graphs/s, batched call vs single-graph calls",
        "value": value, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batch * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"first {B} of {W.D4_B} Barabasi-Albert graphs, n~U[1000,50000], "
                               f"m_attach~U{{3..8}}, 5 planted cliques of 8-20 vertices each, "
                               f"h~U{{2,3}}, seed {W.D4_SEED}",
                   "graphs": B, "sum_n": int(vo[-1]), "sum_m": mt,
                   "workspace_gib": round(wsb / 2**30, 2), "autotuned": tune},
        "plain_1stream_graphs_s": B / t_plain1, "plain_4stream_graphs_s": B / t_plain4,
        "speedup_vs_plain_1stream": t_plain1 / t_batch,
        "speedup_vs_plain_4stream": t_plain4 / t_batch,
        "edges_per_s_batched": mt / t_batch,
        "identical_to_plain": same1 and same4,
    }


def run_serve(args) -> dict:
    """Poisson request stream through a session with a device-memory budget."""
    specs = W.d5_request_specs(args.requests)
    if args.max_class:
        specs = [s if s[0] <= args.max_class else (args.max_class,) + tuple(s[1:])
                 for s in specs]
    gs = _gen_pool(W.d5_graph, specs, _workers())
    _log(f"generated {len(gs)} requests, sum m = {sum(g.m for g in gs)}")
    import torch
    import paper_2411_06405_amd as ht
    dev = torch.device("cuda:0")
    budget = int(args.budget_gib * 2**30)
    rps = [torch.from_numpy(g.row_ptr.view(np.int32)).to(dev) for g in gs]
    cis = [torch.from_numpy(g.col_idx.view(np.int32)).to(dev) for g in gs]
    hs = [s[3] for s in specs]
    N = len(gs)
    sess = ht.Session(pool_bytes=budget, max_slots=args.slots, max_h=max(hs), device=dev)

    def drive(arrivals):
        """Submit request i at arrivals[i] (seconds); return completion times and results."""
        t0 = time.perf_counter()
        done_at = np.full(N, np.nan)
        tickets = [None] * N
        nxt, pending = 0, set()
        while nxt < N or pending:
            now = time.perf_counter() - t0
            while nxt < N and arrivals[nxt] <= now:
                tickets[nxt] = sess.submit(rps[nxt], cis[nxt], gs[nxt].n, hs[nxt])
                pending.add(nxt)
                nxt += 1
            if pending:
                sess.progress(max_graph_launches=1)
                now = time.perf_counter() - t0
                for i in list(pending):
                    if sess.poll(tickets[i]):
                        done_at[i] = now
                        pending.discard(i)
                        _log(f"request {i} (n={gs[i].n}, h={hs[i]}) done at {now:.1f} s, "
                             f"{len(pending)} pending, {N - nxt} to arrive")
            elif nxt < N:
                time.sleep(max(0.0, min(arrivals[nxt] - now, 0.01)))
        res = [sess.result(tk) for tk in tickets]
        return done_at, res

    # warm-up (graph capture, first-touch) on the smallest requests
    small = sorted(range(N), key=lambda i: gs[i].m)[:min(8, N)]
    for i in small:
        sess.submit(rps[i], cis[i], gs[i].n, hs[i])
    sess.progress()
    # capacity: every request queued at time 0
    _log("warm-up done")
    done_cap, res_cap = drive(np.zeros(N))
    capacity = N / float(np.nanmax(done_cap))
    _log(f"capacity run: {capacity:.2f} graphs/s")
    out = {"capacity_graphs_s": capacity, "loads": {}}
    identical = True
    for load in args.loads:
        arr = W.poisson_arrivals(N, load * capacity)
        arr = arr - arr[0]
        done_at, res = drive(arr)
        _log(f"load {load}: done in {float(np.nanmax(done_at)):.2f} s")
        lat = (done_at - arr) * 1e3
        skip = N // 20  # warm-up share of the stream
        lat_s = lat[skip:]
        identical &= all(np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
                         for a, c in zip(res, res_cap))
        out["loads"][str(load)] = {
            "qps": load * capacity, "graphs_s": N / float(np.nanmax(done_at)),
            "p50_ms": float(np.percentile(lat_s, 50)), "p99_ms": float(np.percentile(lat_s, 99)),
            "max_ms": float(np.max(lat_s))}
    sess.close()
    head = out["loads"][str(args.loads[0])]
    classes = sorted({s[0] for s in specs})
    return {
        "metric": "p50/p99 latency and graphs/s, served request stream",
        "value": head["graphs_s"], "unit": "graphs/s", "n_gpus": 1, "steps": N,
        "warmup": len(small), "ms_per_step": 1e3 / head["graphs_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{N} Chung-Lu requests, n in {classes}, gamma~U[2.1,2.8], "
                               f"avg_deg~U[6,20], h~U{{2,3,4}}, Poisson arrivals seed "
                               f"{W.D5_SEED}",
                   "budget_gib": args.budget_gib, "slots": args.slots,
                   "sum_m": int(sum(g.m for g in gs))},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], **out,
        "identical_across_runs": bool(identical),
    }


def main(argv=None):
    # the library reports progress of long calls on stderr (every 10 s at most)
    os.environ.setdefault("HOTRUSS_PROGRESS", "1")
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat18_h2",
                    choices=sorted(WORKLOADS) + ["batched", "serve", "hindex",
                                                 "hindex_iterations"])
    ap.add_argument("--graphs", type=int, default=W.D4_B, help="batched: number of graphs")
    ap.add_argument("--requests", type=int, default=200, help="serve: number of requests")
    ap.add_argument("--max-class", type=int, default=0,
                    help="serve: cap the size classes at this n (0: all classes)")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve: device-memory budget")
    ap.add_argument("--slots", type=int, default=64, help="serve: concurrent requests")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 0.8],
                    help="serve: arrival rates as fractions of the measured capacity")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stats", action="store_true",
                    help="skip the stats-mode decomposition (profiling runs)")
    ap.add_argument("--hx-h", type=int, default=2, help="hindex: hop threshold h")
    ap.add_argument("--hx-sync-only", action="store_true",
                    help="hindex: time the synchronous sweeps only (profiling runs)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also copy a 256 MiB buffer (reference kernel for HBM counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (--gpus 1); "
                                   "the library has no multi-GPU path"}))
        return 2

    if args.workload == "batched":
        print(json.dumps(run_batched(args)), flush=True)
        return 0
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return 0
    if args.workload == "hindex":
        print(json.dumps(run_hindex(args)), flush=True)
        return 0
    if args.workload == "hindex_iterations":
        print(json.dumps(run_hindex_iterations(args)), flush=True)
        return 0

    import torch
    import paper_2411_06405_amd as ht

    make, h, desc = WORKLOADS[args.workload]
    g = make()
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr.view(np.int32)).to(dev)
    ci = torch.from_numpy(g.col_idx.view(np.int32)).to(dev)
    ws = ht.alloc_workspace(g.n, g.m, h, device=dev)
    stats_tune = {"flags": ht._lib.HO_FLAG_STATS}

    for _ in range(args.warmup):
        ht.decompose(rp, ci, g.n, h, workspace=ws, device=dev)
    torch.cuda.synchronize()
    _log(f"{desc}: n={g.n} m={g.m}, timing {args.steps} decompositions")
    device_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t, rho = ht.decompose(rp, ci, g.n, h, workspace=ws, device=dev)
        device_ms.append(ht.last_stats()["device_ms"])  # the call has completed
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ht.last_stats()
    ms = dt * 1000.0 / max(args.steps, 1)
    value = g.m * args.steps / dt
    _log(f"timed: {ms:.1f} ms per decomposition")
    # one more decomposition with every round kernel timed by HIP events on
    # this stream and the chunked kernels' work counted (host-driven rounds)
    stt = None
    if not args.no_stats:
        _log("stats-mode decomposition (host-driven rounds, per-kernel HIP events)")
        ts, _ = ht.decompose(rp, ci, g.n, h, workspace=ws, device=dev, tune=stats_tune)
        torch.cuda.synchronize()
        stt = ht.last_stats()
        if args.steps > 0:
            assert torch.equal(ts, t), "stats-mode decomposition differs"
    dmed = float(np.median(device_ms)) if device_ms else None

    line = {
        "metric": "edges/s to h-trussness (h=2)" if h == 2 else f"edges/s to h-trussness (h={h})",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "m": g.m, "h": h,
                   "rounds": int(st["rounds"]), "levels": int(st["levels"]),
                   "top_level_events": int(st["events"]),
                   "overflow_rounds": int(st["overflows"])},
        "device_ms": {"median": float(np.median(device_ms)) if device_ms else None,
                      "min": float(np.min(device_ms)) if device_ms else None,
                      "max": float(np.max(device_ms)) if device_ms else None,
                      "runs": len(device_ms)},
        "edges_per_s_device_median": (g.m / (float(np.median(device_ms)) * 1e-3)
                                      if device_ms else None),
        "roofline": roofline_from_stats(stt, args.workload) if stt else None,
        "kernel_ms_stats_mode": ({k: round(v, 3) for k, v in stt["kernel_ms"].items()}
                                 if stt else None),
        "whole_run": whole_run(stt or {}, args.workload, dmed),
    }
    if args.calibrate:
        _calibration_copy(torch, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
