"""Benchmark: edges/s to h-trussness on one MI355X.

A step is one full decomposition (every edge's h-trussness) of a synthetic
graph whose CSR is already resident in HBM.  Default workload: Chung-Lu
power-law graph, n = 100,000, average degree 10, exponent 2.5, seed 1, h = 2.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

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
}

CPU_SAMPLE_N = 3000  # Chung-Lu sample the oracle decomposes completely

# Algorithmic bytes per unit of work of the two chunked round kernels (each
# access counted at its natural size, not as cache lines):
#   ball-change events: work item 16 B; examined slot 8 B (srem, col_idx);
#     tested pair 32 B (ball bit word, two row extents, (j-1)-ball word);
#     witness probe 16 B (srem, col_idx, ball word); dropped pair 48 B (two
#     ball-bit atomics, change-mark atomic, event record, follow-up items)
#   support update: work item 16 B; adjacency slot 20 B (srem, col_idx,
#     edge id, ball word); lost common neighbour 8 B (support atomic)
LEVEL_BYTES = {"level_items": 16, "level_slots": 8, "level_candidates": 32,
               "level_probes": 16, "level_drops": 48}
SUPPORT_BYTES = {"support_items": 16, "support_slots": 20, "support_hits": 8}
KERNEL_SYMBOL = {"level_events": "k_level", "support_update": "k_support"}
PROFILES = ROOT / "profiles"


def kernel_source_sha() -> str:
    import hashlib
    src = ROOT / "paper_2411_06405_amd" / "csrc" / "hotruss_kernels.hip"
    return hashlib.sha256(src.read_bytes()).hexdigest()[:16]


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
    traffic = None
    tfile = PROFILES / f"traffic_{KERNEL_SYMBOL[dom]}_{workload}.txt"
    if tfile.exists():
        t = json.loads(tfile.read_text())
        if t.get("source_sha") == kernel_source_sha():
            traffic = t.get("bytes_per_launch")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": KERNEL_SYMBOL[dom], "launches": int(launches),
            "avg_launch_us": avg_ms * 1e3, "alg_bytes_per_launch": per_launch,
            "share_of_device_time": km[dom] / max(sum(km.values()), 1e-9)}


def cpu_baseline(workload: str):
    """Time the plain CPU oracle on a bounded sample of the workload family."""
    import oracle
    make, h, _ = WORKLOADS[workload]
    if workload.startswith("chung_lu"):
        g = W.d2(n=CPU_SAMPLE_N)
        desc = f"oracle full decomposition of Chung-Lu n={CPU_SAMPLE_N} (same avg_deg/gamma/seed)"
    elif workload.startswith("rmat"):
        g = W.d3(scale=10)
        desc = "oracle full decomposition of R-MAT scale 10 (same a,b,c,d, ef, seed)"
    else:
        g = make()
        desc = "oracle full decomposition of the workload itself"
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    _, _, info = oracle.decompose(g, h, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt, "unit": "edges/s", "cores": cores, "kind": "oracle",
            "sample": f"{desc}: m={g.m}, {info['rounds']} rounds, {dt:.2f} s; the oracle "
                      f"re-evaluates every live edge each round, so its rate falls as graphs grow"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chung_lu_100k_h2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="also copy a 256 MiB buffer (reference kernel for HBM counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "multi-GPU runs are not part of this build"}))
        return 2

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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t, rho = ht.decompose(rp, ci, g.n, h, workspace=ws, device=dev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ht.last_stats()
    ms = dt * 1000.0 / max(args.steps, 1)
    value = g.m * args.steps / dt
    # one more decomposition with every round kernel timed by HIP events on
    # this stream and the chunked kernels' work counted (host-driven rounds)
    ht.decompose(rp, ci, g.n, h, workspace=ws, device=dev, tune=stats_tune)
    torch.cuda.synchronize()
    stt = ht.last_stats()

    line = {
        "metric": "edges/s to h-trussness (h=2)" if h == 2 else f"edges/s to h-trussness (h={h})",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "m": g.m, "h": h,
                   "rounds": int(st["rounds"]), "levels": int(st["levels"]),
                   "top_level_events": int(st["events"]),
                   "overflow_rounds": int(st["overflows"])},
        "roofline": roofline_from_stats(stt, args.workload),
        "kernel_ms_stats_mode": {k: round(v, 3) for k, v in stt["kernel_ms"].items()},
    }
    if args.calibrate:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
