"""Autotuner of the initial-pass knobs of libhotruss (host logic only).

The initial pass of a decomposition (edge ids, level-1..h ball build,
h-support of every edge) has three knobs that change speed, never results:

* ``dense_threshold`` -- level-2 ball build: bottom-up (OR of neighbour rows,
  a dense-bitset frontier) versus top-down (scatter of adjacency lists, a
  sparse-list frontier) per row;
* ``word_bits`` -- bitset load width per lane in the h-support pass (64/128);
* ``edges_per_wave`` -- edges sharing one wavefront in that pass (1..16).

``autotune`` times ``hoTrussHSupport`` (which runs exactly that pass) on the
caller's graph for each candidate setting, one knob group at a time, and
keeps the fastest.  ``autotune_rounds`` adds the knob of the peel rounds,
which take almost all of a decomposition's time: ``grid_blocks``, the
workgroups of the round kernels (the ball-change kernel uses a quarter as
many, of four times the size), timed on whole decompositions.  Results are cached in a JSON file keyed by the device
name and a bucket of the graph's shape (vertices, average degree, degree
skew, h), so graphs of a similar shape reuse a measurement.  The timing runs
through the C ABI like any other call; nothing here computes on the CPU.
"""
from __future__ import annotations

import json
import math
import os
import time
from pathlib import Path
from typing import Callable, Iterable

import numpy as np

DENSE_THRESHOLDS = (4, 32, 256, 1 << 30)   # 1 << 30: never bottom-up
WIDTHS = (64, 128)
EDGES_PER_WAVE = (1, 4, 16)
GRID_PER_CU = (4, 8, 16)   # round-kernel workgroups per CU
DEFAULT_CACHE = Path(os.environ.get("HOTRUSS_TUNE_CACHE",
                                    Path.home() / ".cache" / "hotruss_autotune.json"))


def shape_key(device_name: str, n: int, m: int, h: int, max_deg: int) -> str:
    """Cache key: device and log2 buckets of n, average degree and degree skew."""
    avg = 2.0 * m / max(n, 1)
    skew = max_deg / max(avg, 1e-9)
    b = lambda v: int(math.floor(math.log2(max(v, 1.0))))  # noqa: E731
    return f"{device_name}|n2^{b(n)}|d2^{b(avg)}|s2^{b(skew)}|h{h}"


def choose(timings: dict) -> tuple:
    """Fastest candidate; ties go to the first listed (dicts keep order)."""
    best, best_t = None, math.inf
    for cand, t in timings.items():
        if t < best_t:
            best, best_t = cand, t
    return best


def search(time_fn: Callable[[dict], float], repeats: int = 3) -> dict:
    """Coordinate search over the knob groups with a timing function.

    time_fn(tune) returns seconds for one run with that tuning; each candidate
    is run `repeats` times and scored by its minimum."""
    def score(tune):
        return min(time_fn(tune) for _ in range(repeats))
    base = {"word_bits": 64, "edges_per_wave": 0, "dense_threshold": 0}
    dense = {dt: score(dict(base, dense_threshold=dt)) for dt in DENSE_THRESHOLDS}
    base["dense_threshold"] = choose(dense)
    pairs = {(wb, ew): score(dict(base, word_bits=wb, edges_per_wave=ew))
             for wb in WIDTHS for ew in EDGES_PER_WAVE}
    base["word_bits"], base["edges_per_wave"] = choose(pairs)
    return base


def search_rounds(time_fn: Callable[[dict], float], base: dict, num_cu: int,
                  repeats: int = 1) -> dict:
    """The round kernels' grid width, on top of the initial-pass setting
    `base`: time_fn(tune) returns seconds for one whole decomposition."""
    timings = {}
    for per in GRID_PER_CU:
        tune = dict(base, grid_blocks=per * num_cu)
        timings[per * num_cu] = min(time_fn(tune) for _ in range(repeats))
    return dict(base, grid_blocks=choose(timings))


class Cache:
    """JSON file of {shape key: tuning}."""

    def __init__(self, path=None):
        self.path = Path(path) if path is not None else DEFAULT_CACHE
        try:
            self.data = json.loads(self.path.read_text())
        except (OSError, ValueError):
            self.data = {}

    def get(self, key: str):
        v = self.data.get(key)
        return dict(v) if isinstance(v, dict) else None

    def put(self, key: str, tune: dict) -> None:
        self.data[key] = dict(tune)
        try:
            self.path.parent.mkdir(parents=True, exist_ok=True)
            tmp = self.path.with_suffix(".tmp")
            tmp.write_text(json.dumps(self.data, indent=1, sort_keys=True))
            os.replace(tmp, self.path)
        except OSError:
            pass  # an unwritable cache only costs a re-measurement


def autotune(row_ptr, col_idx, n: int, h: int, device="cuda", cache=None, refresh=False,
             repeats: int = 3) -> dict:
    """Tuning dict for hoTrussDecompose / hoTrussHSupport on this graph.

    row_ptr / col_idx: the graph's CSR (device tensors or host arrays)."""
    import torch

    from . import _lib
    rp = _lib._dev_u32(row_ptr, device)
    ci = _lib._dev_u32(col_idx, device)
    m = ci.numel() // 2
    if m == 0:
        return {}
    deg = (rp[1:] - rp[:-1])
    max_deg = int(deg.max().item()) if n else 0
    name = torch.cuda.get_device_name(torch.device(device))
    key = shape_key(name, n, m, h, max_deg)
    c = cache if isinstance(cache, Cache) else Cache(cache)
    if not refresh:
        hit = c.get(key)
        if hit is not None:
            return hit
    ws = _lib.alloc_workspace(n, m, h, device=device)
    out = torch.empty(max(m, 1), dtype=torch.int32, device=device)
    stream = torch.cuda.current_stream(torch.device(device))

    def time_fn(tune: dict) -> float:
        stream.synchronize()
        t0 = time.perf_counter()
        rc = _lib.lib.hoTrussHSupport(rp.data_ptr(), ci.data_ptr(), n, m, h, out.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _lib._tuning(tune),
                                     stream.cuda_stream)
        _lib._check(rc, "hoTrussHSupport")
        return time.perf_counter() - t0

    time_fn({})  # first touch of the workspace
    best = search(time_fn, repeats)
    c.put(key, best)
    return best


def autotune_batch(graphs: Iterable, hs, device="cuda", cache=None, sample: int = 3) -> dict:
    """One tuning for a batch: measured on the largest graphs of the batch
    (graphgen.Graph-like objects with row_ptr, col_idx, n, m), whose initial
    pass dominates; the setting chosen most often wins."""
    graphs = list(graphs)
    hs = np.asarray(hs)
    order = sorted(range(len(graphs)), key=lambda g: -graphs[g].m)[:max(1, sample)]
    votes = {}
    for g in order:
        t = autotune(graphs[g].row_ptr, graphs[g].col_idx, graphs[g].n, int(hs[g]),
                     device=device, cache=cache)
        k = tuple(sorted(t.items()))
        votes[k] = votes.get(k, 0) + 1
    best = max(votes.items(), key=lambda kv: kv[1])[0]
    return dict(best)


def autotune_rounds(row_ptr, col_idx, n: int, h: int, device="cuda", cache=None,
                    refresh=False, repeats: int = 1) -> dict:
    """Initial-pass knobs (``autotune``) plus the round kernels' grid width,
    chosen by timing whole decompositions of this graph (use a graph that
    decomposes in seconds, or a smaller one of the same shape)."""
    import torch

    from . import _lib
    base = autotune(row_ptr, col_idx, n, h, device=device, cache=cache, refresh=refresh)
    rp = _lib._dev_u32(row_ptr, device)
    ci = _lib._dev_u32(col_idx, device)
    m = ci.numel() // 2
    if m == 0:
        return base
    deg = (rp[1:] - rp[:-1])
    max_deg = int(deg.max().item()) if n else 0
    dev = torch.device(device)
    name = torch.cuda.get_device_name(dev)
    key = shape_key(name, n, m, h, max_deg) + "|rounds"
    c = cache if isinstance(cache, Cache) else Cache(cache)
    if not refresh:
        hit = c.get(key)
        if hit is not None:
            return hit
    ws = _lib.alloc_workspace(n, m, h, device=device)
    stream = torch.cuda.current_stream(dev)

    def time_fn(tune: dict) -> float:
        _lib.decompose(rp, ci, n, h, workspace=ws, tune=tune, device=device)
        return _lib.last_stats()["device_ms"] * 1e-3

    time_fn(dict(base))  # first touch of the workspace, graph capture
    stream.synchronize()
    num_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    best = search_rounds(time_fn, base, num_cu, repeats)
    c.put(key, best)
    return best
