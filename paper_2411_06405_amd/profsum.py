"""Summarise rocprofv3 databases of a bench run into short text files.

    python -m paper_2411_06405_amd.profsum TRACE_DB FETCH_DB WRITE_DB OUTDIR TAG CMD
    python -m paper_2411_06405_amd.profsum counters PMC_DB OUTDIR TAG CMD

Writes OUTDIR/kernels_TAG.txt (per-kernel dispatch count and durations from
--kernel-trace), OUTDIR/hbm_counters_TAG.txt (mean FETCH_SIZE / WRITE_SIZE per
dispatch, KiB) and OUTDIR/traffic_KERNEL_TAG.txt for the kernels named in
KERNEL_SOURCES (HBM bytes per launch, scaled by what the same counters read
for a 256 MiB device-to-device copy), and OUTDIR/traffic_whole_TAG.txt: the
scaled bytes of every library kernel (names starting with k_) per
decomposition, a decomposition being one dispatch of k_init_ctl.  The
counters form writes OUTDIR/counters_TAG.txt: the mean per dispatch of every
counter of one --pmc run, per kernel.
"""
from __future__ import annotations

import hashlib
import json
import sqlite3
import sys
from pathlib import Path

import numpy as np

COPY_BYTES = 256 << 20
# kernels whose HBM traffic is recorded, and the source file each is built from
KERNEL_SOURCES = {"k_level": "hotruss_kernels.hip", "k_support": "hotruss_kernels.hip",
                  "k_hx_paths": "hotruss_hindex.hip", "k_hx_edges": "hotruss_hindex.hip"}


def source_sha(srcname: str) -> str:
    src = Path(__file__).resolve().parent / "csrc" / srcname
    return hashlib.sha256(src.read_bytes()).hexdigest()[:16]


def short(name: str) -> str:
    """Kernel name without namespace, parameters or template arguments."""
    base = name.split("(")[0].replace("hotruss::", "")
    if base.startswith("void "):
        base = base[len("void "):]
    return base.split("<")[0]


def kernel_table(db: str):
    c = sqlite3.connect(db)
    rows = {}
    for name, dur in c.execute("select name, end - start from kernels"):
        rows.setdefault(name, []).append(dur / 1e3)
    out = []
    for name, d in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        d = np.array(d)
        out.append((short(name), len(d), d.sum() / 1e3, d.mean(), np.percentile(d, 50),
                    np.percentile(d, 90), d.max()))
    return out


def counter_table(db: str, counter: str):
    c = sqlite3.connect(db)
    rows = {}
    q = "select kernel_name, value from counters_collection where counter_name = ?"
    for name, val in c.execute(q, (counter,)):
        rows.setdefault(name, []).append(float(val))
    return {name: np.array(v) for name, v in rows.items()}


def main(trace_db, fetch_db, write_db, outdir, tag, cmd):
    outdir = Path(outdir)
    outdir.mkdir(parents=True, exist_ok=True)
    kt = kernel_table(trace_db)
    lines = [f"# rocprofv3 --kernel-trace --stats -- {cmd}",
             "# kernel, dispatches, total_ms, mean_us, p50_us, p90_us, max_us"]
    for r in kt:
        lines.append(f"{r[0]:40s} {r[1]:8d} {r[2]:10.3f} {r[3]:10.2f} {r[4]:10.2f} {r[5]:10.2f} {r[6]:10.1f}")
    (outdir / f"kernels_{tag}.txt").write_text("\n".join(lines) + "\n")
    fetch = counter_table(fetch_db, "FETCH_SIZE")
    write = counter_table(write_db, "WRITE_SIZE")
    # calibration: the large device-to-device copy dispatches
    def copy_kib(tab):
        vals = [v for name, arr in tab.items() if "copy" in name.lower() for v in arr
                if v > COPY_BYTES / 1024 * 0.5]
        return float(np.median(vals)) if vals else None
    cf, cw = copy_kib(fetch), copy_kib(write)
    sf = (COPY_BYTES / 1024) / cf if cf else None
    sw = (COPY_BYTES / 1024) / cw if cw else None
    lines = [f"# rocprofv3 --pmc FETCH_SIZE -- {cmd}", f"# rocprofv3 --pmc WRITE_SIZE -- {cmd}",
             f"# calibration: 256 MiB device copy reads FETCH_SIZE {cf} KiB (scale {sf}), "
             f"WRITE_SIZE {cw} KiB (scale {sw})",
             "# kernel, dispatches, mean FETCH_SIZE KiB, mean WRITE_SIZE KiB"]
    names = sorted(set(fetch) | set(write), key=lambda n: -float(fetch.get(n, np.zeros(1)).sum()))
    for n in names:
        f = fetch.get(n, np.zeros(0))
        w = write.get(n, np.zeros(0))
        lines.append(f"{short(n):40s} {len(f):8d} {f.mean() if len(f) else 0:14.2f} "
                     f"{w.mean() if len(w) else 0:14.2f}")
    (outdir / f"hbm_counters_{tag}.txt").write_text("\n".join(lines) + "\n")
    if sf is not None and sw is not None:
        lib = [n for n in set(fetch) | set(write) if short(n).startswith("k_")]
        tot = sum(float(fetch.get(n, np.zeros(0)).sum()) * 1024 * sf +
                  float(write.get(n, np.zeros(0)).sum()) * 1024 * sw for n in lib)
        ndec = sum(len(fetch[n]) for n in fetch if short(n) == "k_init_ctl")
        if ndec:
            (outdir / f"traffic_whole_{tag}.txt").write_text(json.dumps({
                "source_sha": source_sha("hotruss_kernels.hip"), "decompositions": ndec,
                "bytes_per_decomposition": tot / ndec, "fetch_scale": sf, "write_scale": sw,
                "command": cmd}, indent=1) + "\n")
    for kname, srcname in KERNEL_SOURCES.items():
        sha = source_sha(srcname)
        full = [n for n in fetch if short(n) == kname]
        if not full or sf is None or sw is None:
            continue
        f = fetch[full[0]]
        w = write.get(full[0], np.zeros_like(f))
        per_launch = float(f.mean() * 1024 * sf + w.mean() * 1024 * sw)
        (outdir / f"traffic_{kname}_{tag}.txt").write_text(json.dumps({
            "kernel": kname, "source_sha": sha, "launches": int(len(f)),
            "fetch_kib_per_launch": float(f.mean()), "write_kib_per_launch": float(w.mean()),
            "fetch_scale": sf, "write_scale": sw, "bytes_per_launch": per_launch,
            "command": cmd}, indent=1) + "\n")


def counters_main(db, outdir, tag, cmd):
    """Mean value per dispatch of every counter in one --pmc database, per kernel."""
    c = sqlite3.connect(db)
    names = [r[0] for r in c.execute("select distinct counter_name from counters_collection")]
    names.sort()
    rows = {}
    for name in names:
        for k, arr in counter_table(db, name).items():
            rows.setdefault(short(k), {})[name] = (len(arr), float(arr.mean()))
    lines = [f"# rocprofv3 --pmc {' '.join(names)} -- {cmd}",
             "# kernel, dispatches, " + ", ".join(f"mean {n}" for n in names)]
    order = sorted(rows, key=lambda k: -max(v[0] * v[1] for v in rows[k].values()))
    for k in order:
        cnt = max(v[0] for v in rows[k].values())
        vals = " ".join(f"{rows[k].get(n, (0, 0.0))[1]:16.1f}" for n in names)
        lines.append(f"{k:40s} {cnt:8d} {vals}")
    out = Path(outdir)
    out.mkdir(parents=True, exist_ok=True)
    (out / f"counters_{tag}.txt").write_text("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "counters":
        counters_main(*sys.argv[2:6])
    else:
        main(*sys.argv[1:7])
