"""Write tests/golden/d1_oracle.json from the plain CPU oracle only.

Records, for the uniform random graph G(200, 0.05) at seeds 0-4 and h = 1..4,
the oracle's round count, level count, trussness range and SHA-256 of the
per-edge trussness and round arrays (uint32, canonical edge order).  Used as a
regression guard on the oracle and as stored expected values for parity tests.
Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from graphgen import workloads as W  # noqa: E402


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint32).tobytes()).hexdigest()


def main():
    out = {"about": "oracle outputs for G(200,0.05); written by make_golden.py from oracle/ only",
           "cases": []}
    for seed in W.D1_SEEDS:
        g = W.d1(seed)
        for h in (1, 2, 3, 4):
            t, rho, info = oracle.decompose(g, h)
            out["cases"].append({"seed": seed, "h": h, "n": g.n, "m": g.m,
                                 "rounds": info["rounds"], "levels": info["levels"],
                                 "t_min": int(t.min()), "t_max": int(t.max()),
                                 "t_sha256": digest(t), "rho_sha256": digest(rho)})
    path = Path(__file__).parent / "d1_oracle.json"
    path.write_text(json.dumps(out, indent=1) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
