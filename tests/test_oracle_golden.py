"""Regression guard: the oracle still reproduces its stored outputs on G(200,0.05)."""
import hashlib
import json
from pathlib import Path

import numpy as np
import pytest

from graphgen import workloads as W

GOLD = json.loads((Path(__file__).parent / "golden" / "d1_oracle.json").read_text())


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.uint32).tobytes()).hexdigest()


@pytest.mark.parametrize("case", GOLD["cases"], ids=lambda c: f"s{c['seed']}h{c['h']}")
def test_golden(oracle_mod, case):
    g = W.d1(case["seed"])
    assert (g.n, g.m) == (case["n"], case["m"])
    t, rho, info = oracle_mod.decompose(g, case["h"])
    assert info["rounds"] == case["rounds"] and info["levels"] == case["levels"]
    assert digest(t) == case["t_sha256"] and digest(rho) == case["rho_sha256"]
