"""Host check of the re-evaluation rules the GPU H-index sweeps use (no GPU).

hoTrussHIndex skips path-key rows and edges whose values cannot change: rows
by the touched-vertex rule (at h = 2 sharpened by the smallest new value per
vertex), edges by value-bucket masks, either from changed edge values (the
paper's Lemma 4, the default) or from the rows' own path keys.  The claim is
that these rules give exactly the synchronous sequence of the definition, and
that the asynchronous chunk order reaches the same fixpoint.  This test runs
the rules as written in plain Python, with the oracle's path keys and H-index
operator for the arithmetic, on many small random graphs, and compares every
sweep with the oracle's sequence.  It checks the rules, not the kernels (the
GPU tests do that)."""
import numpy as np
import pytest

from graphgen import gen
from oracle import decompose
from oracle.hindex import UNREACHED, hindex, hindex_sequence, path_keys
from tests.conftest import seeded


def bucket(v: int) -> int:
    """0..31 exact, then two buckets per octave, the rest in 63."""
    if v < 32:
        return v
    e = v.bit_length() - 1
    return min(63, 32 + (e - 5) * 2 + ((v >> (e - 1)) & 1))


def range_mask(b: int, a: int) -> int:
    """Buckets of the thresholds c with b < c <= a."""
    lo, hi = bucket(b + 1), bucket(a)
    return ((1 << (hi + 1)) - 1) & ~((1 << lo) - 1)


def balls(n, ends, radius):
    adj = [[] for _ in range(n)]
    for a, b in ends:
        adj[a].append(b)
        adj[b].append(a)
    out = []
    for x in range(n):
        seen, frontier = {x}, [x]
        for _ in range(radius):
            nxt = []
            for y in frontier:
                for z in adj[y]:
                    if z not in seen:
                        seen.add(z)
                        nxt.append(z)
            frontier = nxt
        out.append(seen)
    return out, adj


def run_rules(g, h, rule="lemma4", chunks=1, max_sweeps=200):
    """The sweeps as the GPU runs them; returns the list of H after each sweep."""
    n = g.n
    ends = g.edges().astype(np.int64)
    m = len(ends)
    seq = hindex_sequence(g, h, max_sweeps=1)
    H = seq[0].copy()
    if m == 0:
        return [H]
    eidx = {(int(a), int(b)): i for i, (a, b) in enumerate(ends)}
    Bh1, adj = balls(n, ends.tolist(), h - 1)   # closed (h-1)-balls
    rows = [None] * n
    dmask = [0] * n
    dirty = [True] * n
    out = [H.copy()]
    bounds = [c * n // chunks for c in range(chunks + 1)]
    for sweep in range(max_sweeps):
        first = sweep == 0
        touched, tmin, cmask = set(), {}, [0] * n
        if rule == "keys":
            dmask = [0] * n
        changed = 0
        for c in range(chunks):
            lo, hi = bounds[c], bounds[c + 1]
            for x in range(lo, hi):
                if not dirty[x]:
                    continue
                new = path_keys(n, ends, H, h, x)
                if rule == "keys" and rows[x] is not None:
                    old = rows[x]
                    mk = 0
                    for w in range(n):
                        if old[w] != UNREACHED and new[w] < old[w]:
                            mk |= range_mask(int(new[w]), int(old[w]))
                    dmask[x] = mk
                rows[x] = new
            # edges whose upper endpoint lies in this chunk (all edges when one chunk)
            for i, (u, v) in enumerate(ends):
                if not (lo <= v < hi):
                    continue
                cval = int(H[i])
                if cval == 0:
                    continue
                if not first and not ((dmask[u] | dmask[v]) >> bucket(cval)) & 1:
                    continue
                pu, pv = rows[u], rows[v]
                common = (pu != UNREACHED) & (pv != UNREACHED)
                common[u] = common[v] = False
                y = min(cval, hindex(np.minimum(pu[common], pv[common])))
                if y != cval:
                    H[i] = y
                    changed += 1
                    for z in (int(u), int(v)):
                        touched.add(z)
                        tmin[z] = min(tmin.get(z, 1 << 40), y)
                        cmask[z] |= range_mask(y, cval)
        out.append(H.copy())
        if changed == 0:
            break
        # next sweep's rows
        for x in range(n):
            if h == 1:
                dirty[x] = x in touched
            elif h == 2:
                dirty[x] = x in touched or any(
                    tmin.get(y, 1 << 40) < H[eidx[(min(x, y), max(x, y))]] for y in adj[x])
            else:
                dirty[x] = bool(Bh1[x] & touched)
        if rule == "lemma4":
            dmask = [0] * n
            for x in range(n):
                for y in Bh1[x]:
                    dmask[x] |= cmask[y]
    return out


def random_graph(seed):
    rng = seeded(500 + seed)
    kind = seed % 3
    n = int(rng.integers(8, 40))
    if kind == 0:
        return gen.erdos_renyi(n, float(rng.uniform(0.1, 0.35)), seed=seed)
    if kind == 1:
        return gen.chung_lu(n, float(rng.uniform(3, 8)), float(rng.uniform(2.1, 2.8)), seed=seed)
    return gen.ba_cliques(n + 10, int(rng.integers(2, 4)), 2, (4, 7), seed=seed)


@pytest.mark.parametrize("rule", ["lemma4", "keys"])
@pytest.mark.parametrize("seed", range(12))
def test_synchronous_rules_follow_the_definition(seed, rule):
    g = random_graph(seed)
    for h in (1, 2, 3):
        ref = hindex_sequence(g, h)
        got = run_rules(g, h, rule)
        assert len(got) == len(ref), (seed, h, rule)
        for s, (a, b) in enumerate(zip(got, ref)):
            assert np.array_equal(a, b), (seed, h, rule, s)


@pytest.mark.parametrize("rule", ["lemma4", "keys"])
@pytest.mark.parametrize("seed", range(12))
def test_asynchronous_chunks_reach_the_trussness(seed, rule):
    g = random_graph(seed)
    for h in (1, 2, 3):
        t = decompose(g, h)[0].astype(np.int64)
        got = run_rules(g, h, rule, chunks=4)
        assert np.array_equal(got[-1] + 2, t), (seed, h, rule)
        assert np.array_equal(got[-1], got[-2])


def test_bucket_ranges():
    # the marked buckets of a fall from a to b cover exactly the thresholds in (b, a]
    for b in range(0, 300, 7):
        for a in range(b + 1, 2000, 37):
            mk = range_mask(b, a)
            for c in range(1, 2100, 13):
                marked = (mk >> bucket(c)) & 1
                if b < c <= a:
                    assert marked
