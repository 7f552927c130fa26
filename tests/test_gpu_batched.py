"""GPU parity of the batched and session entry points: every graph's
trussness and round schedule equal the oracle's (small graphs) or the plain
single-graph call's (larger graphs), whatever else shares the GPU."""
import numpy as np
import pytest

import oracle
from graphgen import concat, from_edge_list, gen, workloads as W


pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ht():
    import paper_2411_06405_amd as ht
    return ht


def _mixed_small():
    """Small graphs of every family, mixed h, with an empty and a 2-vertex graph."""
    gs, hs = [], []
    for i, spec in enumerate(W.d4_specs(B=10, seed=3, nrange=(200, 1500))):
        gs.append(W.d4_graph(spec))
        hs.append(spec[2])
    for seed in W.D1_SEEDS[:3]:
        gs.append(W.d1(seed))
        hs.append(1 + seed % 4)
    gs += [gen.complete(7), gen.cycle(9), gen.path(2), from_edge_list(5, [], name="empty5"), gen.star(6)]
    hs += [2, 3, 1, 2, 2]
    gs.append(W.d2(n=1500))
    hs.append(2)
    return gs, hs


def test_batched_equals_oracle():
    gs, hs = _mixed_small()
    b = concat(gs, hs)
    print(f"[gpu] batched B={b.B} total m={int(b.edge_off[-1])}", flush=True)
    ts, rs = _ht().decompose_batch(b)
    for g, h, t, r in zip(gs, hs, ts, rs):
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to), (g.name, h)
        assert np.array_equal(r, ro), (g.name, h)


def _plain(g, h, **kw):
    return _ht().decompose_graph(g, h, **kw)


def test_batched_equals_plain_at_scale():
    specs = W.d4_specs(B=24, seed=7, nrange=(1000, 30000))
    gs = [W.d4_graph(s) for s in specs]
    hs = [s[2] for s in specs]
    b = concat(gs, hs)
    print(f"[gpu] batched B={b.B} total m={int(b.edge_off[-1])}", flush=True)
    ts, rs = _ht().decompose_batch(b)
    for g, h, t, r in zip(gs, hs, ts, rs):
        tp, rp = _plain(g, h)
        assert np.array_equal(t, tp), (g.name, h)
        assert np.array_equal(r, rp), (g.name, h)
    # and the largest against the oracle's certificate on sampled edges
    from tests.gpu_helpers import assert_certified
    big = int(np.argmax([g.m for g in gs]))
    assert_certified(gs[big], hs[big], ts[big], rs[big], 2000)


def test_batched_one_slot_at_a_time():
    # a workspace that holds only the largest graph: graphs run one by one
    import torch
    ht = _ht()
    gs, hs = _mixed_small()
    b = concat(gs, hs)
    one = max(ht.batched_workspace_bytes(np.array([0, g.n], np.uint64),
                                         np.array([0, g.m], np.uint64),
                                         np.array([h], np.uint32)) for g, h in zip(gs, hs))
    ws = torch.empty(one, dtype=torch.uint8, device="cuda")
    ts, rs = ht.decompose_batch(b, workspace=ws)
    for g, h, t, r in zip(gs, hs, ts, rs):
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to) and np.array_equal(r, ro), (g.name, h)


@pytest.mark.parametrize("tune", [{"item_capacity": 64, "event_capacity": 64},
                                  {"flags": 0x4 | 0x8}])
def test_batched_overflow_and_serial_slots_exact(tune):
    # per-slot halts and host-finished rounds (the windowed re-run of an
    # overflowed step) while other slots keep going
    gs, hs = _mixed_small()
    if "flags" in tune:  # every step of every round re-run from the host: keep it small
        keep = [i for i, g in enumerate(gs) if g.m <= 2000][:8]
        gs, hs = [gs[i] for i in keep], [hs[i] for i in keep]
    print(f"[gpu] batched B={len(gs)} {tune}", flush=True)
    b = concat(gs, hs)
    ts, rs = _ht().decompose_batch(b, tune=tune)
    for g, h, t, r in zip(gs, hs, ts, rs):
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to) and np.array_equal(r, ro), (g.name, h, tune)


def test_batched_bad_csr_in_one_graph():
    ht = _ht()
    gs = [W.d1(0), gen.complete(6), W.d1(1)]
    hs = [2, 2, 2]
    b = concat(gs, hs)
    # break graph 1's symmetry: point one of its column ids at a wrong vertex
    s = int(b.adj_off[1])
    b.col_idx_cat[s] = (b.col_idx_cat[s] + 2) % 6
    with pytest.raises(ht.HotrussError) as e:
        ht.decompose_batch(b)
    assert e.value.status == -2


def test_batched_empty_batch():
    ht = _ht()
    b = concat([], [])
    t, r = ht.decompose_batched(b.row_ptr_cat, b.col_idx_cat, b.vtx_off, b.adj_off,
                                b.edge_off, b.h)
    assert t.numel() == 0


# ------------------------------------------------------------------ sessions
def _submit(sess, g, h):
    return sess.submit(g.row_ptr, g.col_idx, g.n, h)


def test_session_alone_vs_mix():
    ht = _ht()
    gs, hs = _mixed_small()
    # alone: each request in a session of its own
    alone = []
    for g, h in zip(gs, hs):
        s = ht.Session(pool_bytes=256 << 20, max_slots=4, max_h=4)
        k = _submit(s, g, h)
        s.progress()
        alone.append(s.result(k))
        s.close()
    # mixed: requests arrive while others run (one graph replay between arrivals)
    s = ht.Session(pool_bytes=256 << 20, max_slots=8, max_h=4)
    tickets = []
    for g, h in zip(gs, hs):
        tickets.append(_submit(s, g, h))
        s.progress(max_graph_launches=1)
    active, queued = s.progress()
    assert active == 0 and queued == 0
    for (g, h), k, (ta, ra) in zip(zip(gs, hs), tickets, alone):
        t, r = s.result(k)
        assert np.array_equal(t, ta) and np.array_equal(r, ra), (g.name, h)
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to) and np.array_equal(r, ro), (g.name, h)
    s.close()


def test_session_budget_and_cancel():
    ht = _ht()
    g = W.d2(n=3000)
    need = ht.batched_workspace_bytes(np.array([0, g.n], np.uint64),
                                      np.array([0, g.m], np.uint64), np.array([2], np.uint32))
    # a pool that fits one such request at a time
    s = ht.Session(pool_bytes=need + need // 2, max_slots=8, max_h=3)
    ks = [_submit(s, g, 2) for _ in range(3)]
    active, queued = s.progress(max_graph_launches=1)
    assert active <= 1 and queued >= 1
    s.cancel(ks[2])
    assert s.status(ks[2]) == -6
    with pytest.raises(ht.HotrussError):
        s.cancel(ks[0])  # already running
    s.progress()
    to, ro, _ = oracle.decompose(g, 2)
    for k in ks[:2]:
        t, r = s.result(k)
        assert np.array_equal(t, to) and np.array_equal(r, ro)
    # larger than the whole pool: rejected at submit
    big = W.d2(n=30000)
    with pytest.raises(ht.HotrussError) as e:
        _submit(s, big, 2)
    assert e.value.status == -5
    # h above the session's bound
    with pytest.raises(ht.HotrussError) as e:
        _submit(s, gen.complete(8), 4)
    assert e.value.status == -1
    s.close()


def test_batched_row_compaction_every_launch_exact():
    gs, hs = _mixed_small()
    b = concat(gs, hs)
    ts, rs = _ht().decompose_batch(b, tune={"flags": _ht()._lib.HO_FLAG_COMPACT_EACH})
    for g, h, t, r in zip(gs, hs, ts, rs):
        to, ro, _ = oracle.decompose(g, h)
        assert np.array_equal(t, to) and np.array_equal(r, ro), (g.name, h)
