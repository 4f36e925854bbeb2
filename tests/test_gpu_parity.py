"""GPU parity: the HIP path (through the C ABI) against the oracle.

Every count is an exact integer, so the bar is equality after every batch:
the tiny Erdos-Renyi workload against stored brute-force counts, random
streams (clean and messy batches) against the static recount of the oracle,
the edge set against the oracle's set semantics, and the region radius
variants against each other.  Radius 1 must fail somewhere (the region is
load-bearing).
"""
import json
import os

import numpy as np
import pytest

from graphgen import (erdos_renyi, er_batches, rmat_graph, rmat_batches, chung_lu_graph,
                      chung_lu_batches, raw_noise_batch, BatchStream)
from oracle import native
from oracle.semantics import apply_batch as oracle_apply, BatchRejected

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def G(*a, **k):
    from paper_2308_14493_amd.graphlet4 import Graph
    return Graph(*a, **k)


def say(*a):
    print(*a, flush=True)


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


def edge_set(src, dst):
    return {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(src, dst)}


def test_er150_golden():
    say("case er150 golden")
    g = json.load(open(os.path.join(HERE, "golden", "er150_counts.json")))
    n = g["n"]
    s, d = erdos_renyi(n, 6 / 149, 0)
    with G(n, s, d) as gr:
        assert gr.counts() == g["counts"][0]
        for i, (b, want) in enumerate(zip(er_batches(n, s, d), g["counts"][1:])):
            got = gr.apply_batch(*b)
            assert got == want, "batch %d" % i
        assert gr.recount() == g["counts"][-1]


def _messy_stream(n, s, d, seed, nb=6):
    rng = np.random.default_rng(seed)
    E = edge_set(s, d)
    out = []
    for i in range(nb):
        if i % 2 == 0:
            es, ed = esorted(E)
            out.append(raw_noise_batch(n, es, ed, int(rng.integers(2, 12)), seed * 100 + i))
        else:
            k = int(rng.integers(1, 30))
            el = sorted(E)
            pick = rng.choice(len(el), min(k, len(el)), replace=False) if el else []
            dsrc = np.array([el[p][0] for p in pick], np.int32)
            ddst = np.array([el[p][1] for p in pick], np.int32)
            out.append((rng.integers(0, n, k).astype(np.int32), rng.integers(0, n, k).astype(np.int32), dsrc, ddst))
        oracle_apply(E, n, *out[-1])
    return out


@pytest.mark.parametrize("radius", [2, 3, 0])
@pytest.mark.parametrize("seed", range(6))
def test_random_streams(seed, radius):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 70))
    p = float(rng.choice([0.05, 0.15, 0.3, 0.6]))
    say("case random n=%d p=%.2f seed=%d radius=%d" % (n, p, seed, radius))
    s, d = erdos_renyi(n, p, seed)
    E = edge_set(s, d)
    with G(n, s, d, radius=radius) as gr:
        assert gr.counts() == native.static_counts(n, s, d)
        for b in _messy_stream(n, s, d, seed):
            got = gr.apply_batch(*b)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            assert got == native.static_counts(n, es, ed)
        gs, gd = gr.edges()
        assert edge_set(gs, gd) == E


@pytest.mark.parametrize("scale,ef,seed", [(9, 8, 1), (11, 8, 2), (12, 16, 3)])
def test_rmat_streams(scale, ef, seed):
    say("case rmat scale=%d ef=%d seed=%d" % (scale, ef, seed))
    n, s, d, samp = rmat_graph(scale, ef, seed)
    sizes = [2, 10, 100, 1000]
    batches = rmat_batches(n, s, d, samp, sizes, seed + 7)
    E = edge_set(s, d)
    with G(n, s, d) as gr:
        assert gr.counts() == native.static_counts(n, s, d)
        for b, sz in zip(batches, sizes):
            got, st = gr.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            say("  batch %d region_v=%d region_e=%d" % (sz, st["region_vertices"], st["region_entries"]))
            assert got == native.static_counts(n, es, ed)
        assert gr.recount() == gr.counts()


@pytest.mark.parametrize("wave_row", [1, 24])
def test_per_vertex_pass_whole_wave_rows(monkeypatch, wave_row):
    """The per-vertex pass deals the rows of 64 vertices over a wave's lanes
    and sends rows of at least wave_row entries (65536 by default) through
    the whole wave.  A low threshold mixes both kinds in most groups (1: every
    nonempty row through the whole wave), for one-batch and three-batch
    passes."""
    monkeypatch.setenv("GC_DEG_WAVE_ROW", str(wave_row))
    say("case per-vertex pass, whole-wave rows >= %d" % wave_row)
    n, s, d, samp = rmat_graph(12, 16, 61)
    batches = rmat_batches(n, s, d, samp, [3, 60, 1500, 20, 400, 7], 62)
    E = edge_set(s, d)
    with G(n, s, d) as gr:
        assert gr.counts() == native.static_counts(n, s, d)
        for b in batches[:3]:
            got = gr.apply_batch(*b)
            oracle_apply(E, n, *b)
            assert got == native.static_counts(n, *esorted(E))
        rows = gr.apply_batch_seq(batches[3:])
        for b, r in zip(batches[3:], rows):
            oracle_apply(E, n, *b)
            want = native.static_counts(n, *esorted(E))
            assert [v & ((1 << 64) - 1) for v in r] == [v & ((1 << 64) - 1) for v in want]
        assert gr.recount() == gr.counts()


def test_chung_lu_small():
    say("case chung-lu n=20000 m=60000")
    n, s, d, _ = chung_lu_graph(20000, 60000, 2.1, 2000.0, 5)
    batches = chung_lu_batches(n, s, d, [10, 300, 3000], 6)
    E = edge_set(s, d)
    with G(n, s, d) as gr:
        assert gr.counts() == native.static_counts(n, s, d)
        for b in batches:
            got = gr.apply_batch(*b)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            assert got == native.static_counts(n, es, ed)


def test_radius_one_is_wrong_somewhere():
    say("case radius-1 negative control")
    bad = 0
    for seed in range(6):
        rng = np.random.default_rng(seed)
        n = 40
        s, d = erdos_renyi(n, 0.12, seed)
        E = edge_set(s, d)
        with G(n, s, d, radius=1) as gr:
            for b in _messy_stream(n, s, d, seed):
                got = gr.apply_batch(*b)
                oracle_apply(E, n, *b)
                es, ed = esorted(E)
                bad += got[:6] != native.static_counts(n, es, ed)[:6]
    assert bad > 0


def test_bad_id_rejected_state_unchanged():
    say("case invalid ids")
    from paper_2308_14493_amd.graphlet4 import GraphletError
    n = 30
    s, d = erdos_renyi(n, 0.2, 3)
    with G(n, s, d) as gr:
        before = gr.counts()
        with pytest.raises(GraphletError) as e:
            gr.apply_batch([1, 2], [3, 30], [], [])
        assert e.value.code == -1
        with pytest.raises(GraphletError):
            gr.apply_batch([], [], [-1], [2])
        assert gr.counts() == before
        assert gr.recount() == before


def test_zero_slack_relocation():
    """slack 0: every insertion moves its row to fresh arena space."""
    say("case zero slack")
    n, s, d, samp = rmat_graph(10, 8, 4)
    batches = rmat_batches(n, s, d, samp, [50, 400, 400, 2000], 9)
    E = edge_set(s, d)
    with G(n, s, d, slack=0.0) as gr:
        for b in batches:
            got = gr.apply_batch(*b)
            oracle_apply(E, n, *b)
        es, ed = esorted(E)
        assert got == native.static_counts(n, es, ed)
        gs, gd = gr.edges()
        assert edge_set(gs, gd) == E


def test_pool_matches_separate():
    say("case pool of 5 graphs")
    from paper_2308_14493_amd.graphlet4 import Graph
    rng = np.random.default_rng(11)
    ns, ss, ds, bs = [], [], [], []
    for i in range(5):
        n, s, d, samp = rmat_graph(int(rng.integers(6, 11)), int(rng.choice([4, 8])), 100 + i)
        ns.append(n); ss.append(s); ds.append(d)
        bs.append(rmat_batches(n, s, d, samp, [int(rng.integers(5, 300))], 200 + i)[0])
    with Graph.pool(ns, ss, ds) as pool:
        for i in range(5):
            assert pool.counts(i) == native.static_counts(ns[i], ss[i], ds[i])
        got = pool.apply_batches(bs)
    for i in range(5):
        E = edge_set(ss[i], ds[i])
        oracle_apply(E, ns[i], *bs[i])
        es, ed = esorted(E)
        assert got[i] == native.static_counts(ns[i], es, ed)


def test_device_arrays_match_host_arrays():
    say("case device-array entry point")
    import torch
    n, s, d, samp = rmat_graph(10, 8, 21)
    bs = rmat_batches(n, s, d, samp, [30, 300], 22)
    with G(n, s, d) as a, G(n, s, d) as b:
        for bt in bs:
            want = a.apply_batch(*bt)
            t = [torch.as_tensor(np.asarray(x, np.int32)).cuda() for x in bt]
            assert b.apply_batch_dev(*t) == want
        from paper_2308_14493_amd.graphlet4 import GraphletError
        t = [torch.tensor([0], dtype=torch.int32).cuda(), torch.tensor([n], dtype=torch.int32).cuda(),
             torch.zeros(0, dtype=torch.int32).cuda(), torch.zeros(0, dtype=torch.int32).cuda()]
        before = b.counts()
        with pytest.raises(GraphletError):
            b.apply_batch_dev(*t)
        assert b.counts() == before == b.recount()


@pytest.mark.parametrize("scale,ef,seed", [(17, 8, 31)])
def test_rmat_large_ids(scale, ef, seed):
    """n above the rank windows of the large 4-cycle tier (8 x 8192), so
    hub work items cover every window and the global tail."""
    say("case rmat scale=%d ef=%d seed=%d (windows + tail)" % (scale, ef, seed))
    n, s, d, samp = rmat_graph(scale, ef, seed)
    sizes = [50, 5000]
    batches = rmat_batches(n, s, d, samp, sizes, seed + 1)
    E = edge_set(s, d)
    with G(n, s, d, delta=-1) as gr:   # region passes: the test asserts on their tiers
        got0, st = gr.counts(), None
        assert got0 == native.static_counts(n, s, d)
        for b in batches:
            got, st = gr.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            say("  tiers c4 large=%d entries=%d" % (st["tier_c4_large"], st["c4_entries_large"]))
            assert st["tier_c4_large"] > 0
            assert got == native.static_counts(n, es, ed)


COMP = [0, 6, 8, 7, 9, 10, 1, 3, 2, 4, 5]   # class of the complement (pinned on the CPU)


@pytest.mark.parametrize("n,p,seed", [(900, 0.05, 41), (1300, 0.03, 42), (1500, 0.02, 45)])
def test_dense_graph_by_complement(n, p, seed):
    """Dense graphs (out-degrees up to ~n) exercise the large-out-degree
    triangle tiers; the oracle counts the sparse complement and the
    complement duality of induced classes maps the result back."""
    say("case dense complement n=%d p=%.2f" % (n, p))
    rng = np.random.default_rng(seed)
    cs, cd = erdos_renyi(n, p, seed)
    comp = edge_set(cs, cd)
    full = {(u, v) for u in range(n) for v in range(u + 1, n)}
    E = full - comp
    s, d = esorted(E)

    def want(Eset):
        c = esorted(full - Eset)
        o = native.static_counts(n, c[0], c[1])
        return [o[COMP[k]] for k in range(11)]

    with G(n, s, d) as gr:
        got, st = gr.counts(), None
        assert got == want(E)
        for k in (40, 400):
            el = sorted(E)
            pick = rng.choice(len(el), k // 2, replace=False)
            du = np.array([el[q][0] for q in pick], np.int32)
            dv = np.array([el[q][1] for q in pick], np.int32)
            iu = rng.integers(0, n, k // 2).astype(np.int32)
            iv = rng.integers(0, n, k // 2).astype(np.int32)
            got, st = gr.apply_batch(iu, iv, du, dv, stats=True)
            oracle_apply(E, n, iu, iv, du, dv)
            say("  max out-degree %d" % st["max_out_degree"])
            assert got == want(E)


@pytest.mark.parametrize("dense_min", [8, 2048, 10**12])
def test_c4_windows_tail_and_wide_counters(monkeypatch, dense_min):
    """Small windows and a low 16-bit threshold force the large 4-cycle tier
    through many windows, the global tail and the 32-bit counter path;
    dense_min moves the switch from dense windows to the tail."""
    monkeypatch.setenv("GC_C4_WINDOW", "128")
    monkeypatch.setenv("GC_C4_NARROW_MAX", "20")
    monkeypatch.setenv("GC_C4_DENSE_MIN", str(dense_min))
    say("case c4 windows 128, narrow <= 20, dense_min %d" % dense_min)
    n, s, d, samp = rmat_graph(13, 16, 51)
    batches = rmat_batches(n, s, d, samp, [100, 2000], 52)
    E = edge_set(s, d)
    with G(n, s, d, delta=-1) as gr:   # region passes: the test asserts on their tiers
        assert gr.counts() == native.static_counts(n, s, d)
        for b in batches:
            got, st = gr.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            say("  c4 large tier %d vertices, tail wedges %d of %d" % (st["tier_c4_large"], st["c4_tail_wedges"],
                                                                    st["wedges"]))
            if dense_min > 8:
                assert st["c4_tail_wedges"] > 0
            assert got == native.static_counts(n, es, ed)


def _two_hub_graph(n, extra, seed):
    """Vertices A and B share the 255 lower neighbours 0..254 (each of those
    also has 20 neighbours in a pool of low-degree vertices), so A and B top
    the degree order, both sit in the large 4-cycle tier and c(B, A) = 255;
    `extra` more neighbours of B lengthen its row."""
    rng = np.random.default_rng(seed)
    A, B = n - 2, n - 1
    pool = np.arange(255, n - 2)
    E = set()
    for l in range(255):
        E.add((l, A))
        E.add((l, B))
        for p in rng.choice(pool, 20, replace=False):
            E.add((l, int(p)))
    for p in pool[:extra]:
        E.add((int(p), B))
    return E, A, B


@pytest.mark.parametrize("extra", [0, 1])
def test_c4_window_field_width_boundary(extra):
    """c(v, w) = 255, the largest value an 8-bit window field holds: every row
    at most 255 long keeps 8-bit windows; one row of 256 entries switches the
    window to 16-bit fields.  Batches then move the row lengths across the
    boundary in both directions, and three-version passes do the same."""
    n = 800
    say("case c4 window field width, row of B = %d" % (255 + extra))
    E, A, B = _two_hub_graph(n, extra, 90 + extra)
    s, d = esorted(E)
    with G(n, s, d, radius=0, delta=-1) as gr:   # region passes: the test asserts on their tiers
        assert gr.counts() == native.static_counts(n, s, d)
        steps = [
            ([(300, A)], []),                     # A: 256 entries
            ([], [(300, A), (0, B)]),             # A back to 255, c(B, A) = 254
            ([(0, B), (301, B), (301, A)], []),   # c(B, A) = 256, both rows 256 or more
            ([], [(301, B), (301, A), (5, A)]),
        ]
        for ins, dels in steps:
            b = tuple(np.array(x, np.int32) for x in ([u for u, v in ins], [v for u, v in ins],
                                                      [u for u, v in dels], [v for u, v in dels]))
            got, st = gr.apply_batch(*b, stats=True)
            assert st["tier_c4_large"] >= 2
            oracle_apply(E, n, *b)
            assert got == native.static_counts(n, *esorted(E))
        seq = [tuple(np.array(x, np.int32) for x in ([310], [B], [7], [A])),
               tuple(np.array(x, np.int32) for x in ([7], [A], [310], [B])),
               tuple(np.array(x, np.int32) for x in ([311, 312], [A, B], [], []))]
        rows = gr.apply_batch_seq(seq)
        for b, r in zip(seq, rows):
            oracle_apply(E, n, *b)
            want = native.static_counts(n, *esorted(E))
            assert [v & ((1 << 64) - 1) for v in r] == [v & ((1 << 64) - 1) for v in want]
        assert gr.recount() == gr.counts()


def test_server_results_same_alone_and_in_the_mix():
    """Requests for three graphs submitted from two host threads, interleaved:
    every ticket's counts equal the counts of the same batch sequence applied
    to a separate handle alone, and the oracle."""
    import threading
    from paper_2308_14493_amd.graphlet4 import Server, Graph
    say("case server mix")
    specs = []
    n, s, d, samp = rmat_graph(10, 8, 61)
    specs.append((n, s, d, rmat_batches(n, s, d, samp, [20, 200, 50, 300], 62)))
    s2, d2 = erdos_renyi(150, 6 / 149, 0)
    specs.append((150, s2, d2, er_batches(150, s2, d2, count=4)))
    n3, s3, d3, _ = chung_lu_graph(5000, 15000, 2.1, 800.0, 63)
    specs.append((n3, s3, d3, chung_lu_batches(n3, s3, d3, [30, 300, 100, 10], 64)))
    alone = []
    for n_, s_, d_, bs in specs:
        with Graph(n_, s_, d_) as g:
            alone.append([g.apply_batch(*b) for b in bs])
    with Server() as srv:
        gids = [srv.add_graph(n_, s_, d_) for n_, s_, d_, _ in specs]
        tickets = {}
        lock = threading.Lock()

        def client(which):
            for j in range(4):
                for gi in which:
                    t = srv.submit(gids[gi], *specs[gi][3][j])
                    with lock:
                        tickets[(gi, j)] = t

        # graph 0 from one thread, graphs 1 and 2 from another (per-graph order kept)
        th = [threading.Thread(target=client, args=([0],)), threading.Thread(target=client, args=([1, 2],))]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for (gi, j), t in sorted(tickets.items()):
            c, st, lat, qms = srv.wait(t)
            assert [int(v) for v in c] == [v & ((1 << 64) - 1) if v < 2**63 else v - 2**64 for v in alone[gi][j]]
            assert lat >= qms >= 0
        for gi in range(3):
            assert srv.counts(gids[gi]) == alone[gi][-1]
    for gi, (n_, s_, d_, bs) in enumerate(specs):
        E = edge_set(s_, d_)
        for b in bs:
            oracle_apply(E, n_, *b)
        es, ed = esorted(E)
        assert alone[gi][-1] == native.static_counts(n_, es, ed)
