"""GPU parity at the stated sizes of the workloads, with the library's
default knobs (no environment overrides): the plain per-batch path after
every batch, the scale-22 stream with every batch edge-local or every batch
a region pass, and the pool of 256 graphs in one pass, against counts stored by
tests/golden/make_scale.py, which calls only the oracle (static recount of
the whole graph after every batch) and the input generators.  The inputs are
drawn again here from the same seeds; their digest must equal the stored one
before any count is compared.  Counts are exact integers: the bar is
equality of all eleven classes, and the int64 view (low 64 bits plus the
overflow mask) is checked against the exact value.
"""
import json
import math
import os

import numpy as np
import pytest

from graphgen import workloads as wl

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
INT64_MAX = 2**63 - 1
# edges and 2-paths inside each of the eleven classes (in count order)
E_OF = [3, 3, 4, 4, 5, 6, 3, 2, 2, 1, 0]
W_OF = [2, 3, 4, 5, 8, 12, 3, 1, 0, 0, 0]


def say(*a):
    print(*a, flush=True)


def golden(name):
    return json.load(open(os.path.join(HERE, "golden", name)))


@pytest.fixture(autouse=True)
def default_knobs(monkeypatch):
    for k in ("GC_C4_WINDOW", "GC_C4_NARROW_MAX", "GC_C4_DENSE_MIN", "GC_DEG_WAVE_ROW"):
        monkeypatch.delenv(k, raising=False)


def check_int64(g, want, graph=0):
    out, mask = g.counts_int64(graph)
    for c in range(11):
        lo = want[c] & (2**64 - 1)
        assert int(np.uint64(out[c])) == lo, "class %d low 64 bits" % c
        assert bool(mask >> c & 1) == (want[c] > INT64_MAX), "class %d overflow bit" % c


def run_stream(w, gold, dev_every=0, delta=None):
    from paper_2308_14493_amd.graphlet4 import Graph
    assert wl.workload_digest(w) == gold["input_sha256"], "inputs differ from the stored ones"
    steps = gold["steps"]
    assert steps == list(range(len(w.batches) + 1))
    with Graph(w.n, w.src, w.dst, delta=delta) as g:
        assert g.counts() == gold["counts"][0], "initial counts"
        check_int64(g, gold["counts"][0])
        for j, b in enumerate(w.batches):
            if dev_every and j % dev_every == dev_every - 1:
                import torch
                db = [torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32)).cuda() for x in b]
                got, st = g.apply_batch_dev(*db, stats=True)
            else:
                got, st = g.apply_batch(*b, stats=True)
            say("%s batch %d (%d updates, whole %d, edge-local %d): %s" % (
                w.name, j, b[0].size + b[2].size, st["whole_graph"], st["delta"], got == gold["counts"][j + 1]))
            assert got == gold["counts"][j + 1], "counts after batch %d" % j
            if delta == 1:
                assert st["delta"] == 1
            assert g.info()["m"] == gold["m"][j + 1]
            assert g.last_int64 == [x & (2**64 - 1) for x in got]
            check_int64(g, got)


@pytest.mark.parametrize("delta", [None, 1])
def test_rmat_s18_ef8_every_batch(delta):
    """R-MAT scale 18, ef 8; ten batches each of 1k, 10k and 100k updates;
    every third batch through the device-array entry point; the pass kind
    chosen by the library, or every batch edge-local."""
    say("case rmat_s18_ef8 stream delta=%s" % delta)
    run_stream(wl.rmat_s18_stream(), golden("scale_rmat_s18_ef8.json"), dev_every=3, delta=delta)


@pytest.mark.parametrize("delta", [None, 1])
def test_chung_lu_2_4m_every_batch(delta):
    """Chung-Lu n = 2.4M, m = 5M, gamma 2.1: hubs of tens of thousands of
    neighbours, batches of 1e3, 1e4 and 1e5 degree-proportional updates; the
    pass kind chosen by the library, or every batch edge-local."""
    say("case chung_lu 2.4M/5M stream delta=%s" % delta)
    run_stream(wl.chung_lu_stream(), golden("scale_chung_lu.json"), delta=delta)


@pytest.mark.parametrize("delta", [None, 1])
def test_pool256_one_round(delta):
    """The 256-graph pool: initial counts and the counts after one batch per
    graph in one pooled pass (the pass kind chosen by the library, or
    edge-local), graph by graph."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case pool256 delta=%s" % delta)
    gold = golden("scale_pool256.json")
    graphs = wl.pool256()
    assert wl.pool_digest(graphs) == gold["input_sha256"]
    pool = Graph.pool([x["n"] for x in graphs], [x["src"] for x in graphs], [x["dst"] for x in graphs], delta=delta)
    try:
        for i in range(len(graphs)):
            assert pool.counts(i) == gold["counts_initial"][i], "graph %d initial" % i
        got = pool.apply_batches([x["batch"] for x in graphs])
        bad = [i for i in range(len(graphs)) if got[i] != gold["counts_after"][i]]
        assert not bad, "graphs with wrong counts after the batch: %s" % bad[:10]
        over = 0
        for i in range(len(graphs)):
            check_int64(pool, got[i], i)
            over += got[i][10] > INT64_MAX
        say("pool256: %d graphs with the empty class beyond int64" % over)
        assert over > 0
    finally:
        pool.close()


@pytest.fixture(scope="module")
def s22_stream():
    w, _, _ = wl.rmat_s22_bench_stream(total=25)
    return w


@pytest.mark.parametrize("delta", [1, -1])
def test_rmat_s22_stream_one_pass_kind(s22_stream, delta):
    """R-MAT scale 22, ef 16 (n = 4,194,304, m = 67,108,864) and its 25
    batches of log-uniform size in [10, 1e5], every batch through the same
    kind of pass (1: edge-local, also for batches of 57,032 updates; -1:
    region or whole-graph), against the oracle's counts before and after
    the stream."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case rmat_s22 stream delta=%d" % delta)
    w = s22_stream
    gold = golden("scale_rmat_s22_bench.json")
    assert gold["steps"] == [0, 25]
    assert wl.prefix_digest(w, 0) == gold["prefix_sha256"][0], "graph differs from the stored one"
    assert wl.prefix_digest(w, 25) == gold["prefix_sha256"][1], "batches differ from the stored ones"
    n = w.n
    with Graph(n, w.src, w.dst, delta=delta) as g:
        assert g.counts() == gold["counts"][0], "initial counts"
        for j, b in enumerate(w.batches):
            got, st = g.apply_batch(*b, stats=True)
            assert st["delta"] == (1 if delta == 1 else 0)
            # between the stored points, identities that hold for any graph:
            # the classes partition the 4-subsets, and each edge lies in
            # C(n-2, 2) of them
            m = g.info()["m"]
            assert sum(got) == math.comb(n, 4), "batch %d: sum" % j
            assert sum(e * x for e, x in zip(E_OF, got)) == m * math.comb(n - 2, 2), "batch %d: edges" % j
        say("  after %d batches: equal %s" % (len(w.batches), got == gold["counts"][1]))
        assert got == gold["counts"][1], "counts after the stream"
        assert g.info()["m"] == gold["m"][1]
        check_int64(g, got)
        # each 2-path lies in n - 3 of the 4-subsets; W from the exported edges
        es, ed = g.edges()
        deg = np.bincount(es, minlength=n).astype(np.int64) + np.bincount(ed, minlength=n)
        W = int((deg * (deg - 1) // 2).sum())
        assert sum(x * c for x, c in zip(W_OF, got)) == W * (n - 3)
