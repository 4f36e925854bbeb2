"""GPU: paths that ordinary workloads rarely take, each asserted to be taken
(batch statistics) and checked against the oracle, and the failure path.

* a batch that pushes a vertex past the scratch sized so far: the counting
  stage runs again with more scratch (retries > 0), counts exact;
* the same batch with the retry limit at 0 (GC_RETRY_LIMIT): the call fails
  after the merge has started, and the handle refuses every later call
  (GC_ESTATE) instead of counting on a half-applied graph;
* the global-scratch triangle tier (out-degree above the LDS tiers) and the
  per-version rebuild of a vertex with more version-specific edges than its
  exception list holds, on dense graphs checked through the complement;
* batches at the capacity edges of the one-workgroup sort (4096 keys, and
  one past it), edge-local and region passes.
"""
import numpy as np
import pytest

from graphgen import erdos_renyi
from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu

COMP = [0, 6, 8, 7, 9, 10, 1, 3, 2, 4, 5]   # class of the complement (pinned on the CPU)


def say(*a):
    print(*a, flush=True)


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


def hub_growth_case():
    """Vertices a = 0 and b = 401 adjacent to each of u = 1..400; vertices
    402..411 isolated.  b ranks highest (degree, then id) and has 400 wedges
    (through a), so it is not a hub of the large 4-cycle tier at build time.
    The batch joins every u to each of 402..411: b then has 4400 wedges and
    400 lower neighbours, more than the hub scratch sized so far."""
    n = 420
    E = {(0, u) for u in range(1, 401)} | {(u, 401) for u in range(1, 401)}
    iu = np.repeat(np.arange(1, 401, dtype=np.int32), 10)
    iv = np.tile(np.arange(402, 412, dtype=np.int32), 400)
    return n, E, (iu, iv, np.zeros(0, np.int32), np.zeros(0, np.int32))


def test_scratch_growth_retry_exact(monkeypatch):
    from paper_2308_14493_amd.graphlet4 import Graph
    monkeypatch.delenv("GC_RETRY_LIMIT", raising=False)
    say("case scratch growth retry")
    n, E, b = hub_growth_case()
    s, d = esorted(E)
    with Graph(n, s, d, delta=-1) as g:
        assert g.counts() == native.static_counts(n, s, d)
        got, st = g.apply_batch(*b, stats=True)
        say("  retries %d hubs %d" % (st["retries"], st["tier_c4_large"]))
        assert st["retries"] >= 1 and st["tier_c4_large"] >= 1
        oracle_apply(E, n, *b)
        es, ed = esorted(E)
        assert got == native.static_counts(n, es, ed)
        assert g.recount() == got


def test_failure_after_merge_marks_handle_unusable(monkeypatch):
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case failure after merge")
    n, E, b = hub_growth_case()
    s, d = esorted(E)
    monkeypatch.setenv("GC_RETRY_LIMIT", "0")
    with Graph(n, s, d, delta=-1) as g:
        before = g.counts()
        with pytest.raises(GraphletError) as e1:
            g.apply_batch(*b)
        assert e1.value.code == -3   # GC_EDEVICE
        with pytest.raises(GraphletError) as e2:
            g.apply_batch([1], [2], [], [])
        assert e2.value.code == -5   # GC_ESTATE
        with pytest.raises(GraphletError) as e3:
            g.recount()
        assert e3.value.code == -5
        assert g.counts() == before   # the last good counts stay readable


@pytest.mark.parametrize("n,p,k,seed,what", [(1500, 0.02, 400, 45, "global"), (600, 0.05, 1200, 46, "rebuild")])
def test_dense_fallback_paths(n, p, k, seed, what):
    say("case dense %s n=%d" % (what, n))
    from paper_2308_14493_amd.graphlet4 import Graph
    rng = np.random.default_rng(seed)
    cs, cd = erdos_renyi(n, p, seed)
    comp = {(int(a), int(b)) for a, b in zip(cs, cd)}
    full = {(u, v) for u in range(n) for v in range(u + 1, n)}
    E = full - comp
    s, d = esorted(E)

    def want(Eset):
        c = esorted(full - Eset)
        o = native.static_counts(n, c[0], c[1])
        return [o[COMP[j]] for j in range(11)]

    with Graph(n, s, d, delta=-1) as g:
        el = sorted(E)
        pick = rng.choice(len(el), k // 2, replace=False)
        du = np.array([el[q][0] for q in pick], np.int32)
        dv = np.array([el[q][1] for q in pick], np.int32)
        iu = rng.integers(0, n, k // 2).astype(np.int32)
        iv = rng.integers(0, n, k // 2).astype(np.int32)
        got, st = g.apply_batch(iu, iv, du, dv, stats=True)
        oracle_apply(E, n, iu, iv, du, dv)
        say("  global-tier vertices %d, rebuilds %d, max out-degree %d" %
            (st["tri_global_vertices"], st["tri_exc_rebuilds"], st["max_out_degree"]))
        if what == "global":
            assert st["tri_global_vertices"] > 0
        else:
            assert st["tri_exc_rebuilds"] > 0
        assert got == want(E)


def test_footprint_bounds_real_use_and_admission():
    """The footprint estimate covers what a handle really allocates after
    single- and multi-version passes and a recount; a server whose budget is
    below the real footprint refuses the graph, one at the estimate admits
    it and answers a batch."""
    import torch
    from graphgen import rmat_graph, rmat_batches
    from paper_2308_14493_amd.graphlet4 import Graph, Server, GraphletError, footprint
    say("case footprint")
    n, s, d, samp = rmat_graph(16, 16, 7)
    est = footprint(n, s, d)
    torch.cuda.init()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    g = Graph(n, s, d)
    bs = rmat_batches(n, s, d, samp, [2000] * 5, 8)
    g.apply_batch_seq(bs[:3])
    g.apply_batch(*bs[3])
    g.recount()
    free1 = torch.cuda.mem_get_info()[0]
    g.close()
    real = free0 - free1
    say("  footprint: estimate %.1f MB, measured %.1f MB" % (est / 1e6, real / 1e6))
    assert 0 < real <= est
    with Server(hbm_budget_bytes=real - 1, hbm_reserve_bytes=0) as srv:
        with pytest.raises(GraphletError) as e:
            srv.add_graph(n, s, d)
        assert e.value.code == -2
    with Server(hbm_budget_bytes=est, hbm_reserve_bytes=0) as srv:
        gid = srv.add_graph(n, s, d)
        c, st, lat, q = srv.wait(srv.submit(gid, *bs[4]))
        assert st["eff_ins"] + st["eff_del"] > 0


def test_forced_tier_thresholds_exact():
    """Tier thresholds far below the defaults (tri 16, 4-cycle 32 / 512):
    vertices move to higher tiers, the counts stay those of the oracle after
    every batch, in region and whole-graph passes; the statistics report the
    thresholds; values beyond the kernels' capacities are refused."""
    from graphgen import rmat_graph, rmat_batches
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case forced tier thresholds")
    n, s, d, samp = rmat_graph(12, 16, 71)
    batches = rmat_batches(n, s, d, samp, [40, 400, 3000], 72)
    E = {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(s, d) if a != b}
    for radius in (2, 0):
        Ek = set(E)
        with Graph(n, s, d, delta=-1, radius=radius, tiers=(16, 32, 512)) as g, \
                Graph(n, s, d, delta=-1, radius=radius, autotune=0) as ref:
            es, ed = esorted(Ek)
            assert g.counts() == ref.counts() == native.static_counts(n, es, ed)
            for b in batches:
                got, st = g.apply_batch(*b, stats=True)
                assert ref.apply_batch(*b) == got
                oracle_apply(Ek, n, *b)
                es, ed = esorted(Ek)
                assert got == native.static_counts(n, es, ed)
                assert (st["tri_small_max"], st["c4_small_max"], st["c4_mid_max"]) == (16, 32, 512)
    for bad in ((65, 0, 0), (0, 257, 0), (0, 0, 4097), (0, 200, 100)):
        with pytest.raises(GraphletError) as e:
            Graph(n, s, d, tiers=bad)
        assert e.value.code == -1


def test_tier_trials_autotune_exact():
    """With autotune, passes that count a region after the hub-window
    trials try the five threshold sets in turn, then keep one of them; the
    counts match the oracle throughout."""
    from graphgen import rmat_graph, rmat_batches
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case tier trials")
    n, s, d, samp = rmat_graph(12, 16, 73)
    batches = rmat_batches(n, s, d, samp, [300] * 12, 74)
    E = {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(s, d) if a != b}
    seen = []
    with Graph(n, s, d, delta=-1) as g:
        for b in batches:
            got, st = g.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            assert got == native.static_counts(n, es, ed)
            seen.append((st["tri_small_max"], st["c4_small_max"], st["c4_mid_max"]))
    trials = [(64, 256, 4096), (32, 256, 4096), (64, 128, 4096), (64, 256, 2048), (64, 256, 1024)]
    say("  thresholds per pass %s" % seen)
    # the trials in order (a pass that had to grow scratch repeats its trial)
    tail = seen[5:]
    runs = [t for i, t in enumerate(tail) if i == 0 or t != tail[i - 1]]
    assert runs[:5] == trials
    kept = seen[-1]
    assert kept[0] in (64, 32) and (kept[1], kept[2]) in [(t[1], t[2]) for t in trials]
    assert seen[-2] == kept


@pytest.mark.parametrize("delta", [1, -1])
def test_sort_capacity_edges_exact(delta):
    """Batches whose key counts sit at the edges of the one-workgroup sort:
    2048 + 2048 updates (4096 keys: its capacity, full), 2049 + 2047 (the
    keys and insertions then take the multi-block sort, the deletions the
    small one), one insertion, and deletions only; no self-loops, so every
    update is a key.  Edge-local and region passes, oracle after each."""
    from paper_2308_14493_amd.graphlet4 import Graph
    from graphgen import rmat_graph
    say("case sort capacity edges delta=%d" % delta)
    n, s, d, samp = rmat_graph(12, 8, 77)
    E = set(zip(s.tolist(), d.tolist()))
    rng = np.random.default_rng(78)

    def batch(ni, nd):
        iu = rng.integers(0, n, ni).astype(np.int32)
        iv = ((iu + 1 + rng.integers(0, n - 1, ni)) % n).astype(np.int32)  # never equal to iu
        el = sorted(E)
        pick = rng.choice(len(el), nd, replace=False)
        du = np.array([el[k][1] for k in pick], np.int32)  # reversed orientation on purpose
        dv = np.array([el[k][0] for k in pick], np.int32)
        return iu, iv, du, dv

    with Graph(n, s, d, delta=delta) as g:
        for ni, nd in [(2048, 2048), (2049, 2047), (1, 0), (0, 300), (2048, 2048)]:
            b = batch(ni, nd)
            got = g.apply_batch(*b)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            want = native.static_counts(n, es, ed)
            say("  %d + %d updates: equal %s" % (ni, nd, got == want))
            assert got == want


def test_copy_tuning_skips_trials():
    """gc_copy_tuning: a second handle on the same graph takes over what the
    first one's autotuner learned (its trials done on ten region passes), so
    its first pass already runs with the first handle's knobs; counts stay
    exact on both."""
    from paper_2308_14493_amd.graphlet4 import Graph
    from graphgen import rmat_batches, rmat_graph
    say("case copy tuning")
    n, s, d, samp = rmat_graph(12, 16, 93)
    E = set(zip(s.tolist(), d.tolist()))
    batches = rmat_batches(n, s, d, samp, [300] * 12 + [500], 94)
    with Graph(n, s, d, delta=-1) as a:
        seen = set()
        for b in batches[:12]:
            _, st = a.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            seen.add((st["c4_dense_min"], st["tri_small_max"], st["c4_small_max"], st["c4_mid_max"]))
        assert len(seen) > 1, "the autotuner tried no knobs"
        es, ed = esorted(E)
        with Graph(n, es, ed, delta=-1) as b2:
            b2.copy_tuning(a)
            last = batches[12]
            ga, sa = a.apply_batch(*last, stats=True)
            gb, sb = b2.apply_batch(*last, stats=True)
            oracle_apply(E, n, *last)
            want = native.static_counts(n, *esorted(E))
            knobs = lambda x: (x["c4_dense_min"], x["tri_small_max"], x["c4_small_max"], x["c4_mid_max"])
            say("  knobs seen %s; copied %s, source %s" % (sorted(seen), knobs(sb), knobs(sa)))
            assert ga == want and gb == want
            assert knobs(sb) == knobs(sa)
