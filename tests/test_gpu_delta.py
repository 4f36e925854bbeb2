"""GPU: edge-local passes (gc_options.delta = 1: only the structures that
contain a changed pair are enumerated, with the triangles at every vertex
kept on the device) against the oracle after every batch, and against the
region passes on the same streams.

Cases: messy batches on small dense and sparse random graphs (many changed
pairs inside one triangle, 4-clique or 4-cycle, so the attribution of a
structure to its changed pair of smallest key matters); R-MAT streams with
hubs; dense graphs through the complement duality (4-cliques and diamonds
everywhere); a changed edge between two hubs whose common neighbours
outgrow the first scratch sizes (the stage runs again, counts exact);
region and edge-local passes alternating on one graph (the per-vertex
triangle counts move with both)."""
import numpy as np
import pytest

from graphgen import erdos_renyi, rmat_graph, rmat_batches, raw_noise_batch
from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu

COMP = [0, 6, 8, 7, 9, 10, 1, 3, 2, 4, 5]   # class of the complement (pinned on the CPU)


def say(*a):
    print(*a, flush=True)


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


def messy(n, E, rng, k):
    """k deletions of existing edges, k random insertions, plus noise."""
    el = sorted(E)
    pick = rng.choice(len(el), min(k, len(el)), replace=False) if el else []
    du = [el[q][0] for q in pick] + list(rng.integers(0, n, k // 3))
    dv = [el[q][1] for q in pick] + list(rng.integers(0, n, k // 3))
    iu = list(rng.integers(0, n, k)) + [el[q][1] for q in pick[: k // 4]]
    iv = list(rng.integers(0, n, k)) + [el[q][0] for q in pick[: k // 4]]
    return [np.array(x, np.int32) for x in (iu, iv, du, dv)]


@pytest.mark.parametrize("n,p,k,seed", [(40, 0.3, 30, 1), (60, 0.6, 80, 2), (80, 0.1, 40, 3), (30, 0.9, 60, 4)])
def test_delta_random_messy(n, p, k, seed):
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta random n=%d p=%.1f" % (n, p))
    rng = np.random.default_rng(seed)
    s, d = erdos_renyi(n, p, seed)
    E = set(zip(s.tolist(), d.tolist()))
    with Graph(n, s, d, delta=1) as g:
        for j in range(8):
            b = messy(n, E, rng, k)
            got, st = g.apply_batch(*b, stats=True)
            assert st["delta"] == 1
            oracle_apply(E, n, *b)
            assert got == native.static_counts(n, *esorted(E)), "batch %d" % j
        assert g.recount() == g.counts()


@pytest.mark.parametrize("scale,ef,seed", [(11, 8, 11), (13, 16, 12)])
def test_delta_rmat_vs_region(scale, ef, seed):
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta rmat scale=%d" % scale)
    n, s, d, samp = rmat_graph(scale, ef, seed)
    E = set(zip(s.tolist(), d.tolist()))
    batches = rmat_batches(n, s, d, samp, [10, 100, 1000, 5000, 30], seed + 1)
    with Graph(n, s, d, delta=1) as a, Graph(n, s, d, delta=-1) as b:
        for j, bt in enumerate(batches):
            if j == 2:
                bt = raw_noise_batch(n, *esorted(E), 200, seed + 2)
            ga, sa = a.apply_batch(*bt, stats=True)
            gb = b.apply_batch(*bt)
            oracle_apply(E, n, *bt)
            want = native.static_counts(n, *esorted(E))
            say("  batch %d: %d updates, delta %d, equal %s" % (j, bt[0].size + bt[2].size, sa["delta"], ga == want))
            assert ga == gb == want


@pytest.mark.parametrize("n,p,seed", [(300, 0.08, 21), (500, 0.05, 22)])
def test_delta_dense_by_complement(n, p, seed):
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta dense n=%d" % n)
    rng = np.random.default_rng(seed)
    cs, cd = erdos_renyi(n, p, seed)
    full = {(u, v) for u in range(n) for v in range(u + 1, n)}
    E = full - {(int(x), int(y)) for x, y in zip(cs, cd)}

    def want(Eset):
        c = esorted(full - Eset)
        o = native.static_counts(n, c[0], c[1])
        return [o[COMP[j]] for j in range(11)]

    with Graph(n, *esorted(E), delta=1) as g:
        for k in (6, 60, 600):
            b = messy(n, E, rng, k)
            got = g.apply_batch(*b)
            oracle_apply(E, n, *b)
            assert got == want(E)


def test_delta_hub_pair_scratch_growth():
    """Hubs 0 and 1 with 6000 common neighbours; deleting and re-inserting
    the edge between them needs more common-neighbour and affected-edge
    room than first sized."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta hub pair")
    n = 9000
    E = {(0, 1)} | {(0, w) for w in range(2, 6002)} | {(1, w) for w in range(2, 6002)}
    E |= {(w, w + 1) for w in range(2, 8999)}
    with Graph(n, *esorted(E), delta=1) as g:
        for j, b in enumerate((([], [], [0], [1]), ([1], [0], [], []), ([0, 1], [8500, 8600], [2], [3]))):
            b = [np.array(x, np.int32) for x in b]
            got, st = g.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            say("  retries %d, split edges %d" % (st["retries"], st["k4_split_edges"]))
            assert got == native.static_counts(n, *esorted(E))
            if j < 2:
                # (0, 1) and its 6000 common neighbours: 4-cliques in chunks
                assert st["k4_split_edges"] >= 1


def test_delta_and_region_alternate():
    """Edge-local single batches and two-batch sequences (four-version
    region passes) alternate on one graph."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta/region alternate")
    n, s, d, samp = rmat_graph(12, 8, 31)
    E = set(zip(s.tolist(), d.tolist()))
    with Graph(n, s, d, delta=1) as g:
        for r in range(3):
            bt = rmat_batches(n, *esorted(E), samp, [60, 500, 500], 32 + r)
            got, st = g.apply_batch(*bt[0], stats=True)
            assert st["delta"] == 1
            oracle_apply(E, n, *bt[0])
            assert got == native.static_counts(n, *esorted(E))
            rows = g.apply_batch_seq(bt[1:])
            for b in bt[1:]:
                oracle_apply(E, n, *b)
            assert g.counts() == native.static_counts(n, *esorted(E))


@pytest.mark.parametrize("delta,graphs", [(1, 0), (0, 0), (1, 1), (0, 1)])
def test_delta_pool_matches_oracle(delta, graphs):
    """A pool of graphs of several sizes, one batch per graph per round,
    edge-local (or auto) passes, launched kernel by kernel or replayed from
    captured HIP graphs: every graph equals the oracle."""
    from graphgen import multi_graph_workload
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta pool delta=%d graphs=%d" % (delta, graphs))
    work = multi_graph_workload(count=12, seed=7, n_lo=1e3, n_hi=2e4, b_lo=10, b_hi=2e3)
    pool = Graph.pool([w["n"] for w in work], [w["src"] for w in work], [w["dst"] for w in work], delta=delta,
                      graphs=graphs)
    try:
        Es = [set(zip(w["src"].tolist(), w["dst"].tolist())) for w in work]
        rng = np.random.default_rng(8)
        sizes = [int(x) for x in rng.integers(2, 60, len(work))]
        for r in range(10):
            # the same batch sizes every round: captured passes replay
            bs = [messy(w["n"], E, rng, k) for w, E, k in zip(work, Es, sizes)]
            got = pool.apply_batches(bs)
            for i, (w, E, b) in enumerate(zip(work, Es, bs)):
                oracle_apply(E, w["n"], *b)
                assert got[i] == native.static_counts(w["n"], *esorted(E)), "round %d graph %d" % (r, i)
        say("  captures %d, launches %d" % pool.graph_replays())
    finally:
        pool.close()


def test_delta_pair_room_regrow_keeps_vertex_triangles():
    """Regression: a batch whose 4-cycle pairs outgrow their first room is
    counted again; the per-vertex triangle counts must move once, not once
    per attempt (R-MAT scale 12, ef 16, batches of 3477 updates)."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta pair regrow")
    n, s, d, samp = rmat_graph(12, 16, 1487244190, n=3157)
    E = set(zip(s.tolist(), d.tolist()))
    with Graph(n, s, d, delta=1) as g:
        for j, b in enumerate(rmat_batches(n, s, d, samp, [3477] * 4, 1487244191)):
            got, st = g.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            say("  batch %d retries %d" % (j, st["retries"]))
            assert got == native.static_counts(n, *esorted(E)), "batch %d" % j


def test_delta_tabled_pairs_hash_and_index():
    """4-cycle pairs (e, a) with a short N(a) against the row of a hub: one
    hub of 3000 neighbours (N(a) walked against an LDS hash table of the hub's
    row) and one of 20000 (above the table's 16384 entries: the hub's row
    searched lane by lane), with changed edges at both hubs whose other ends
    have short rows, plus a ring and chords so that the paths s - a - b - hub
    exist; insertions, deletions and re-insertions."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case delta tabled pairs")
    rng = np.random.default_rng(41)
    n = 25000
    E = {(0, w) for w in range(1, 20001)} | {(w, 20001) for w in range(1, 6001, 2)}
    E |= {(w, w + 1) for w in range(1, n - 1)}
    for a, b in rng.integers(1, n, (3000, 2)).tolist():
        if a != b:
            E.add((min(a, b), max(a, b)))
    ins1 = [(21000 + j, 0) for j in range(60)] + [(21500 + j, 20001) for j in range(40)]
    batches = [
        ([u for u, v in ins1], [v for u, v in ins1], [0, 0, 7], [5, 9, 20001]),
        ([0, 20001, 22000], [5, 21003, 0], [21000, 21001, 21502], [0, 0, 20001]),
        ([21000 + j for j in range(0, 60, 3)], [0] * 20, [21000 + j for j in range(1, 60, 3)], [0] * 20),
    ]
    with Graph(n, *esorted(E), delta=1) as g:
        for j, b in enumerate(batches):
            b = [np.array(x, np.int32) for x in b]
            got, st = g.apply_batch(*b, stats=True)
            assert st["delta"] == 1
            oracle_apply(E, n, *b)
            assert got == native.static_counts(n, *esorted(E)), "batch %d" % j
        for j in range(3):
            b = messy(n, E, rng, 200)
            got = g.apply_batch(*b)
            oracle_apply(E, n, *b)
            assert got == native.static_counts(n, *esorted(E)), "messy batch %d" % j
        assert g.recount() == g.counts()
