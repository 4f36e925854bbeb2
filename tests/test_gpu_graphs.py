"""GPU parity of passes replayed from captured HIP graphs.

A handle with the graphs option captures the whole pass (upload through
result download) on first use of a pass shape and replays it afterwards.
Every replay is checked against a second handle that launches the same
passes kernel by kernel, and against the oracle; eager work (static
recounts, edge exports, passes of other shapes) and synchronisations run
between the replays.
"""
import numpy as np
import pytest

from graphgen import erdos_renyi, rmat_graph, rmat_batches, raw_noise_batch
from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu


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


def test_replays_equal_direct_launches_small():
    say("case graph replay, ER n=60")
    n = 60
    s, d = erdos_renyi(n, 0.15, 5)
    E = edge_set(s, d)
    rng = np.random.default_rng(6)
    with G(n, s, d, autotune=0, graphs=1) as a, G(n, s, d, autotune=0, graphs=0) as b:
        for i in range(12):
            es, ed = esorted(E)
            bt = raw_noise_batch(n, es, ed, int(rng.integers(2, 20)), 600 + i)
            ga = a.apply_batch(*bt)
            gb = b.apply_batch(*bt)
            oracle_apply(E, n, *bt)
            want = native.static_counts(n, *esorted(E))
            assert ga == gb == want, "batch %d" % i
            if i % 4 == 3:
                assert a.recount() == want          # eager work between replays
                assert edge_set(*a.edges()) == E
        cap, launches = a.graph_replays()
        say("  captures %d launches %d" % (cap, launches))
        assert launches == 12 and cap < launches
        assert b.graph_replays() == (0, 0)


@pytest.mark.parametrize("scale,ef,seed", [(11, 8, 81), (13, 16, 82)])
def test_replays_rmat_mixed_shapes(scale, ef, seed):
    """Batches of three capacity classes interleaved: each class is captured
    once and replayed; multi-version passes are captured too."""
    say("case graph replay rmat scale=%d" % scale)
    n, s, d, samp = rmat_graph(scale, ef, seed)
    sizes = [30, 40, 500, 50, 300, 20, 600, 45, 35, 400]
    batches = rmat_batches(n, s, d, samp, sizes, seed + 1)
    E = edge_set(s, d)
    with G(n, s, d, autotune=0, graphs=1) as a, G(n, s, d, autotune=0, graphs=0) as b:
        for i, bt in enumerate(batches[:6]):
            ga, gb = a.apply_batch(*bt), b.apply_batch(*bt)
            oracle_apply(E, n, *bt)
            assert ga == gb == native.static_counts(n, *esorted(E)), "batch %d" % i
        rest = batches[6:]
        ra = a.apply_batch_seq(rest[:2]) + a.apply_batch_seq(rest[2:])
        rb = b.apply_batch_seq(rest[:2]) + b.apply_batch_seq(rest[2:])
        assert ra == rb
        for bt in rest:
            oracle_apply(E, n, *bt)
        assert a.counts() == b.counts() == native.static_counts(n, *esorted(E))
        assert a.recount() == a.counts()
        cap, launches = a.graph_replays()
        say("  captures %d launches %d" % (cap, launches))
        assert launches == 8 and cap < launches


def test_pool_replays_equal_direct_launches():
    say("case graph replay, pool of 6")
    rng = np.random.default_rng(91)
    ns, ss, ds, samps = [], [], [], []
    for i in range(6):
        n, s, d, samp = rmat_graph(int(rng.integers(6, 11)), int(rng.choice([4, 8])), 300 + i)
        ns.append(n); ss.append(s); ds.append(d); samps.append(samp)
    from paper_2308_14493_amd.graphlet4 import Graph
    Es = [edge_set(ss[i], ds[i]) for i in range(6)]
    with Graph.pool(ns, ss, ds, autotune=0, graphs=1) as a, Graph.pool(ns, ss, ds, autotune=0, graphs=0) as b:
        for r in range(4):
            bs = [rmat_batches(ns[i], *esorted(Es[i]), samps[i], [20], 400 + 10 * r + i)[0] for i in range(6)]
            ga, gb = a.apply_batches(bs), b.apply_batches(bs)
            for i in range(6):
                oracle_apply(Es[i], ns[i], *bs[i])
                assert ga[i] == gb[i] == native.static_counts(ns[i], *esorted(Es[i])), "round %d graph %d" % (r, i)
        cap, launches = a.graph_replays()
        say("  captures %d launches %d" % (cap, launches))
        assert launches == 4 and cap < launches
