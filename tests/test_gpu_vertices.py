"""GPU parity of vertex insertion and deletion (Sec. 3: vertex operations
reduce to edge operations; a vertex loses its incident edges before it
leaves V) against the oracle: after every step, the counts equal the
oracle's static recount of the live vertices relabelled onto 0 .. |V| - 1,
and the exported edge set equals the oracle's.  Covers additions within the
reserved id capacity and beyond it (the graph is rebuilt over a larger id
space), removals of hubs, new vertices and isolated vertices, rejection of
removed and unissued ids on every entry point, and the edge-local and
region passes."""
import numpy as np
import pytest

from graphgen import rmat_graph
from oracle import native
from oracle.semantics import apply_batch as oracle_apply, compact, remove_vertices as oracle_remove

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def edge_set(src, dst):
    return {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(src, dst)}


def want(E, live):
    return native.static_counts(*compact(E, live))


def want3(E, live):
    return native.static_counts3(*compact(E, live))


def rand_batch(rng, E, pool, n_ins, n_del, hot=None):
    """Insertions between random vertices of `pool` (one endpoint from `hot`
    when given), deletions of random existing edges."""
    pool = np.asarray(sorted(pool), np.int32)
    a = rng.choice(pool, n_ins)
    b = rng.choice(np.asarray(sorted(hot), np.int32) if hot else pool, n_ins)
    El = sorted(E)
    pick = rng.choice(len(El), min(n_del, len(El)), replace=False) if El else []
    du = np.array([El[i][0] for i in pick], np.int32)
    dv = np.array([El[i][1] for i in pick], np.int32)
    return a.astype(np.int32), b.astype(np.int32), du, dv


@pytest.mark.parametrize("delta", [0, 1, -1])
def test_vertex_stream(delta):
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case vertex stream delta=%d" % delta)
    rng = np.random.default_rng(100 + delta)
    n, s, d, _ = rmat_graph(11, 8, 7)
    E = edge_set(s, d)
    E = {e for e in E if e[0] != e[1]}
    live = set(range(n))
    with Graph(n, s, d, delta=delta, vertex_capacity=n + 64) as gr:
        assert gr.counts() == want(E, live)
        # additions within the capacity
        first, c = gr.add_vertices(50)
        assert first == n
        new = set(range(n, n + 50))
        live |= new
        assert c == want(E, live) and gr.info()["n"] == len(live)
        b = rand_batch(rng, E, live, 300, 100, hot=new)
        got = gr.apply_batch(*b)
        oracle_apply(E, n + 50, *b)
        assert got == want(E, live)
        # removals: hubs, new vertices, isolated ones
        deg = {}
        for u, v in E:
            deg[u] = deg.get(u, 0) + 1
            deg[v] = deg.get(v, 0) + 1
        hubs = sorted(deg, key=lambda x: -deg[x])[:5]
        newbies = sorted(new - set(hubs))[:3]
        isolated = [x for x in sorted(live) if x not in deg and x not in newbies][:2]
        gone = hubs + newbies + isolated
        inc = sum(1 for u, v in E if u in gone or v in gone)
        got, st = gr.remove_vertices(gone, stats=True)
        oracle_remove(E, live, gone)
        assert got == want(E, live)
        assert st["eff_del"] == inc and st["eff_ins"] == 0
        assert gr.info()["n"] == len(live) and gr.info()["m"] == len(E)
        assert gr.counts3() == want3(E, live)
        # removed and unissued ids are rejected, state unchanged
        before = gr.counts()
        for bad in ([hubs[0]], [n + 50]):
            with pytest.raises(GraphletError) as e:
                gr.apply_batch([bad[0]], [1 if bad[0] != 1 else 2], [], [])
            assert e.value.code == -1
            with pytest.raises(GraphletError):
                gr.apply_batch([], [], bad, [3])
        for bad in ([hubs[0]], [hubs[1], hubs[1]], [n + 50], [-1]):
            with pytest.raises(GraphletError) as e:
                gr.remove_vertices(bad)
            assert e.value.code == -1
        assert gr.counts() == before and gr.recount() == before
        # additions beyond the capacity: rebuilt over a larger id space
        first, c = gr.add_vertices(200)
        assert first == n + 50
        new2 = set(range(n + 50, n + 250))
        live |= new2
        assert c == want(E, live)
        assert edge_set(*gr.edges()) == E
        for j in range(3):
            b = rand_batch(rng, E, live, 400, 150, hot=new2)
            got = gr.apply_batch(*b)
            oracle_apply(E, n + 250, *b)
            assert got == want(E, live), j
        assert gr.recount() == gr.counts()
        # removed ids stay rejected after the rebuild
        with pytest.raises(GraphletError):
            gr.apply_batch([hubs[2]], [first], [], [])
        gone2 = sorted(rng.choice(sorted(live), 40, replace=False).tolist())
        got = gr.remove_vertices(gone2)
        oracle_remove(E, live, gone2)
        assert got == want(E, live)
        assert edge_set(*gr.edges()) == E
        # several batches in one call: checked as a whole
        bs = [rand_batch(rng, E, live, 60, 20) for _ in range(3)]
        bad = list(bs[2])
        bad[0] = np.concatenate([bad[0], np.array([gone2[0]], np.int32)])
        bad[1] = np.concatenate([bad[1], np.array([first], np.int32)])
        with pytest.raises(GraphletError):
            gr.apply_batch_seq(bs[:2] + [tuple(bad)])
        outs = gr.apply_batch_seq(bs)
        for j, b in enumerate(bs):
            oracle_apply(E, n + 250, *b)
            assert outs[j] == want(E, live), j


def test_vertex_device_paths():
    """Device-array and allocation-free batches reject removed ids too."""
    import torch
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case vertex device paths")
    rng = np.random.default_rng(5)
    n, s, d, _ = rmat_graph(10, 8, 3)
    E = {e for e in edge_set(s, d) if e[0] != e[1]}
    live = set(range(n))
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.asarray(a, np.int32), device=dev).contiguous()
    with Graph(n, s, d) as gr:
        gone = [0, 5, 17]
        got = gr.remove_vertices(gone)
        oracle_remove(E, live, gone)
        assert got == want(E, live)
        # one device-array batch first: it sizes the handle's buffers for
        # batches of this size, which the allocation-free call requires
        b = rand_batch(rng, E, live, 100, 40)
        got = gr.apply_batch_dev(*[t(x) for x in b])
        oracle_apply(E, n, *b)
        assert got == want(E, live)
        before = gr.counts()
        for fn in (gr.apply_batch_dev, gr.apply_batch_dev_noalloc):
            with pytest.raises(GraphletError) as e:
                fn(t([1, 2]), t([3, 5]), t([]), t([]))
            assert e.value.code == -1
            with pytest.raises(GraphletError) as e:
                fn(t([]), t([]), t([17]), t([2]))
            assert e.value.code == -1
            assert gr.counts() == before
        for fn in (gr.apply_batch_dev, gr.apply_batch_dev_noalloc):
            b = rand_batch(rng, E, live, 100, 40)
            got = fn(*[t(x) for x in b])
            oracle_apply(E, n, *b)
            assert got == want(E, live)
        assert gr.recount() == gr.counts()


def test_vertex_degenerate():
    """Removing down to fewer than four vertices, and to none; additions to
    an emptied graph; count 0; pools refuse vertex operations."""
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case vertex degenerate")
    n = 8
    s = np.array([0, 1, 2, 3, 4, 5, 0], np.int32)
    d = np.array([1, 2, 3, 4, 5, 6, 2], np.int32)
    E = edge_set(s, d)
    live = set(range(n))
    with Graph(n, s, d) as gr:
        first, c = gr.add_vertices(0)
        assert first == n and c == want(E, live)
        for gone in ([7, 6, 5], [4, 3], [2], [1, 0]):
            got = gr.remove_vertices(gone)
            oracle_remove(E, live, gone)
            assert got == want(E, live) and gr.counts3() == want3(E, live)
        assert gr.info()["n"] == 0 and gr.info()["m"] == 0
        first, c = gr.add_vertices(6)
        assert first == n
        live |= set(range(n, n + 6))
        b = (np.array([8, 9, 10, 8], np.int32), np.array([9, 10, 11, 11], np.int32), [], [])
        got = gr.apply_batch(*b)
        oracle_apply(E, n + 6, *b)
        assert got == want(E, live)
        with pytest.raises(GraphletError):
            gr.apply_batch([0], [8], [], [])
    with Graph.pool([10, 12], [s, s], [d, d]) as pool:
        with pytest.raises(GraphletError):
            pool.add_vertices(1)
        with pytest.raises(GraphletError):
            pool.remove_vertices([1])


def test_vertex_ops_rmat_s16():
    """R-MAT scale 16 (65,536 vertices, hubs of thousands of edges): vertex
    additions within the reserved ids, a batch on the new vertices, removal
    of the 50 largest hubs (one deletion batch of tens of thousands of
    edges), growth past the reservation, then a large mixed batch; the
    counts equal the oracle's after every step."""
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case vertex ops R-MAT s16")
    rng = np.random.default_rng(16)
    n, s, d, _ = rmat_graph(16, 8, 11)
    E = {e for e in edge_set(s, d) if e[0] != e[1]}
    live = set(range(n))
    with Graph(n, s, d, vertex_capacity=n + 500) as gr:
        assert gr.counts() == want(E, live)
        first, c = gr.add_vertices(300)
        new = set(range(first, first + 300))
        live |= new
        assert c == want(E, live)
        b = rand_batch(rng, E, live, 2000, 1000, hot=new)
        got = gr.apply_batch(*b)
        oracle_apply(E, n + 300, *b)
        assert got == want(E, live)
        deg = {}
        for u, v in E:
            deg[u] = deg.get(u, 0) + 1
            deg[v] = deg.get(v, 0) + 1
        hubs = sorted(deg, key=lambda x: -deg[x])[:50]
        got, st = gr.remove_vertices(hubs, stats=True)
        inc = sum(1 for u, v in E if u in hubs or v in hubs)
        oracle_remove(E, live, hubs)
        say("  removed 50 hubs: %d edges" % inc)
        assert st["eff_del"] == inc and got == want(E, live)
        first2, c = gr.add_vertices(1000)
        assert first2 == first + 300
        live |= set(range(first2, first2 + 1000))
        assert c == want(E, live)
        b = rand_batch(rng, E, live, 5000, 5000)
        got = gr.apply_batch(*b)
        oracle_apply(E, first2 + 1000, *b)
        assert got == want(E, live)
        assert gr.recount() == got
        assert edge_set(*gr.edges()) == E
