"""GPU: gc_apply_batch_dev_noalloc (no allocation in the call; batch staging
in a static device array) against gc_apply_batch_dev, through the C ABI.

* two calls in a row, the second with a smaller batch, on two handles built
  from the same graph: equal counts (exact and int64 view) after each call,
  and equal to the oracle's static recount;
* a batch beyond the static array's limit is refused with the graph unchanged;
* a batch after which a vertex outgrows the counting scratch is undone on the
  device and refused with the graph unchanged; after one allocating call of
  that batch the allocation-free call works again.
"""
import numpy as np
import pytest

from graphgen import rmat_graph, rmat_batches
from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


def dev(b):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32)).cuda() for x in b]


def test_noalloc_equals_dev_two_calls():
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case noalloc vs dev, R-MAT s13")
    n, s, d, samp = rmat_graph(13, 8, 61)
    big, small = rmat_batches(n, s, d, samp, [6000, 700], 62)
    E = set(zip(s.tolist(), d.tolist()))
    with Graph(n, s, d) as a, Graph(n, s, d) as b:
        for j, bt in enumerate((big, small)):
            ga, sa = a.apply_batch_dev(*dev(bt), stats=True)
            gb, sb = b.apply_batch_dev_noalloc(*dev(bt), stats=True)
            oracle_apply(E, n, *bt)
            es, ed = esorted(E)
            want = native.static_counts(n, es, ed)
            say("  call %d: %d updates, equal %s, oracle %s" % (j, bt[0].size + bt[2].size, ga == gb, gb == want))
            assert gb == ga == want
            assert b.last_int64 == a.last_int64
            assert sb["eff_ins"] == sa["eff_ins"] and sb["eff_del"] == sa["eff_del"]
        assert b.recount() == a.counts()


def test_noalloc_limit_refused_unchanged():
    import torch
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case noalloc batch limit")
    n, s, d, samp = rmat_graph(12, 8, 63)
    with Graph(n, s, d) as g:
        before = g.counts()
        k = 262145   # both sides round up to 2^19: the staging exceeds 64 MiB
        rng = np.random.default_rng(64)
        bt = (rng.integers(0, n, k), rng.integers(0, n, k), rng.integers(0, n, k), rng.integers(0, n, k))
        with pytest.raises(GraphletError) as e:
            g.apply_batch_dev_noalloc(*dev(bt))
        assert e.value.code == -1
        assert g.counts() == before and g.recount() == before
        torch.cuda.synchronize()


def hub_growth_with_room():
    """Vertices a = 0 and b = 401 adjacent to each u = 1..400, vertices
    402..411 isolated, plus a path on 412..20411 (room in the region view for
    the batch).  The batch joins every u to 402..411: b then becomes a hub of
    the large 4-cycle tier with 400 lower neighbours, beyond the hub scratch
    sized at build time."""
    n = 20412
    E = {(0, u) for u in range(1, 401)} | {(u, 401) for u in range(1, 401)}
    E |= {(v, v + 1) for v in range(412, 20411)}
    iu = np.repeat(np.arange(1, 401, dtype=np.int32), 10)
    iv = np.tile(np.arange(402, 412, dtype=np.int32), 400)
    return n, E, (iu, iv, np.zeros(0, np.int32), np.zeros(0, np.int32))


def test_noalloc_scratch_growth_undone():
    from paper_2308_14493_amd.graphlet4 import Graph, GraphletError
    say("case noalloc undo")
    n, E, bt = hub_growth_with_room()
    s, d = esorted(E)
    with Graph(n, s, d) as g:
        before = g.counts()
        assert before == native.static_counts(n, s, d)
        with pytest.raises(GraphletError) as e:
            g.apply_batch_dev_noalloc(*dev(bt))
        assert e.value.code == -2 and "undone" in str(e.value)
        assert g.counts() == before and g.recount() == before
        es, ed = g.edges()
        assert {(min(x, y), max(x, y)) for x, y in zip(es.tolist(), ed.tolist())} == E
        got = g.apply_batch_dev(*dev(bt))       # allocating call grows the scratch
        oracle_apply(E, n, *bt)
        assert got == native.static_counts(n, *esorted(E))
        more = (np.array([5, 6], np.int32), np.array([9000, 9001], np.int32),
                np.array([1], np.int32), np.array([402], np.int32))
        got = g.apply_batch_dev_noalloc(*dev(more))
        oracle_apply(E, n, *more)
        assert got == native.static_counts(n, *esorted(E))
