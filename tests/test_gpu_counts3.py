"""GPU: the induced 3-vertex counts (triangle, 2-path, edge + isolated,
empty) of the resident graph against the oracle (brute force over 3-subsets
where small, else its static recount) after every batch, single graphs (the
pass kind chosen by the library, every batch edge-local, every batch a
region pass) and a pool; at the R-MAT scale-18 size the four counts must add
up to C(n, 3)."""
import math

import numpy as np
import pytest

from graphgen import erdos_renyi, er_batches, rmat_graph, rmat_batches, raw_noise_batch
from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


@pytest.mark.parametrize("delta", [None, 1, -1])
def test_counts3_er150_brute_force(delta):
    from paper_2308_14493_amd.graphlet4 import Graph
    print("case counts3 er150 delta=%s" % delta, flush=True)
    n = 150
    s, d = erdos_renyi(n, 6 / 149, 0)
    E = set(zip(s.tolist(), d.tolist()))
    with Graph(n, s, d, delta=delta) as g:
        assert g.counts3() == native.brute3_counts(n, s, d)
        for b in er_batches(n, s, d):
            g.apply_batch(*b)
            oracle_apply(E, n, *b)
            assert g.counts3() == native.brute3_counts(n, *esorted(E))


@pytest.mark.parametrize("delta", [None, 1, -1])
@pytest.mark.parametrize("scale,ef,seed", [(12, 8, 71), (14, 16, 72)])
def test_counts3_rmat_messy(scale, ef, seed, delta):
    from paper_2308_14493_amd.graphlet4 import Graph
    print("case counts3 rmat scale=%d delta=%s" % (scale, delta), flush=True)
    n, s, d, samp = rmat_graph(scale, ef, seed)
    E = set(zip(s.tolist(), d.tolist()))
    with Graph(n, s, d, delta=delta) as g:
        for k, b in enumerate(rmat_batches(n, s, d, samp, [50, 3000, 20000], seed + 1)):
            if k == 1:
                b = raw_noise_batch(n, *esorted(E), 300, seed + 2)
            g.apply_batch(*b)
            oracle_apply(E, n, *b)
            assert g.counts3() == native.static_counts3(n, *esorted(E))


def test_counts3_pool_and_large_sum():
    from paper_2308_14493_amd.graphlet4 import Graph
    print("case counts3 pool", flush=True)
    gs = [rmat_graph(10 + i, 4 + 4 * i, 80 + i) for i in range(3)]
    pool = Graph.pool([x[0] for x in gs], [x[1] for x in gs], [x[2] for x in gs])
    try:
        for i, (n, s, d, _) in enumerate(gs):
            assert pool.counts3(i) == native.static_counts3(n, s, d)
    finally:
        pool.close()
    n, s, d, _ = rmat_graph(18, 8, 18)
    with Graph(n, s, d) as g:
        c3 = g.counts3()
        assert sum(c3) == math.comb(n, 3) and c3[3] > 0
