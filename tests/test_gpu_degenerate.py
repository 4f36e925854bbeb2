"""GPU parity on the degenerate inputs of the method: graphs of one to seven
vertices (below four vertices every count is zero), built with no edges,
then empty batches, batches that insert every pair, batches that change
nothing (only self-loops, pairs already present, missing pairs deleted,
pairs both inserted and deleted in the same batch), batches that delete
every edge, and batches that rebuild a path; edge-local and region passes,
the oracle after every batch, the GPU recount and the edge export at the
end."""
import itertools

import numpy as np
import pytest

from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu

Z = np.zeros(0, np.int32)


def say(*a):
    print(*a, flush=True)


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


def arr(x):
    return np.array(x, np.int32)


def stream(n):
    """The batch sequence for a graph of n vertices (ids 0..n-1)."""
    pairs = list(itertools.combinations(range(n), 2))
    every_u, every_v = arr([u for u, v in pairs]), arr([v for u, v in pairs])
    loops = arr(list(range(n)))
    out = [
        (Z, Z, Z, Z),                                               # empty
        (loops, loops, Z, Z),                                       # self-loops only
        (every_v, every_u, Z, Z),                                   # every pair, reversed orientation
        (every_u, every_u, loops, loops),                           # loops inserted and deleted
        (every_u, every_v, Z, Z),                                   # every pair again: nothing new
        (every_u, every_v, every_v, every_u),                       # each pair in both lists: cancelled
        (Z, Z, every_u, every_v),                                   # every edge deleted
        (Z, Z, every_u, every_v),                                   # deleting missing pairs
        (arr(list(range(n - 1))), arr(list(range(1, n))), Z, Z),    # a path
        (Z, Z, Z, Z),                                               # empty again
    ]
    if n >= 4:
        # a 4-cycle closed and a chord swapped in one batch
        out.append((arr([0, 1]), arr([3, 3]), arr([2]), arr([3])))
    return out


@pytest.mark.parametrize("delta", [1, -1])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7])
def test_tiny_graphs_every_batch_kind(n, delta):
    from paper_2308_14493_amd.graphlet4 import Graph
    say("case degenerate n=%d delta=%d" % (n, delta))
    E = set()
    with Graph(n, Z, Z, delta=delta) as g:
        assert g.counts() == native.static_counts(n, Z, Z)
        for j, b in enumerate(stream(n)):
            got = g.apply_batch(*b)
            oracle_apply(E, n, *b)
            es, ed = esorted(E)
            want = native.static_counts(n, es, ed)
            say("  batch %d: %d + %d updates, m = %d, equal %s" % (j, b[0].size, b[2].size, len(E), got == want))
            assert got == want
        assert g.recount() == g.counts()
        gs, gd = g.edges()
        assert {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(gs, gd)} == E
