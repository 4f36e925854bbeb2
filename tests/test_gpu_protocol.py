"""GPU: the paper's experimental protocol (Sec. 6) on a WikiVote-shaped
stand-in, checked against the oracle after every batch: insert-only batches
of 10 and of 100 from the empty graph (Alg. 1: passes without deletions take
the insert-only path), and fully dynamic batches of 100 with the p = 0.7
labelling (Alg. 2), each with edge-local and region passes."""
import numpy as np
import pytest

from graphgen import protocol
from oracle import native
from oracle.semantics import apply_batch as oracle_apply

pytestmark = pytest.mark.gpu


def esorted(E):
    E = sorted(E)
    return (np.array([u for u, v in E], np.int32), np.array([v for u, v in E], np.int32))


@pytest.mark.parametrize("kind,size,delta", [("insert", 10, 1), ("insert", 100, -1), ("insert", 100, 0),
                                             ("dynamic", 100, 1), ("dynamic", 100, -1)])
def test_protocol_from_empty(kind, size, delta):
    from paper_2308_14493_amd.graphlet4 import Graph
    print("case protocol %s size %d delta %d" % (kind, size, delta), flush=True)
    n, s, d = protocol.table1_standin("WikiVote", 5, scale_down=2)
    s, d = protocol.edge_order(s, d, 6)
    if kind == "insert":
        batches = protocol.incremental_batches(s, d, size, count=60)
    else:
        batches = protocol.fully_dynamic_batches(s[:8000], d[:8000], size, 0.7, 7, count=60, lag=1000)
    E = set()
    with Graph(n, [], [], delta=delta) as g:
        for j, b in enumerate(batches):
            got, st = g.apply_batch(*b, stats=True)
            oracle_apply(E, n, *b)
            if kind == "insert":
                assert st["eff_del"] == 0
            if j % 6 == 5 or j == len(batches) - 1:
                assert got == native.static_counts(n, *esorted(E)), "batch %d" % j
        assert g.recount() == g.counts()
        assert g.info()["m"] == len(E)
