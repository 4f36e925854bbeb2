"""Host checks of the update streams of the paper's experiments (Sec. 6):
insert-only batches in edge order, and the p-labelled fully dynamic stream
(each negative removes an edge some batches after its positive)."""
import numpy as np

from graphgen import protocol


def test_incremental_batches_cover_edges_in_order():
    n, s, d = protocol.table1_standin("WikiVote", 1, scale_down=8)
    s, d = protocol.edge_order(s, d, 2)
    bs = protocol.incremental_batches(s, d, 10, start=100, count=50)
    assert len(bs) == 50 and all(b[0].size == 10 and b[2].size == 0 for b in bs)
    assert np.array_equal(np.concatenate([b[0] for b in bs]), s[100:600])


def test_fully_dynamic_stream_labels():
    n, s, d = protocol.table1_standin("WikiVote", 1, scale_down=4)
    s, d = protocol.edge_order(s, d, 3)
    u, v, sg = protocol.fully_dynamic_updates(s, d, 0.7, 4, lag=500)
    pos, neg = int((sg > 0).sum()), int((sg < 0).sum())
    # positives ~ p m, negatives ~ (1 - p) of the positives
    assert abs(pos / s.size - 0.7) < 0.02
    assert abs(neg / pos - 0.3) < 0.02
    # every negative follows its positive by at least `lag` positives
    seen = {}
    npos = 0
    for a, b, g in zip(u.tolist(), v.tolist(), sg.tolist()):
        if g > 0:
            seen[(a, b)] = npos
            npos += 1
        else:
            assert (a, b) in seen and npos - seen[(a, b)] > 500 or npos == pos
    bs = protocol.fully_dynamic_batches(s, d, 100, 0.7, 4, lag=500)
    assert all(b[0].size + b[2].size == 100 for b in bs[:-1])
    assert sum(b[2].size for b in bs) == neg
