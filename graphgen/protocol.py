"""Update streams of the paper's experiments (Sec. 6), on synthetic edge lists.

* Incremental streams: the edges of a graph, in a seeded random order,
  grouped into insert-only batches of a fixed size (Alg. 1, IGC; batches of
  10 and 100 in Figs. 2 and 3).
* Fully dynamic streams: every edge is labelled positive (an insertion) with
  probability p and queued; queued edges are then taken in order and each is
  also labelled negative (a deletion) with probability 1 - p.  The positives
  and negatives are merged into one stream -- a queued edge is taken once a
  fixed number of newer positives (`lag`) have followed it, the reading of
  the paper's "later", so a deletion comes some batches after its
  insertion -- and grouped into batches of a fixed size (Fig. 4: batches of
  100, p = 0.7).  Pairs both inserted and deleted inside one batch are left
  to the batch rules (they cancel).

The SNAP graphs of Table 1 are not available; seeded stand-ins with their
vertex and edge counts come from ``table1_standin``.  Nothing here counts.
"""
from __future__ import annotations

import numpy as np

from .generators import chung_lu_graph, rmat_graph

# Table 1 of the paper: |V|, |E|
TABLE1 = {
    "WikiTalk": (2394385, 4659565),
    "WikiVote": (7115, 100762),
    "Pokec": (1632803, 22301964),
    "LiveJournal": (4033137, 27933062),
}


def table1_standin(name: str, seed: int = 0, scale_down: int = 1):
    """(n, src, dst) shaped like a Table 1 graph: R-MAT (a=0.57, b=0.19,
    c=0.19) for the social networks and WikiVote, Chung-Lu with exponent 2.1
    and hubs of 1e5 for WikiTalk; ``scale_down`` divides |V| and |E|."""
    n, m = TABLE1[name]
    n //= scale_down
    m //= scale_down
    if name == "WikiTalk":
        n_, s, d, _ = chung_lu_graph(n, m, 2.1, min(1e5, n / 4), seed)
    else:
        scale = max(1, int(np.ceil(np.log2(n))))
        n_, s, d, _ = rmat_graph(scale, 0, seed, n=n, m=m)
    return n_, s, d


def edge_order(src, dst, seed):
    """The edges in a seeded random order (the order the stream takes them)."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(len(src))
    return np.asarray(src)[p], np.asarray(dst)[p]


def incremental_batches(src, dst, size, start=0, count=None):
    """Insert-only batches of `size` edges taken in order from position
    `start` of the ordered edge list."""
    end = len(src) if count is None else min(len(src), start + size * count)
    out = []
    for b in range(start, end, size):
        e = min(end, b + size)
        out.append((np.asarray(src[b:e], np.int32), np.asarray(dst[b:e], np.int32),
                    np.zeros(0, np.int32), np.zeros(0, np.int32)))
    return out


def fully_dynamic_updates(src, dst, p, seed, lag=1000):
    """Signed update stream: (u, v, +1) for the positives, (u, v, -1) for the
    negatives, in stream order.  A queued edge is taken from the queue once
    `lag` newer positives have followed it (and the rest at the end), and
    turns negative with probability 1 - p."""
    rng = np.random.default_rng(seed)
    pos = rng.random(len(src)) < p
    neg = rng.random(len(src)) < 1.0 - p   # one draw per queued edge, in queue order
    out_u, out_v, out_s = [], [], []
    queue = []
    head = 0

    def take():
        nonlocal head
        j = queue[head]
        if neg[head]:
            out_u.append(src[j]); out_v.append(dst[j]); out_s.append(-1)
        head += 1

    for i in range(len(src)):
        if not pos[i]:
            continue
        out_u.append(src[i]); out_v.append(dst[i]); out_s.append(1)
        queue.append(i)
        if len(queue) - head > lag:
            take()
    while head < len(queue):
        take()
    return np.asarray(out_u, np.int32), np.asarray(out_v, np.int32), np.asarray(out_s, np.int8)


def fully_dynamic_batches(src, dst, size, p=0.7, seed=0, count=None, lag=1000):
    """Batches of `size` signed updates from fully_dynamic_updates."""
    u, v, sg = fully_dynamic_updates(src, dst, p, seed, lag)
    n = len(u) if count is None else min(len(u), size * count)
    out = []
    for b in range(0, n, size):
        e = min(n, b + size)
        ins = sg[b:e] > 0
        out.append((u[b:e][ins], v[b:e][ins], u[b:e][~ins], v[b:e][~ins]))
    return out
