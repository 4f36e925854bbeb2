"""ORACLE -- test infrastructure.  Set-based reference of the paper's Alg. 2.

FDGC (Sec. 4.5, Alg. 2): for a batch B = A u D,
    H   = union over changed edges e = (u, v) of G[N_r(u) u N_r(v)]
    G_a = (H - D) u A,    G_b = (H - A) u D
    F  += PGD(G_a) - PGD(G_b)
    G   = G - D u A
with F the six connected induced 4-graphlet counts (Fig. 1), starting from
F = 0 on the empty graph.  The paper takes r = 3 (a 4-vertex graphlet has
diameter at most 3, Sec. 4.3).  Lemma 2 states that F then equals a recount
of the updated graph.

The batch is first reduced to its effective part (semantics.py): Sec. 6
cancels pairs that are both added and deleted; an insertion of an existing
edge or a deletion of a missing one is not a change.

``region`` selects how H is formed, for the tests that probe Lemma 2:
    "paper"      union of the induced balls, as written in Alg. 2
    "induced"    the subgraph induced on the union of the balls (a superset)
    "whole"      the whole graph (the largest induced superset)
    "tree"       only the BFS-tree edges of each ball (not induced; a
                 deliberately wrong region used as a negative control)
The local counter is any exact static counter of connected induced
4-graphlets (brute force or the static recount), applied to a graph
relabelled onto 0..k-1.
"""
from __future__ import annotations

from collections import deque

from . import native
from .semantics import apply_batch, canon


def _adj(E):
    adj = {}
    for u, v in E:
        adj.setdefault(u, set()).add(v)
        adj.setdefault(v, set()).add(u)
    return adj


def _ball(adj, src, r):
    """Vertices within r hops of any vertex in src (BFS), plus tree edges."""
    dist = {s: 0 for s in src}
    tree = set()
    q = deque(src)
    while q:
        x = q.popleft()
        if dist[x] == r:
            continue
        for y in adj.get(x, ()):
            if y not in dist:
                dist[y] = dist[x] + 1
                tree.add(canon(x, y))
                q.append(y)
    return set(dist), tree


def _induced(E, S):
    return {(u, v) for (u, v) in E if u in S and v in S}


def _connected_counts(edges):
    """Connected induced 4-graphlet counts of an edge set (relabelled)."""
    verts = sorted({x for e in edges for x in e})
    if len(verts) < 4:
        return [0] * 6
    idx = {x: i for i, x in enumerate(verts)}
    src = [idx[u] for u, v in edges]
    dst = [idx[v] for u, v in edges]
    k = len(verts)
    if k <= 64:
        c = native.brute_counts(k, src, dst)
    else:
        c = native.static_counts(k, src, dst)
    return c[:6]


class FDGCRef:
    def __init__(self, n, src=(), dst=(), radius=3, region="paper"):
        self.n = n
        self.E = set()
        self.F = [0] * 6
        self.radius = radius
        self.region = region
        if len(src):
            self.apply(src, dst, [], [])

    def _region(self, A, D):
        G = self.E
        if self.region == "whole":
            return set(G)
        adj = _adj(G)
        H = set()
        if self.region == "induced":
            S = set()
            for (u, v) in A | D:
                b, _ = _ball(adj, [u, v], self.radius)
                S |= b
            return _induced(G, S)
        for (u, v) in A | D:
            b, tree = _ball(adj, [u, v], self.radius)
            if self.region == "paper":
                H |= _induced(G, b)
            elif self.region == "tree":
                H |= tree
            else:
                raise ValueError(self.region)
        return H

    def apply(self, ins_src, ins_dst, del_src, del_dst):
        """One FDGC step; returns the six connected counts after the batch."""
        from .semantics import effective_batch
        A, D, st = effective_batch(self.E, self.n, ins_src, ins_dst, del_src, del_dst)
        H = self._region(A, D)
        Ga = (H - D) | A
        Gb = (H - A) | D
        Ca = _connected_counts(Ga)
        Cb = _connected_counts(Gb)
        self.F = [f + a - b for f, a, b in zip(self.F, Ca, Cb)]
        self.E -= D
        self.E |= A
        return list(self.F)


__all__ = ["FDGCRef", "apply_batch"]
