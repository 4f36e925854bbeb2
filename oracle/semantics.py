"""ORACLE -- test infrastructure.  Batch semantics on a Python edge set.

The stream model (Sec. 3) applies a tuple <e, o> by set union (o = +) or set
difference (o = -); Problem 1 maintains the counts of
G^{t+1} = (V, E^t + A - D) for a batch B = A u D of a simple undirected graph.
Sec. 6 first removes the edges that are both added and deleted in a batch and
runs the algorithm on the rest.  Together:

  * (u, v) and (v, u) are the same edge; self loops are not edges (dropped);
  * repeats inside A, and inside D, collapse (set semantics);
  * a pair in both A and D is removed from the batch (unchanged);
  * inserting an existing edge or deleting a missing one changes nothing,
    so the effective batch is A' = A - E^t, D' = D & E^t;
  * an id outside [0, n) rejects the whole batch (V is fixed).
"""
from __future__ import annotations


class BatchRejected(ValueError):
    pass


def canon(u, v):
    u, v = int(u), int(v)
    return (u, v) if u < v else (v, u)


def effective_batch(E: set, n: int, ins_src, ins_dst, del_src, del_dst):
    """Returns (A', D', stats) without modifying E."""
    for arr in (ins_src, ins_dst, del_src, del_dst):
        for x in arr:
            if int(x) < 0 or int(x) >= n:
                raise BatchRejected("vertex id out of range")
    stats = dict(offered_ins=len(ins_src), offered_del=len(del_src), loops=0)
    A, D = set(), set()
    for u, v in zip(ins_src, ins_dst):
        if int(u) == int(v):
            stats["loops"] += 1
            continue
        A.add(canon(u, v))
    for u, v in zip(del_src, del_dst):
        if int(u) == int(v):
            stats["loops"] += 1
            continue
        D.add(canon(u, v))
    both = A & D
    A -= both
    D -= both
    stats["cancelled"] = len(both)
    Ae = {e for e in A if e not in E}
    De = {e for e in D if e in E}
    stats["ins_existing"] = len(A) - len(Ae)
    stats["del_missing"] = len(D) - len(De)
    stats["eff_ins"] = len(Ae)
    stats["eff_del"] = len(De)
    return Ae, De, stats


def apply_batch(E: set, n: int, ins_src, ins_dst, del_src, del_dst):
    """E <- E - D' + A' in place; returns (A', D', stats)."""
    A, D, st = effective_batch(E, n, ins_src, ins_dst, del_src, del_dst)
    E -= D
    E |= A
    return A, D, st


# ---------------------------------------------------------------- arrays ---
# The same rules on sorted arrays of pair keys (min << 32 | max, uint64), for
# graphs too large for a Python set.  Every step names the rule it applies.

def _keys(u, v):
    import numpy as np
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    return ((lo << 32) | hi).astype(np.uint64), u != v


def _member(sorted_keys, q):
    import numpy as np
    if sorted_keys.size == 0 or q.size == 0:
        return np.zeros(q.shape, dtype=bool)
    pos = np.minimum(np.searchsorted(sorted_keys, q), sorted_keys.size - 1)
    return sorted_keys[pos] == q


def effective_batch_keys(E_keys, n: int, ins_src, ins_dst, del_src, del_dst):
    """effective_batch on a sorted uint64 key array E_keys (not modified).
    Returns (A' keys, D' keys, stats), both sorted."""
    import numpy as np
    for arr in (ins_src, ins_dst, del_src, del_dst):
        a = np.asarray(arr, dtype=np.int64)
        if a.size and (a.min() < 0 or a.max() >= n):
            raise BatchRejected("vertex id out of range")
    ka, keep_a = _keys(ins_src, ins_dst)          # (u, v) and (v, u) are one edge
    kd, keep_d = _keys(del_src, del_dst)
    stats = dict(offered_ins=len(ins_src), offered_del=len(del_src),
                 loops=int((~keep_a).sum() + (~keep_d).sum()))
    A = np.unique(ka[keep_a])                     # loops dropped, repeats collapse
    D = np.unique(kd[keep_d])
    both = np.intersect1d(A, D, assume_unique=True)
    A = np.setdiff1d(A, both, assume_unique=True)  # a pair in A and D is dropped
    D = np.setdiff1d(D, both, assume_unique=True)
    stats["cancelled"] = int(both.size)
    Ae = A[~_member(E_keys, A)]                   # no-op insertions / deletions
    De = D[_member(E_keys, D)]
    stats["ins_existing"] = int(A.size - Ae.size)
    stats["del_missing"] = int(D.size - De.size)
    stats["eff_ins"] = int(Ae.size)
    stats["eff_del"] = int(De.size)
    return Ae, De, stats


def apply_batch_keys(E_keys, n: int, ins_src, ins_dst, del_src, del_dst):
    """Returns (E - D' + A' as a sorted key array, stats)."""
    import numpy as np
    A, D, st = effective_batch_keys(E_keys, n, ins_src, ins_dst, del_src, del_dst)
    kept = E_keys[~_member(D, E_keys)]
    return np.union1d(kept, A).astype(np.uint64), st


def keys_to_pairs(E_keys):
    """Sorted key array -> (src, dst) int32 arrays with src < dst."""
    import numpy as np
    E_keys = np.asarray(E_keys, dtype=np.uint64)
    return ((E_keys >> np.uint64(32)).astype(np.int32),
            (E_keys & np.uint64(0xFFFFFFFF)).astype(np.int32))


# Vertex operations (Sec. 3): they reduce to edge operations -- a vertex that
# leaves V first loses every incident edge.  The vertex set is then the live
# ids; the counts of (V, E) depend on |V| and on E only, so they are those of
# the graph relabelled onto 0 .. |V| - 1.

def remove_vertices(E: set, live: set, ids):
    """Deletes every edge at `ids`, then the vertices; E and live in place."""
    ids = {int(x) for x in ids}
    if not ids <= live:
        raise BatchRejected("vertex not in V")
    for e in [e for e in E if e[0] in ids or e[1] in ids]:
        E.discard(e)
    live -= ids


def compact(E: set, live: set):
    """(n, src, dst) of (live, E) relabelled onto 0 .. |live| - 1 in id order."""
    import numpy as np
    rank = {v: i for i, v in enumerate(sorted(live))}
    pairs = sorted((rank[u], rank[v]) for u, v in E)
    return (len(live), np.array([u for u, _ in pairs], np.int32), np.array([v for _, v in pairs], np.int32))
