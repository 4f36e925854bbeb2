"""ORACLE -- test infrastructure.  Batch semantics on a Python edge set.

The stream model (Sec. 3) applies a tuple <e, o> by set union (o = +) or set
difference (o = -); Problem 1 maintains the counts of
G^{t+1} = (V, E^t + A - D) for a batch B = A u D of a simple undirected graph.
Sec. 5 first removes the edges that are both added and deleted in a batch and
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
