"""ORACLE -- test infrastructure.  Pure-Python brute force (tiny graphs).

A second, independent implementation of the plain definition: every 4-subset
S is mapped to the isomorphism class of G[S] by canonical labelling (the
smallest 6-bit adjacency code over all 24 vertex orders), and the canonical
codes of the 11 classes are derived from explicit edge lists of each class.
It shares nothing with oracle.c's classifier (edge count + degree sequence).
"""
from __future__ import annotations

import itertools

# pair order inside a 4-set (a, b, c, d) -> bit index
_PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
_PERMS = list(itertools.permutations(range(4)))

# one labelled representative of each class, output order of the library
_CLASS_EDGES = [
    [(0, 1), (1, 2), (2, 3)],                          # 0 P4 (3-path)
    [(0, 1), (0, 2), (0, 3)],                          # 1 3-star
    [(0, 1), (1, 2), (2, 3), (3, 0)],                  # 2 4-cycle
    [(0, 1), (1, 2), (2, 0), (0, 3)],                  # 3 paw (tailed triangle)
    [(0, 1), (1, 2), (2, 0), (0, 3), (2, 3)],          # 4 diamond
    [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],  # 5 4-clique
    [(0, 1), (1, 2), (2, 0)],                          # 6 triangle + isolated
    [(0, 1), (1, 2)],                                  # 7 2-path + isolated
    [(0, 1), (2, 3)],                                  # 8 two disjoint edges
    [(0, 1)],                                          # 9 edge + 2 isolated
    [],                                                # 10 empty
]


def _code(adj_pairs):
    """6-bit code of an edge set on labels 0..3."""
    c = 0
    for k, (i, j) in enumerate(_PAIRS):
        if (i, j) in adj_pairs or (j, i) in adj_pairs:
            c |= 1 << k
    return c


def _canon(code):
    edges = {_PAIRS[k] for k in range(6) if code >> k & 1}
    best = None
    for p in _PERMS:
        mapped = {(p[i], p[j]) for (i, j) in edges}
        c = _code(mapped)
        best = c if best is None or c < best else best
    return best


_CANON_TO_CLASS = {}
for _cls, _edges in enumerate(_CLASS_EDGES):
    _CANON_TO_CLASS[_canon(_code(set(_edges)))] = _cls
assert len(_CANON_TO_CLASS) == 11
_CODE_TO_CLASS = [_CANON_TO_CLASS[_canon(c)] for c in range(64)]


def brute_counts_py(n, edges):
    """edges: iterable of (u, v) pairs (simple graph).  n <= ~40."""
    E = set()
    for u, v in edges:
        u, v = int(u), int(v)
        assert u != v
        E.add((min(u, v), max(u, v)))
    out = [0] * 11
    for S in itertools.combinations(range(n), 4):
        c = 0
        for k, (i, j) in enumerate(_PAIRS):
            if (S[i], S[j]) in E:
                c |= 1 << k
        out[_CODE_TO_CLASS[c]] += 1
    return out
