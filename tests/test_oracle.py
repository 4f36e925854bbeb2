"""Pins of the oracle against facts it does not compute itself.

* brute force, two independent implementations (edge-count/degree
  classification in C, canonical labelling in Python);
* the static recount (the baseline of Sec. 4.1) against brute force on many
  small graphs of several shapes;
* closed forms on K_n, stars, paths, cycles, complete bipartite graphs,
  K_n - e, K_n + pendant, a triangle plus isolated vertices, including sizes
  where C(n,4) exceeds int64;
* the complement duality of induced 4-vertex classes;
* the FDGC reference (Alg. 2) against the static recount after every batch
  (Lemma 2), with negative controls that must fail.
"""
import itertools
import math
import random

import numpy as np
import pytest

from oracle import native
from oracle.brute_py import brute_counts_py
from oracle.fdgc import FDGCRef
from oracle.semantics import BatchRejected, apply_batch, effective_batch
from graphgen import erdos_renyi, rmat_graph, keys_to_edges, canon_keys

C = math.comb


def edges_of(E):
    E = sorted(E)
    return [u for u, v in E], [v for u, v in E]


def rand_graph(n, p, rng):
    E = set()
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                E.add((u, v))
    return E


def test_brute_c_vs_python():
    rng = random.Random(11)
    for trial in range(120):
        n = rng.randint(4, 10)
        E = rand_graph(n, rng.choice([0.1, 0.3, 0.5, 0.7, 0.9]), rng)
        s, d = edges_of(E)
        assert native.brute_counts(n, s, d) == brute_counts_py(n, E)


def test_static_vs_brute_random():
    rng = random.Random(12)
    for trial in range(300):
        n = rng.randint(4, 18)
        E = rand_graph(n, rng.choice([0.05, 0.2, 0.4, 0.6, 0.8, 0.95]), rng)
        s, d = edges_of(E)
        b = native.brute_counts(n, s, d)
        assert sum(b) == C(n, 4)
        assert native.static_counts(n, s, d) == b, (n, sorted(E))


@pytest.mark.parametrize("scale,ef,seed", [(6, 4, 1), (7, 4, 2), (7, 8, 3), (8, 6, 4)])
def test_static_vs_brute_rmat(scale, ef, seed):
    """Heavy-tailed graphs (hubs, many triangles) up to n = 256."""
    n, s, d, _ = rmat_graph(scale, ef, seed)
    assert native.static_counts(n, s, d) == native.brute_counts(n, s, d)


def test_static_vs_brute_er150():
    s, d = erdos_renyi(150, 6 / 149, 0)
    assert native.static_counts(150, s, d) == native.brute_counts(150, s, d)


def _complete(n):
    return [(u, v) for u in range(n) for v in range(u + 1, n)]


def counts(n, E):
    s, d = edges_of(E)
    return native.static_counts(n, s, d)


def vec(n, **kw):
    names = ["P4", "star", "C4", "paw", "dia", "K4", "K3K1", "P3K1", "2K2", "K2K1K1", "empty"]
    out = [0] * 11
    for k, v in kw.items():
        out[names.index(k)] = v
    return out


@pytest.mark.parametrize("n", [4, 5, 9, 30, 64])
def test_closed_form_complete(n):
    assert counts(n, _complete(n)) == vec(n, K4=C(n, 4))


@pytest.mark.parametrize("n", [4, 7, 50, 200000])
def test_closed_form_star(n):
    E = [(0, i) for i in range(1, n)]
    assert counts(n, E) == vec(n, star=C(n - 1, 3), empty=C(n - 1, 4))


@pytest.mark.parametrize("n", [4, 5, 8, 100, 150000])
def test_closed_form_path(n):
    E = [(i, i + 1) for i in range(n - 1)]
    assert counts(n, E) == vec(n, P4=n - 3, **{"2K2": C(n - 3, 2)}, P3K1=2 * C(n - 3, 2),
                               K2K1K1=3 * C(n - 3, 3), empty=C(n - 3, 4))


@pytest.mark.parametrize("n", [5, 6, 11, 97, 130000])
def test_closed_form_cycle(n):
    E = [(i, (i + 1) % n) for i in range(n)]
    E = [(min(a, b), max(a, b)) for a, b in E]
    assert counts(n, E) == vec(n, P4=n, P3K1=n * (n - 5), **{"2K2": n * (n - 5) // 2},
                               K2K1K1=n * C(n - 5, 2), empty=n * C(n - 5, 3) // 4)


def test_closed_form_c4():
    assert counts(4, [(0, 1), (1, 2), (2, 3), (0, 3)]) == vec(4, C4=1)


@pytest.mark.parametrize("a,b", [(1, 3), (2, 2), (3, 5), (40, 60)])
def test_closed_form_bipartite(a, b):
    E = [(i, a + j) for i in range(a) for j in range(b)]
    assert counts(a + b, E) == vec(a + b, C4=C(a, 2) * C(b, 2), star=C(a, 3) * b + a * C(b, 3),
                                   empty=C(a, 4) + C(b, 4))


@pytest.mark.parametrize("n", [4, 6, 25])
def test_closed_form_complete_minus_edge(n):
    E = [e for e in _complete(n) if e != (0, 1)]
    assert counts(n, E) == vec(n, dia=C(n - 2, 2), K4=C(n, 4) - C(n - 2, 2))


@pytest.mark.parametrize("n", [4, 5, 20])
def test_closed_form_complete_plus_pendant(n):
    E = _complete(n) + [(0, n)]
    assert counts(n + 1, E) == vec(n + 1, paw=C(n - 1, 2), K3K1=C(n - 1, 3), K4=C(n, 4))


@pytest.mark.parametrize("n", [4, 9, 140000])
def test_closed_form_triangle_isolated(n):
    E = [(0, 1), (1, 2), (0, 2)]
    assert counts(n, E) == vec(n, K3K1=n - 3, K2K1K1=3 * C(n - 3, 2),
                               empty=3 * C(n - 3, 3) + C(n - 3, 4))


# induced class of the complement: P4<->P4, star<->K3+K1, C4<->2K2,
# paw<->P3+K1, diamond<->K2+2K1, K4<->empty
COMP = [0, 6, 8, 7, 9, 10, 1, 3, 2, 4, 5]


@pytest.mark.parametrize("seed", range(6))
def test_complement_duality(seed):
    rng = random.Random(seed)
    n = rng.randint(20, 90)
    E = rand_graph(n, rng.choice([0.1, 0.3, 0.6]), rng)
    Ec = set(_complete(n)) - E
    a, b = counts(n, E), counts(n, Ec)
    assert [b[COMP[c]] for c in range(11)] == a


def test_int128_path_exact():
    """C(n,4) > 2^63 - 1 for n > 121977: the empty class needs 128 bits."""
    n = 200000
    c = counts(n, [(0, 1)])
    assert c == vec(n, K2K1K1=C(n - 2, 2), empty=C(n, 4) - C(n - 2, 2))
    assert c[10] > 2**63


# ------------------------------------------------------------ semantics ---
def test_semantics_rules():
    E = {(0, 1), (1, 2), (2, 3)}
    ins_s = [1, 4, 4, 3, 5, 6, 6]
    ins_d = [0, 5, 5, 3, 4, 7, 8]       # existing (reversed), dup x3, loop, new (6,7), (6,8)
    del_s = [2, 3, 0, 8, 7]
    del_d = [1, 2, 5, 6, 6]              # existing x2, missing, cancel (6,8), cancel (6,7)
    A, D, st = effective_batch(E, 10, ins_s, ins_d, del_s, del_d)
    assert A == {(4, 5)}
    assert D == {(1, 2), (2, 3)}
    assert st["loops"] == 1 and st["cancelled"] == 2
    assert st["ins_existing"] == 1 and st["del_missing"] == 1
    with pytest.raises(BatchRejected):
        effective_batch(E, 4, [0], [4], [], [])
    E2 = set(E)
    apply_batch(E2, 10, ins_s, ins_d, del_s, del_d)
    assert E2 == {(0, 1), (4, 5)}


# --------------------------------------------------------------- FDGC ------
def _stream(seed, n=28, p=0.18, nb=6):
    rng = np.random.default_rng(seed)
    s, d = erdos_renyi(n, p, seed)
    batches = []
    for _ in range(nb):
        k = int(rng.integers(1, 8))
        batches.append((rng.integers(0, n, k), rng.integers(0, n, k),
                        rng.integers(0, n, k), rng.integers(0, n, k)))
    # deletions of existing edges too
    return n, s, d, batches


def _run(ref, n, s, d, batches):
    E = set(zip(s.tolist(), d.tolist()))
    ok = True
    for b in batches:
        b = list(b)
        # make half the deletions hit real edges
        if len(E):
            el = sorted(E)
            rng = random.Random(len(E))
            for i in range(0, len(b[2]), 2):
                u, v = el[rng.randrange(len(el))]
                b[2][i], b[3][i] = u, v
        F = ref.apply(*b)
        apply_batch(E, n, *b)
        es, ed = edges_of(E)
        ok &= F == native.static_counts(n, es, ed)[:6]
    return ok


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("radius,region", [(3, "paper"), (2, "paper"), (2, "induced"), (0, "whole")])
def test_fdgc_matches_recount(seed, radius, region):
    n, s, d, batches = _stream(seed)
    ref = FDGCRef(n, s, d, radius=radius, region=region)
    assert ref.F == native.static_counts(n, s, d)[:6]
    assert _run(ref, n, s, d, batches)


def test_fdgc_negative_controls():
    """Radius 1 and a non-induced region must give a wrong count on some
    pinned stream: the tests above can fail."""
    bad_r1 = bad_tree = 0
    for seed in range(8):
        n, s, d, batches = _stream(seed)
        bad_r1 += not _run(FDGCRef(n, s, d, radius=1, region="paper"), n, s, d, batches)
        bad_tree += not _run(FDGCRef(n, s, d, radius=2, region="tree"), n, s, d, batches)
    assert bad_r1 > 0 and bad_tree > 0


def test_fdgc_insert_only_alg1():
    """Alg. 1 is the D = empty case."""
    rng = np.random.default_rng(5)
    n = 30
    ref = FDGCRef(n, radius=3)
    E = set()
    for _ in range(8):
        k = 6
        u, v = rng.integers(0, n, k), rng.integers(0, n, k)
        F = ref.apply(u, v, [], [])
        apply_batch(E, n, u, v, [], [])
        es, ed = edges_of(E)
        assert F == native.static_counts(n, es, ed)[:6]


def test_golden_er150():
    """Stored brute-force counts of the tiny workload (written by
    tests/golden/make_er150.py from oracle/ only) equal the static recount."""
    import json, os
    from graphgen import er_batches
    path = os.path.join(os.path.dirname(__file__), "golden", "er150_counts.json")
    g = json.load(open(path))
    n = g["n"]
    s, d = erdos_renyi(n, 6 / 149, 0)
    E = set(zip(s.tolist(), d.tolist()))
    assert native.static_counts(n, s, d) == g["counts"][0]
    for b, want in zip(er_batches(n, s, d), g["counts"][1:]):
        apply_batch(E, n, *b)
        es, ed = edges_of(E)
        assert native.static_counts(n, es, ed) == want
        assert sum(want) == C(n, 4)


@pytest.mark.parametrize("kind,seed", [("rmat12", 1), ("rmat13", 2), ("chung_lu", 3)])
def test_static_two_formulations(kind, seed):
    """Graphs with hubs, too large for brute force: the recount (degree
    order, marks, 4-cycles over pairs counted once) equals the second
    formulation (id order, sorted merges, 4-cycles over ordered pairs)."""
    from graphgen import chung_lu_graph
    if kind == "chung_lu":
        n, s, d, _ = chung_lu_graph(20000, 60000, 2.1, 2000.0, seed)
    else:
        n, s, d, _ = rmat_graph(int(kind[4:]), 16, seed)
    a = native.static_counts(n, s, d)
    assert a == native.static_counts_merge(n, s, d)
    assert sum(a) == C(n, 4)


@pytest.mark.parametrize("seed", range(5))
def test_semantics_keys_equal_sets(seed):
    """The array form of the batch rules equals the set form on messy
    batches (loops, repeats in both orientations, no-ops, A and D overlap)."""
    from graphgen import raw_noise_batch
    from oracle.semantics import apply_batch_keys, keys_to_pairs
    n, s, d, _ = rmat_graph(9, 6, seed)
    E = set(zip(s.tolist(), d.tolist()))
    K = np.unique(canon_keys(s, d))
    for k in range(4):
        b = raw_noise_batch(n, *keys_to_pairs(K), 40, 100 * seed + k)
        A, D, st = apply_batch(E, n, *b)
        K, st2 = apply_batch_keys(K, n, *b)
        assert st == st2
        assert set(zip(*[x.tolist() for x in keys_to_pairs(K)])) == E
    with pytest.raises(BatchRejected):
        apply_batch_keys(K, n, [0], [n], [], [])


# ------------------------------------------------------ 3-vertex counts ---
def test_counts3_static_vs_brute():
    rng = random.Random(31)
    for trial in range(200):
        n = rng.randint(3, 16)
        E = rand_graph(n, rng.choice([0.05, 0.3, 0.6, 0.95]), rng)
        s, d = edges_of(E)
        b = native.brute3_counts(n, s, d)
        assert sum(b) == C(n, 3)
        assert native.static_counts3(n, s, d) == b, (n, sorted(E))
    n, s, d, _ = rmat_graph(8, 8, 5)
    assert native.static_counts3(n, s, d) == native.brute3_counts(n, s, d)


@pytest.mark.parametrize("n", [3, 7, 40, 200000])
def test_counts3_closed_forms(n):
    star = [(0, i) for i in range(1, n)]
    assert native.static_counts3(n, *edges_of(star)) == [0, C(n - 1, 2), 0, C(n - 1, 3)]
    path = [(i, i + 1) for i in range(n - 1)]
    # an end edge sees n - 3 vertices adjacent to neither endpoint, an inner edge n - 4
    one_edge = 2 * (n - 3) + (n - 3) * (n - 4) if n > 3 else 0
    assert native.static_counts3(n, *edges_of(path)) == [0, n - 2, one_edge, C(n, 3) - (n - 2) - one_edge]
    if n <= 40:
        assert native.static_counts3(n, *edges_of(_complete(n))) == [C(n, 3), 0, 0, 0]


def test_vertex_removal_vs_subset_brute():
    """Vertex deletion (Sec. 3: incident edges first, then the vertex) and
    the relabelling onto the live ids, against a classification of every
    4-subset of the surviving vertices in the ORIGINAL graph."""
    from oracle.semantics import compact, remove_vertices
    rng = random.Random(21)
    for trial in range(40):
        n = rng.randint(5, 12)
        E = rand_graph(n, rng.choice([0.2, 0.5, 0.8]), rng)
        S = set(rng.sample(range(n), rng.randint(1, n - 4)))
        rest = sorted(set(range(n)) - S)
        want = [0] * 11
        for Q in itertools.combinations(rest, 4):
            loc = {v: i for i, v in enumerate(Q)}
            sub = {(loc[u], loc[v]) for u, v in E if u in loc and v in loc}
            c = brute_counts_py(4, sub)
            want = [a + b for a, b in zip(want, c)]
        E2, live = set(E), set(range(n))
        remove_vertices(E2, live, S)
        n2, s2, d2 = compact(E2, live)
        assert n2 == len(rest)
        assert native.static_counts(n2, s2, d2) == want
        with pytest.raises(BatchRejected):
            remove_vertices(E2, live, [min(S)])


# Per class (order of the eleven counts): edges e(c), 2-paths w(c) (pairs of
# edges sharing an end) and triangles tau(c) inside the induced subgraph.
E_OF = [3, 3, 4, 4, 5, 6, 3, 2, 2, 1, 0]
W_OF = [2, 3, 4, 5, 8, 12, 3, 1, 0, 0, 0]
TAU_OF = [0, 0, 0, 1, 2, 4, 1, 0, 0, 0, 0]


@pytest.mark.parametrize("kind,seed", [("rmat10", 5), ("rmat11", 6), ("er1500", 7)])
def test_weighted_identities(kind, seed):
    """Counting the 4-subsets by what they contain: each edge lies in
    C(n-2, 2) of them, each 2-path in n-3 and each triangle in n-3, so
    sum_c e(c) I_c = m C(n-2, 2), sum_c w(c) I_c = W (n-3) with W the 2-paths
    of the graph, and sum_c tau(c) I_c = T (n-3).  m, W and T come from the
    degrees and a dense adjacency product, independently of the oracle, on
    graphs too large for brute force (n up to 2048)."""
    if kind == "rmat10":
        n, s, d, _ = rmat_graph(10, 16, seed)
    elif kind == "rmat11":
        n, s, d, _ = rmat_graph(11, 8, seed)
    else:
        n = 1500
        s, d = erdos_renyi(n, 0.02, seed)
    I = native.static_counts(n, s, d)
    m = int(s.size)
    deg = np.bincount(s, minlength=n) + np.bincount(d, minlength=n)
    W = int(sum(int(x) * (int(x) - 1) // 2 for x in deg))
    A = np.zeros((n, n))
    A[s, d] = 1.0
    A[d, s] = 1.0
    T = int(round(float((A @ A)[s, d].sum()) / 3))  # common neighbours per edge, each triangle thrice
    assert sum(I) == C(n, 4)
    assert sum(e * x for e, x in zip(E_OF, I)) == m * C(n - 2, 2)
    assert sum(w * x for w, x in zip(W_OF, I)) == W * (n - 3)
    assert sum(t * x for t, x in zip(TAU_OF, I)) == T * (n - 3)
    assert T > 0
    # the 3-vertex classes (triangle, 2-path, edge + isolated, empty): each
    # edge lies in n - 2 triples, each 2-path in one, each triangle in one
    I3 = native.static_counts3(n, s, d)
    assert sum(I3) == C(n, 3)
    assert 3 * I3[0] + 2 * I3[1] + I3[2] == m * (n - 2)
    assert 3 * I3[0] + I3[1] == W
    assert I3[0] == T
