"""Seeded graph and batch-stream generators.

Shapes follow the graphs the paper evaluates on (Table 1: sparse social and
communication networks with heavy-tailed degrees) and the batch protocol of
its experiments section (batches of insertions and deletions, an edge that is
both added and removed in one batch is dropped).  The public SNAP files are
not available, so these synthetic stand-ins replace them:

* Erdos-Renyi G(n, p)                         -- tiny brute-force cases
* R-MAT (a, b, c, d) with a seeded id permutation (Graph500 practice)
* Chung-Lu power law with exponent gamma (WikiTalk-like hub structure)

All randomness comes from ``numpy.random.default_rng`` (PCG64).  Graphs are
returned as canonical edge lists ``(src, dst)`` of int32 with ``src < dst``,
no self loops and no duplicates.  Batches are returned as
``(ins_src, ins_dst, del_src, del_dst)`` int32 arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_CHUNK = 1 << 24


# --------------------------------------------------------------------------
# key helpers (bookkeeping of the generator's own edge set)
# --------------------------------------------------------------------------
def canon_keys(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Unordered pair -> uint64 key (min << 32 | max).  Self loops -> drop."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    return ((lo << 32) | hi).astype(np.uint64)


def keys_to_edges(keys: np.ndarray):
    keys = np.asarray(keys, dtype=np.uint64)
    src = (keys >> np.uint64(32)).astype(np.int32)
    dst = (keys & np.uint64(0xFFFFFFFF)).astype(np.int32)
    return src, dst


def edges_to_keys(src, dst) -> np.ndarray:
    return canon_keys(src, dst)


def _contains(sorted_keys: np.ndarray, q: np.ndarray) -> np.ndarray:
    if sorted_keys.size == 0 or q.size == 0:
        return np.zeros(q.shape, dtype=bool)
    pos = np.searchsorted(sorted_keys, q)
    pos = np.minimum(pos, sorted_keys.size - 1)
    return sorted_keys[pos] == q


def _merge_sorted(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Union of two sorted, disjoint uint64 arrays (result sorted)."""
    if b.size == 0:
        return a
    b = np.sort(b)
    pos = np.searchsorted(a, b)
    return np.insert(a, pos, b)


# --------------------------------------------------------------------------
# Erdos-Renyi
# --------------------------------------------------------------------------
def erdos_renyi(n: int, p: float, seed: int):
    """G(n, p): every unordered pair independently with probability p."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < p
    return iu[keep].astype(np.int32), ju[keep].astype(np.int32)


# --------------------------------------------------------------------------
# R-MAT
# --------------------------------------------------------------------------
def rmat_edges(scale: int, count: int, rng, a=0.57, b=0.19, c=0.19):
    """Raw R-MAT samples: one quadrant draw per level, most significant first.

    Returns int64 (src, dst) in [0, 2**scale), loops and repeats included.
    """
    src = np.zeros(count, dtype=np.int64)
    dst = np.zeros(count, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for lo in range(0, count, _CHUNK):
        hi = min(count, lo + _CHUNK)
        s = np.zeros(hi - lo, dtype=np.int64)
        d = np.zeros(hi - lo, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(hi - lo)
            sbit = r >= ab
            dbit = ((r >= a) & (r < ab)) | (r >= abc)
            s = (s << 1) | sbit
            d = (d << 1) | dbit
        src[lo:hi] = s
        dst[lo:hi] = d
    return src, dst


@dataclass
class _RmatSampler:
    scale: int
    n: int
    perm: np.ndarray
    a: float = 0.57
    b: float = 0.19
    c: float = 0.19

    def __call__(self, k: int, rng):
        """k candidate pairs (permuted ids, ids < n; loops allowed)."""
        out_u, out_v, got = [], [], 0
        while got < k:
            want = max(64, int((k - got) * 1.3))
            s, d = rmat_edges(self.scale, want, rng, self.a, self.b, self.c)
            s = self.perm[s]
            d = self.perm[d]
            ok = (s < self.n) & (d < self.n)
            out_u.append(s[ok])
            out_v.append(d[ok])
            got += int(ok.sum())
        return np.concatenate(out_u)[:k], np.concatenate(out_v)[:k]


def _fill_unique(target_m: int, sampler, rng, initial: int):
    """Sample pairs, drop loops and repeats, resample until exactly target_m."""
    u, v = sampler(initial, rng)
    keys = np.unique(canon_keys(u, v))
    if keys.size > target_m:
        keys = np.sort(rng.choice(keys, target_m, replace=False))
    rounds = 0
    while keys.size < target_m:
        need = target_m - keys.size
        rounds += 1
        u, v = sampler(int(need * 1.5) + 64 * rounds, rng)
        cand = np.unique(canon_keys(u, v))
        cand = cand[~_contains(keys, cand)]
        if cand.size > need:
            cand = rng.choice(cand, need, replace=False)
        keys = _merge_sorted(keys, cand)
        if rounds > 200:
            raise RuntimeError("cannot reach the requested edge count")
    return keys


def rmat_graph(scale: int, edge_factor: int, seed: int, n: int | None = None,
               a=0.57, b=0.19, c=0.19, m: int | None = None):
    """R-MAT graph with exactly m = edge_factor * n unique undirected edges.

    A seeded permutation of the 2**scale ids is applied (Graph500 practice);
    for n < 2**scale, permuted ids >= n are rejected.  Returns
    (n, src, dst, sampler) where ``sampler(k, rng)`` draws further pairs
    from the same distribution (used for insertion batches).
    """
    rng = np.random.default_rng(seed)
    N = 1 << scale
    if n is None:
        n = N
    perm = rng.permutation(N).astype(np.int64)
    sampler = _RmatSampler(scale, n, perm, a, b, c)
    target = edge_factor * n if m is None else m
    keys = _fill_unique(target, sampler, rng, initial=target)
    src, dst = keys_to_edges(keys)
    return n, src, dst, sampler


# --------------------------------------------------------------------------
# Chung-Lu
# --------------------------------------------------------------------------
@dataclass
class _WeightedSampler:
    cdf: np.ndarray
    perm: np.ndarray

    def __call__(self, k: int, rng):
        r = rng.random(2 * k) * self.cdf[-1]
        ids = np.searchsorted(self.cdf, r, side="right")
        ids = np.minimum(ids, self.cdf.size - 1)
        ids = self.perm[ids]
        return ids[:k], ids[k:]


def chung_lu_weights(n: int, m: int, gamma: float, wmax: float):
    """w_i = c (i + i0)^(-1/(gamma-1)) with sum 2m and w_0 = wmax."""
    ex = -1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def total(i0):
        cc = wmax / (i0 ** ex)
        return cc * np.sum((idx + i0) ** ex)

    lo, hi = 1e-6, 1e7
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if total(mid) > 2 * m:
            hi = mid
        else:
            lo = mid
    i0 = math.sqrt(lo * hi)
    cc = wmax / (i0 ** ex)
    return cc * (idx + i0) ** ex


def chung_lu_graph(n: int, m: int, gamma: float, wmax: float, seed: int):
    """Chung-Lu graph: endpoints i.i.d. proportional to w, exactly m edges.

    Returns (n, src, dst, sampler) with ids permuted by a seeded permutation.
    """
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, m, gamma, wmax)
    perm = rng.permutation(n).astype(np.int64)
    sampler = _WeightedSampler(np.cumsum(w), perm)
    keys = _fill_unique(m, sampler, rng, initial=m)
    src, dst = keys_to_edges(keys)
    return n, src, dst, sampler


# --------------------------------------------------------------------------
# batch streams
# --------------------------------------------------------------------------
@dataclass
class BatchStream:
    """Clean fully dynamic batches over a tracked edge set.

    Deletions are drawn uniformly without replacement from the current edge
    set; insertions come from ``ins_sampler`` (a pair sampler) and are
    resampled until each is a non-edge not already in the batch.  After a
    batch is drawn the tracked set is advanced (set semantics), so the next
    batch is drawn from the graph the previous batch produced.
    """
    n: int
    keys: np.ndarray
    rng: np.random.Generator
    ins_sampler: object = None
    degree_prop_ins: bool = False
    history: list = field(default_factory=list)

    @classmethod
    def from_edges(cls, n, src, dst, seed, ins_sampler=None, degree_prop_ins=False):
        keys = np.unique(canon_keys(src, dst))
        return cls(n=n, keys=keys, rng=np.random.default_rng(seed),
                   ins_sampler=ins_sampler, degree_prop_ins=degree_prop_ins)

    def _sample_ins(self, k: int):
        if k == 0:
            return np.zeros(0, dtype=np.uint64)
        got = np.zeros(0, dtype=np.uint64)
        rounds = 0
        while got.size < k:
            rounds += 1
            need = k - got.size
            if self.degree_prop_ins:
                src, dst = keys_to_edges(self.keys)
                deg = np.bincount(np.concatenate([src, dst]), minlength=self.n)
                cdf = np.cumsum(deg.astype(np.float64))
                r = self.rng.random(2 * (need + 16)) * cdf[-1]
                ids = np.minimum(np.searchsorted(cdf, r, side="right"), self.n - 1)
                u, v = ids[: need + 16], ids[need + 16:]
            elif self.ins_sampler is not None:
                u, v = self.ins_sampler(need + 16, self.rng)
            else:
                u = self.rng.integers(0, self.n, need + 16)
                v = self.rng.integers(0, self.n, need + 16)
            cand = canon_keys(u, v)
            cand = cand[~_contains(self.keys, cand)]
            # keep first occurrences, in draw order, that are not already taken
            _, first = np.unique(cand, return_index=True)
            cand = cand[np.sort(first)]
            if got.size:
                cand = cand[~np.isin(cand, got)]
            got = np.concatenate([got, cand[:need]])
            if rounds > 100000:
                raise RuntimeError("cannot draw enough non-edges")
        return got

    def next_batch(self, n_del: int, n_ins: int):
        n_del = min(n_del, self.keys.size)
        di = self.rng.choice(self.keys.size, n_del, replace=False) if n_del else np.zeros(0, np.int64)
        dkeys = self.keys[di]
        ikeys = self._sample_ins(n_ins)
        mask = np.ones(self.keys.size, dtype=bool)
        mask[di] = False
        self.keys = _merge_sorted(self.keys[mask], ikeys)
        isrc, idst = keys_to_edges(ikeys)
        dsrc, ddst = keys_to_edges(dkeys)
        # random endpoint order: the library must canonicalise
        flip = self.rng.random(isrc.size) < 0.5
        isrc, idst = np.where(flip, idst, isrc), np.where(flip, isrc, idst)
        flip = self.rng.random(dsrc.size) < 0.5
        dsrc, ddst = np.where(flip, ddst, dsrc), np.where(flip, dsrc, ddst)
        return (isrc.astype(np.int32), idst.astype(np.int32),
                dsrc.astype(np.int32), ddst.astype(np.int32))


def er_batches(n, src, dst, count=5, size=50, first_seed=1):
    """Config of the tiny case: ``size/2`` deletions of uniform existing edges
    and ``size/2`` insertions of uniform non-edges, one seed per batch."""
    keys = np.unique(canon_keys(src, dst))
    out = []
    iu, ju = np.triu_indices(n, k=1)
    all_keys = canon_keys(iu, ju)
    for b in range(count):
        rng = np.random.default_rng(first_seed + b)
        nd = min(size // 2, keys.size)
        dk = rng.choice(keys, nd, replace=False) if nd else np.zeros(0, np.uint64)
        non = all_keys[~_contains(keys, all_keys)]
        ik = rng.choice(non, size - size // 2, replace=False)
        keys = np.sort(np.concatenate([np.setdiff1d(keys, dk), ik]))
        isrc, idst = keys_to_edges(ik)
        dsrc, ddst = keys_to_edges(dk)
        out.append((isrc, idst, dsrc, ddst))
    return out


def rmat_batches(n, src, dst, sampler, sizes, seed):
    """50/50 batches: uniform deletions, R-MAT insertions (same generator)."""
    st = BatchStream.from_edges(n, src, dst, seed, ins_sampler=sampler)
    return [st.next_batch(s // 2, s - s // 2) for s in sizes]


def chung_lu_batches(n, src, dst, sizes, seed):
    """50/50 batches: uniform deletions (endpoints therefore follow degree),
    insertions with both endpoints drawn proportional to current degree."""
    st = BatchStream.from_edges(n, src, dst, seed, degree_prop_ins=True)
    return [st.next_batch(s // 2, s - s // 2) for s in sizes]


def multi_graph_workload(count=256, seed=4, n_lo=1e3, n_hi=2e5,
                         efs=(4, 8, 16), b_lo=1e2, b_hi=1e4):
    """Many independent R-MAT graphs, one update batch each.

    n log-uniform in [n_lo, n_hi], edge factor uniform in ``efs``, batch size
    log-uniform in [b_lo, b_hi], half deletions and half insertions.
    Returns a list of dicts with keys n, src, dst, batch.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(10 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))))
        ef = int(rng.choice(efs))
        bs = int(round(10 ** rng.uniform(math.log10(b_lo), math.log10(b_hi))))
        scale = max(1, math.ceil(math.log2(n)))
        gseed = int(rng.integers(0, 2**31 - 1))
        n_, s, d, sampler = rmat_graph(scale, ef, gseed, n=n)
        batch = rmat_batches(n_, s, d, sampler, [bs], gseed + 1)[0]
        out.append(dict(n=n_, src=s, dst=d, batch=batch, edge_factor=ef))
    return out


def raw_noise_batch(n, src, dst, n_each, seed):
    """A deliberately messy batch exercising every ingest rule.

    Contains: self loops, duplicates in both orientations, insertions of
    existing edges, deletions of missing edges, pairs both inserted and
    deleted, plus some clean insertions and deletions.
    """
    rng = np.random.default_rng(seed)
    keys = np.unique(canon_keys(src, dst))
    es, ed = keys_to_edges(keys)
    ins_u, ins_v, del_u, del_v = [], [], [], []
    k = min(n_each, keys.size)
    # self loops
    x = rng.integers(0, n, n_each)
    ins_u.append(x); ins_v.append(x)
    del_u.append(x[: n_each // 2]); del_v.append(x[: n_each // 2])
    # insert existing (both orientations)
    pick = rng.choice(keys.size, k, replace=False)
    ins_u.append(ed[pick]); ins_v.append(es[pick])
    # clean deletions, duplicated, reversed
    pick2 = rng.choice(keys.size, k, replace=False)
    del_u.append(es[pick2]); del_v.append(ed[pick2])
    del_u.append(ed[pick2[: k // 2]]); del_v.append(es[pick2[: k // 2]])
    # delete missing
    mu = rng.integers(0, n, n_each); mv = rng.integers(0, n, n_each)
    mk = canon_keys(mu, mv)
    mk = mk[~_contains(keys, mk)]
    a, b = keys_to_edges(mk)
    del_u.append(a); del_v.append(b)
    # clean insertions with duplicates; some also deleted (cancel)
    cu = rng.integers(0, n, n_each); cv = rng.integers(0, n, n_each)
    ck = np.unique(canon_keys(cu, cv))
    ck = ck[~_contains(keys, ck)]
    a, b = keys_to_edges(ck)
    ins_u.append(a); ins_v.append(b)
    ins_u.append(b[: a.size // 3]); ins_v.append(a[: a.size // 3])
    del_u.append(a[: a.size // 4]); del_v.append(b[: a.size // 4])
    # existing edges deleted and re-inserted in the same batch (cancel)
    pick3 = rng.choice(keys.size, max(1, k // 4), replace=False)
    del_u.append(es[pick3]); del_v.append(ed[pick3])
    ins_u.append(es[pick3]); ins_v.append(ed[pick3])
    cat = lambda xs: rng.permutation(np.concatenate(xs)).astype(np.int32)
    iu = np.concatenate(ins_u).astype(np.int32)
    iv = np.concatenate(ins_v).astype(np.int32)
    p = rng.permutation(iu.size)
    du = np.concatenate(del_u).astype(np.int32)
    dv = np.concatenate(del_v).astype(np.int32)
    q = rng.permutation(du.size)
    del cat
    return iu[p], iv[p], du[q], dv[q]


def poisson_arrivals(rate_per_s: float, count: int, seed: int):
    """Arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, count))


def log_uniform_sizes(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return [int(round(10 ** rng.uniform(math.log10(lo), math.log10(hi)))) for _ in range(count)]
