"""The named workloads at their stated sizes: graph plus batch sequence.

Each function returns a ``Workload`` (n, src, dst, batches) drawn from the
generators of this package with fixed seeds, so that the stored expected
counts (written by a script that calls only the oracle), the GPU parity tests
and the benchmark all see the same inputs.  ``digest`` fingerprints the
inputs so that a change of generator is caught before counts are compared.
Nothing here counts anything.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

from .generators import (BatchStream, chung_lu_graph, log_uniform_sizes, multi_graph_workload,
                         rmat_batches, rmat_graph)


@dataclass
class Workload:
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    batches: list = field(default_factory=list)   # (ins_src, ins_dst, del_src, del_dst)
    recipe: str = ""


def digest(arrays) -> str:
    """sha256 over the bytes of a sequence of arrays (and their lengths)."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(np.int64(a.size).tobytes())
        h.update(a.tobytes())
    return h.hexdigest()


def workload_digest(w: Workload) -> str:
    parts = [np.array([w.n], np.int64), w.src, w.dst]
    for b in w.batches:
        parts.extend(b)
    return digest(parts)


def rmat_s18_stream(per_size: int = 10) -> Workload:
    """R-MAT scale 18, edge factor 8 (n = 262,144, m = 2,097,152), then
    ``per_size`` batches each of 1k, 10k and 100k updates (half uniform
    deletions of existing edges, half insertions from the same generator),
    in that order."""
    n, s, d, sampler = rmat_graph(18, 8, 18)
    sizes = [1000] * per_size + [10000] * per_size + [100000] * per_size
    return Workload("rmat_s18_ef8", n, s, d, rmat_batches(n, s, d, sampler, sizes, 19),
                    "rmat_graph(18, 8, seed 18); rmat_batches(sizes=%d x [1e3, 1e4, 1e5], seed 19)" % per_size)


def chung_lu_stream(per_size: int = 3) -> Workload:
    """Chung-Lu power law, n = 2.4M, m = 5M, gamma = 2.1, largest weight 1e5,
    then ``per_size`` batches each of 1e3, 1e4 and 1e5 updates (half uniform
    deletions, half insertions with both endpoints drawn in proportion to the
    current degree)."""
    from .generators import chung_lu_batches
    n, s, d, _ = chung_lu_graph(2_400_000, 5_000_000, 2.1, 1e5, 3)
    sizes = [1000] * per_size + [10000] * per_size + [100000] * per_size
    return Workload("chung_lu_2.4M_5M", n, s, d, chung_lu_batches(n, s, d, sizes, 31),
                    "chung_lu_graph(2.4e6, 5e6, gamma 2.1, wmax 1e5, seed 3); "
                    "chung_lu_batches(sizes=%d x [1e3, 1e4, 1e5], seed 31)" % per_size)


def pool256():
    """256 independent R-MAT graphs (n log-uniform in [1e3, 2e5], edge factor
    in {4, 8, 16}), one batch each of log-uniform size in [100, 1e4]."""
    return multi_graph_workload(256, seed=4)


def pool_digest(graphs) -> str:
    parts = []
    for g in graphs:
        parts.append(np.array([g["n"]], np.int64))
        parts.extend([g["src"], g["dst"]])
        parts.extend(g["batch"])
    return digest(parts)


# The scale-22 benchmark stream: warm-up and timed batches through the
# device-array entry point, then a few more through the host-array one.
S22_SEED = 22


def rmat_s22_bench_stream(total: int = 25, host_steps: int = 0, lo: float = 10, hi: float = 1e5,
                          scale: int = 22, ef: int = 16, seed: int = S22_SEED, snapshot_at=None):
    """R-MAT scale 22, edge factor 16 (n = 4,194,304, m = 67,108,864) with
    ``total`` batches of log-uniform size in [lo, hi] (half uniform
    deletions, half R-MAT insertions), then ``host_steps`` more batches of
    the same kind with sizes of their own.  The sequence depends on
    ``total`` and ``host_steps`` only.  Returns (Workload with all batches in
    order, sizes of the first ``total``, the stream); with ``snapshot_at``
    = j the stream also keeps ``stream.snapshot``, its edge keys after the
    first j batches."""
    n, s, d, sampler = rmat_graph(scale, ef, seed)
    sizes = log_uniform_sizes(total, lo, hi, seed + 1)
    stream = BatchStream.from_edges(n, s, d, seed + 2, ins_sampler=sampler)
    batches = []
    for j, sz in enumerate(sizes):
        if snapshot_at == j:
            stream.snapshot = stream.keys.copy()
        batches.append(stream.next_batch(sz // 2, sz - sz // 2))
    if snapshot_at == len(sizes):
        stream.snapshot = stream.keys.copy()
    hsizes = log_uniform_sizes(host_steps, lo, hi, seed + 3)
    more = [stream.next_batch(sz // 2, sz - sz // 2) for sz in hsizes]
    w = Workload("rmat_s%d_ef%d_bench" % (scale, ef), n, s, d, batches + more,
                 "rmat_graph(%d, %d, seed %d); %d batches, sizes log_uniform_sizes(%d, %g, %g, seed %d); "
                 "BatchStream(seed %d, R-MAT insertions); then %d batches of sizes log_uniform_sizes(%d, %g, %g, "
                 "seed %d)" % (scale, ef, seed, total, total, lo, hi, seed + 1, seed + 2, host_steps, host_steps,
                               lo, hi, seed + 3))
    return w, sizes, stream


def graph_digest(w: Workload) -> str:
    return digest([np.array([w.n], np.int64), w.src, w.dst])


def prefix_digest(w: Workload, j: int) -> str:
    """Digest of the graph and its first j batches."""
    parts = [np.array([w.n], np.int64), w.src, w.dst]
    for b in w.batches[:j]:
        parts.extend(b)
    return digest(parts)


def net_batch(keys_from, keys_to):
    """One clean batch taking the edge-key set keys_from to keys_to (both
    sorted uint64 pair keys): insert keys_to - keys_from, delete
    keys_from - keys_to."""
    from .generators import keys_to_edges
    ins = np.setdiff1d(keys_to, keys_from, assume_unique=True)
    dele = np.setdiff1d(keys_from, keys_to, assume_unique=True)
    a, b = keys_to_edges(ins)
    c, d = keys_to_edges(dele)
    return a, b, c, d
