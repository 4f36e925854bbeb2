"""Writes the expected counts of the workloads at their stated sizes.

For each workload of ``graphgen.workloads`` the oracle's static recount
(oracle/oracle.c, the recount-from-scratch baseline of Sec. 4.1) gives the
eleven induced 4-vertex counts of the initial graph and of the graph after
the listed batches, which are applied with the batch rules of
``oracle.semantics`` (array form).  Calls only oracle/ and graphgen/.

    python tests/golden/make_scale.py [rmat_s18] [chung_lu] [pool256] [rmat_s22]

Each output file records the recipe, an input digest, the batch counts after
which counts are stored (0 = the initial graph), the counts, and the
oracle's wall time and thread count per recount.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from graphgen import canon_keys  # noqa: E402
from graphgen import workloads as wl  # noqa: E402
from oracle import native  # noqa: E402
from oracle.semantics import apply_batch_keys, keys_to_pairs  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recount(n, K):
    s, d = keys_to_pairs(K)
    t0 = time.time()
    c = native.static_counts(n, s, d)
    return c, time.time() - t0


def stream_golden(w, steps, path):
    """Counts after each listed number of batches.  Each stored step carries
    the digest of the graph and the batches before it, so a stored count
    stays valid for any stream that starts with the same batches."""
    K = np.unique(canon_keys(w.src, w.dst))
    out = {"workload": w.name, "recipe": w.recipe, "n": w.n, "m0": int(K.size),
           "input_sha256": wl.workload_digest(w), "batches": len(w.batches),
           "steps": [], "prefix_sha256": [], "m": [], "counts": [], "oracle_seconds": [],
           "oracle_threads": native.threads()}
    want = set(steps)
    # resume: counts already stored for the same prefix of inputs are kept
    done = {}
    if os.path.exists(path):
        old = json.load(open(path))
        for j, ps, m, c, t in zip(old["steps"], old.get("prefix_sha256", []), old["m"], old["counts"],
                                  old["oracle_seconds"]):
            done[ps] = (m, c, t)
    for j in range(len(w.batches) + 1):
        if j > 0:
            K, _ = apply_batch_keys(K, w.n, *w.batches[j - 1])
        if j not in want:
            continue
        ps = wl.prefix_digest(w, j)
        if ps in done and done[ps][0] == K.size:
            m, c, secs = done[ps]
            log("%s: after %d batches: stored counts kept" % (w.name, j))
        else:
            c, secs = recount(w.n, K)
            secs = round(secs, 3)
            log("%s: after %d batches m=%d counts=%s (%.1fs)" % (w.name, j, K.size, c, secs))
        out["steps"].append(j)
        out["prefix_sha256"].append(ps)
        out["m"].append(int(K.size))
        out["counts"].append(c)
        out["oracle_seconds"].append(secs)
        with open(path, "w") as f:   # partial results survive an interruption
            json.dump(out, f, indent=1)
    return out


def pool_golden(path):
    graphs = wl.pool256()
    out = {"workload": "pool256", "recipe": "multi_graph_workload(256, seed 4): one batch per graph",
           "input_sha256": wl.pool_digest(graphs), "graphs": len(graphs),
           "n": [], "counts_initial": [], "counts_after": [], "oracle_seconds": 0.0,
           "oracle_threads": native.threads()}
    t0 = time.time()
    for i, g in enumerate(graphs):
        K = np.unique(canon_keys(g["src"], g["dst"]))
        out["n"].append(g["n"])
        out["counts_initial"].append(recount(g["n"], K)[0])
        K, _ = apply_batch_keys(K, g["n"], *g["batch"])
        out["counts_after"].append(recount(g["n"], K)[0])
        if i % 32 == 31:
            log("pool: %d graphs done (%.0fs)" % (i + 1, time.time() - t0))
    out["oracle_seconds"] = round(time.time() - t0, 1)
    with open(path, "w") as f:
        json.dump(out, f)
    return out


def main():
    which = sys.argv[1:] or ["rmat_s18", "chung_lu", "pool256"]
    native.build()
    for name in which:
        t0 = time.time()
        if name == "rmat_s18":
            w = wl.rmat_s18_stream()
            stream_golden(w, range(len(w.batches) + 1), os.path.join(HERE, "scale_rmat_s18_ef8.json"))
        elif name == "chung_lu":
            w = wl.chung_lu_stream()
            stream_golden(w, range(len(w.batches) + 1), os.path.join(HERE, "scale_chung_lu.json"))
        elif name == "pool256":
            pool_golden(os.path.join(HERE, "scale_pool256.json"))
        elif name == "rmat_s22":
            w, sizes, _ = wl.rmat_s22_bench_stream()
            log("rmat_s22: inputs drawn in %.0fs" % (time.time() - t0))
            stream_golden(w, [0, 25], os.path.join(HERE, "scale_rmat_s22_bench.json"))
        else:
            raise SystemExit("unknown workload %s" % name)
        log("%s done in %.0fs" % (name, time.time() - t0))


if __name__ == "__main__":
    main()
