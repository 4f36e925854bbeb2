"""ORACLE -- test infrastructure.  Times one full static recount of an
R-MAT graph by the oracle (the per-batch work of the recount-from-scratch
baseline) on this host and prints key: value lines (threads, host, seconds).

    python -m oracle.time_recount --scale 22 --ef 16 [--seed 22]

The thread count is OpenMP's (OMP_NUM_THREADS, else every usable core).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--ef", type=int, default=16)
    ap.add_argument("--seed", type=int, default=22)
    a = ap.parse_args()
    from graphgen import rmat_graph
    from oracle import native
    native.build()
    t0 = time.time()
    n, s, d, _ = rmat_graph(a.scale, a.ef, a.seed)
    print("graph: R-MAT scale %d ef %d seed %d, n=%d m=%d (drawn in %.1fs)" % (a.scale, a.ef, a.seed, n, s.size,
                                                                               time.time() - t0), flush=True)
    model = ""
    for line in open("/proc/cpuinfo"):
        if line.startswith("model name"):
            model = line.split(":", 1)[1].strip()
            break
    print("cpu_model: %s" % model)
    print("nproc: %d" % len(os.sched_getaffinity(0)))
    print("threads: %d" % native.threads(), flush=True)
    t0 = time.perf_counter()
    c = native.static_counts(n, s, d)
    print("recount_s: %.2f" % (time.perf_counter() - t0))
    print("counts: %s" % c, flush=True)


if __name__ == "__main__":
    main()
