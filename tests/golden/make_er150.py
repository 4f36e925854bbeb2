"""Writes er150_counts.json: brute-force induced 4-vertex counts of the tiny
Erdos-Renyi workload (G(150, 6/149), seed 0; five batches of 25 uniform
deletions and 25 uniform non-edge insertions, seeds 1..5) after
initialisation and after every batch.  Calls only oracle/ and graphgen/.

    python tests/golden/make_er150.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from graphgen import erdos_renyi, er_batches  # noqa: E402
from oracle import native  # noqa: E402
from oracle.semantics import apply_batch  # noqa: E402


def main():
    n = 150
    s, d = erdos_renyi(n, 6 / 149, 0)
    E = set(zip(s.tolist(), d.tolist()))
    out = {"recipe": "erdos_renyi(150, 6/149, seed 0); er_batches(count=5, size=50, first_seed=1)",
           "n": n, "m0": len(E), "counts": []}
    out["counts"].append(native.brute_counts(n, s, d))
    for b in er_batches(n, s, d):
        apply_batch(E, n, *b)
        es = sorted(E)
        out["counts"].append(native.brute_counts(n, [u for u, v in es], [v for u, v in es]))
    with open(os.path.join(HERE, "er150_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
