"""ORACLE -- test infrastructure, not product code.

Plain, slow CPU implementations of what the counting path computes, written
from the paper (Problem 1, Alg. 2, Lemma 2, the batch protocol of Sec. 6)
and from the definition of induced 4-vertex graphlet counts.  Only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this package.  It shares no code with the HIP path and never
imports it.
"""
