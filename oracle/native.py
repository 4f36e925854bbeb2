"""ORACLE -- test infrastructure.  ctypes wrapper of oracle.c.

``static_counts``  the static recount of Sec. 4.1 (the baseline recounts the
                   whole updated graph after every batch), 11 induced classes.
``brute_counts``   the plain definition: classify every 4-subset.
``static_counts_merge``  the same recount through a second formulation
                   (sorted merges per edge in id order), for cross-checks.
``sample_seconds`` time of the recount's loops over a sample of vertices.
``static_counts3`` / ``brute3_counts``  the four induced 3-vertex counts.
Results are exact Python ints (the C side works in __int128).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle library (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.static_counts.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P, P, P]
        lib.static_counts.restype = ctypes.c_int
        lib.static_counts_merge.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P]
        lib.static_counts_merge.restype = ctypes.c_int
        lib.brute_counts.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P]
        lib.brute_counts.restype = ctypes.c_int
        lib.static_counts_sample_time.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int64,
                                                  ctypes.c_int64, P]
        lib.static_counts_sample_time.restype = ctypes.c_int
        for fn in ("brute3_counts", "static_counts3"):
            getattr(lib, fn).argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P]
            getattr(lib, fn).restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _join(hi, lo):
    return [(int(h) << 64) | int(l) for h, l in zip(hi.tolist(), lo.tolist())]


def _edges(src, dst):
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    assert s.shape == d.shape
    return s, d


def static_counts(n: int, src, dst, with_terms: bool = False):
    """Induced 4-vertex counts of the simple graph given by (src, dst)."""
    lib = _load()
    s, d = _edges(src, dst)
    hi = np.zeros(11, np.int64); lo = np.zeros(11, np.uint64)
    shi = np.zeros(9, np.int64); slo = np.zeros(9, np.uint64)
    rc = lib.static_counts(n, s.size, s.ctypes.data, d.ctypes.data, hi.ctypes.data,
                           lo.ctypes.data, shi.ctypes.data, slo.ctypes.data)
    if rc != 0:
        raise ValueError("oracle static_counts failed (%d): not a simple graph?" % rc)
    counts = _join(hi, lo)
    if with_terms:
        names = ["N_P4", "N_K13", "N_C4", "N_paw", "N_diamond", "N_K4", "T", "W", "m"]
        return counts, dict(zip(names, _join(shi, slo)))
    return counts


def static_counts_merge(n: int, src, dst):
    """static_counts through the merge formulation (O(sum of d^2) steps)."""
    lib = _load()
    s, d = _edges(src, dst)
    hi = np.zeros(11, np.int64); lo = np.zeros(11, np.uint64)
    rc = lib.static_counts_merge(n, s.size, s.ctypes.data, d.ctypes.data, hi.ctypes.data, lo.ctypes.data)
    if rc != 0:
        raise ValueError("oracle static_counts_merge failed (%d)" % rc)
    return _join(hi, lo)


def brute_counts(n: int, src, dst):
    """Induced 4-vertex counts by enumerating all C(n,4) subsets (n <= 4096)."""
    lib = _load()
    s, d = _edges(src, dst)
    hi = np.zeros(11, np.int64); lo = np.zeros(11, np.uint64)
    rc = lib.brute_counts(n, s.size, s.ctypes.data, d.ctypes.data, hi.ctypes.data, lo.ctypes.data)
    if rc != 0:
        raise ValueError("oracle brute_counts failed (%d)" % rc)
    return _join(hi, lo)


def sample_seconds(n: int, src, dst, stride: int, offset: int = 0):
    """(build seconds, seconds of the per-vertex loops of static_counts over
    the vertices offset, offset + stride, ...).  No counts: timing only."""
    lib = _load()
    s, d = _edges(src, dst)
    secs = np.zeros(2, np.float64)
    rc = lib.static_counts_sample_time(n, s.size, s.ctypes.data, d.ctypes.data, stride, offset, secs.ctypes.data)
    if rc != 0:
        raise ValueError("oracle static_counts_sample_time failed (%d)" % rc)
    return float(secs[0]), float(secs[1])


def _counts3(fn, n, src, dst):
    lib = _load()
    s, d = _edges(src, dst)
    hi = np.zeros(4, np.int64); lo = np.zeros(4, np.uint64)
    rc = getattr(lib, fn)(n, s.size, s.ctypes.data, d.ctypes.data, hi.ctypes.data, lo.ctypes.data)
    if rc != 0:
        raise ValueError("oracle %s failed (%d)" % (fn, rc))
    return _join(hi, lo)


def static_counts3(n: int, src, dst):
    """Induced 3-vertex counts [triangle, 2-path, edge + isolated, empty]
    from the static recount's totals."""
    return _counts3("static_counts3", n, src, dst)


def brute3_counts(n: int, src, dst):
    """Induced 3-vertex counts by enumerating all C(n,3) subsets (n <= 4096)."""
    return _counts3("brute3_counts", n, src, dst)


def threads() -> int:
    return int(_load().oracle_threads())
