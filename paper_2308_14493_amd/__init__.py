"""MI355X-native batch fully dynamic 4-vertex graphlet counting.

The compute path is the HIP library libgraphlet4.so (csrc/, C ABI in
include/graphlet4.h); ``graphlet4`` is its Python binding.
"""
from .graphlet4 import Graph, Server, BatchStats, GraphletError, CLASSES, load  # noqa: F401
