"""Seeded synthetic workloads (graphs and update-batch streams).

This package only draws random inputs.  It holds none of the counting
method's arithmetic and is shared by the oracle, the tests and the
benchmark; neither side of a parity check imports the other through it.
"""
from .generators import (  # noqa: F401
    canon_keys, keys_to_edges, edges_to_keys,
    erdos_renyi, rmat_edges, rmat_graph, chung_lu_graph,
    BatchStream, er_batches, rmat_batches, chung_lu_batches,
    multi_graph_workload, raw_noise_batch, poisson_arrivals,
    log_uniform_sizes, chung_lu_weights,
)
from . import protocol  # noqa: F401,E402
