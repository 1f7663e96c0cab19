"""Seeded synthetic signed bipartite graphs.

This package only draws inputs (vertex pairs and edge signs).  It holds none of
the counting arithmetic, so both the CPU oracle and the GPU library may take
their inputs from it without sharing any part of the method.
"""

from .graphs import (  # noqa: F401
    SignedGraph,
    uniform_graph,
    chung_lu_graph,
    config_graph,
    batch_graph,
    batch_graphs,
    pool_graph,
    pool_graphs,
    upload_graph,
    CONFIGS,
)
from .text import edge_text, messy_edge_text, raw_ids  # noqa: F401
