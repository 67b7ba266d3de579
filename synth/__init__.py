"""Seeded synthetic graph generators.

This module only produces raw inputs (edge lists, possibly with self-loops and
repeated pairs, plus arrival times for request streams).  It holds none of the
decomposition's arithmetic: canonicalisation, clique enumeration and the
h-index iteration live on the two sides that consume these inputs (the CPU
oracle and the HIP library), which never share code.
"""

from .graphs import (  # noqa: F401
    RawGraph,
    books,
    erdos_renyi,
    chung_lu,
    chung_lu_weights,
    sbm,
    request_stream,
    workload,
    WORKLOADS,
)
