"""Seeded synthetic inputs for the Free Join executor and for its oracle.

This package only draws random relations (numpy PCG64, explicit seeds).  It
contains none of the join arithmetic: no hashing, no plan logic, no counting.
Both the HIP path (through its Python binding) and the CPU oracle consume the
arrays produced here, which is the only thing the two sides share.
"""

from .synth import (  # noqa: F401
    Relation,
    Query,
    clover_instance,
    clover_u_instance,
    triangle_edges,
    star_schema,
    rmat_edges,
    zipf_keys,
    random_tiny_query,
    fanout_chain,
    batch_mix,
    batch_query,
    seed_for,
)
