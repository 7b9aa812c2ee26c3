"""Helpers for GPU parity tests: build the same plans on both sides, run the
HIP path through the C-ABI binding and the oracle, compare."""

import numpy as np

from oracle import cfj
from oracle import plans as P


def gj_nodes(dq, var_order):
    """Generic Join plan written out directly: node i = every atom holding v_i."""
    return [[(a, (v,)) for a, (_, vs) in enumerate(dq.atoms) if v in vs] for v in var_order]


def oracle_run(dq, nodes, batch=1000, materialize=True, counters=True):
    return cfj.run(dq, [list(n) for n in nodes], batch=batch, materialize=materialize, counters=counters)


def assert_same_rows(got_rows, want_rows):
    assert got_rows.shape == want_rows.shape, (got_rows.shape, want_rows.shape)
    assert np.array_equal(got_rows, want_rows)


def oracle_plan_binary(dq, order, factor):
    p = P.binary2fj(dq, order)
    return P.factor(p) if factor else p
