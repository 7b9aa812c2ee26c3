"""Bushy binary plans, written from the paper (oracle side; test
infrastructure only).

Section 2.2: a bushy plan runs as a series of left-deep plans.  Each join
node that is a right child is the root of a plan of its own, run first, and
its result is materialized; the parent plan then joins that result like a
base relation.  In the paper's example, (R join S) join (T join U) becomes
P1 = [T, U] and then P2 = [R, S, P1].  A materialized intermediate keeps
every attribute of the base tables under it (Section 5.2, run-time
comparison, where the paper describes its materialization), i.e. all of its
variables; here they are kept in increasing variable order.

A tree is an atom index (a leaf) or a pair (left, right) of trees.
"""

from __future__ import annotations

from typing import List, Sequence, Tuple, Union

import numpy as np

from datagen.synth import Relation, make_query

from . import cfj
from . import plans as P

Tree = Union[int, Tuple["Tree", "Tree"]]


def leaves(tree: Tree) -> List[int]:
    if isinstance(tree, int):
        return [tree]
    return leaves(tree[0]) + leaves(tree[1])


def decompose(tree: Tree) -> List[List[int]]:
    """The left-deep plans of ``tree`` in the order they run (the whole plan
    last).  A plan lists its inputs left to right; an input is an atom index
    or ``-(j + 1)`` for the result of plan ``j``."""
    out: List[List[int]] = []

    def plan_of(t: Tree) -> int:
        # a left-deep chain: descend through left children to the first
        # leaf; the right children met on the way join in, bottom-up
        inputs: List[int] = []

        def spine(u: Tree):
            if isinstance(u, int):
                inputs.append(u)
                return
            spine(u[0])
            r = u[1]
            if isinstance(r, int):
                inputs.append(r)
            else:
                inputs.append(-(plan_of(r) + 1))

        spine(t)
        out.append(inputs)
        return len(out) - 1

    plan_of(tree)
    return out


def evaluate(query, tree: Tree, batch: int = 1000, factor: bool = True):
    """Run ``tree`` on ``query`` by its decomposition with the oracle's Free
    Join (each left-deep plan converted by binary2fj, optionally factored).
    Returns dict(count, rows): rows in the query's head order, sorted."""
    if sorted(leaves(tree)) != list(range(len(query.atoms))):
        raise ValueError("the tree's leaves must be the query's atoms, once each")
    steps = decompose(tree)
    results = []   # per step: (variables in increasing order, column arrays)
    for k, inputs in enumerate(steps):
        last = k == len(steps) - 1
        vs = set()
        for x in inputs:
            vs |= set(query.atoms[x][1]) if x >= 0 else set(results[-x - 1][0])
        vs = sorted(vs)
        dense = {v: i for i, v in enumerate(vs)}
        rels, atoms, filters = [], [], []
        for x in inputs:
            if x >= 0:
                r, avars = query.atoms[x]
                rels.append(query.relations[r])
                atoms.append((len(rels) - 1, tuple(dense[v] for v in avars)))
                filters.append(query.filters[x])
            else:
                ivars, icols = results[-x - 1]
                rels.append(Relation(f"P{-x}", icols))
                atoms.append((len(rels) - 1, tuple(dense[v] for v in ivars)))
                filters.append(None)
        head = [dense[v] for v in query.head] if last else list(range(len(vs)))
        names = [query.var_names[v] for v in vs]
        qk = make_query(names, rels, atoms, filters, head)
        plan = P.binary2fj(qk, list(range(len(inputs))))
        if factor:
            plan = P.factor(plan)
        res = cfj.run(qk, plan, batch=batch, materialize=True, counters=False)
        if last:
            return {"count": res["count"], "rows": res["rows"]}
        rows = res["rows"]
        cols = [np.ascontiguousarray(rows[:, j], dtype=np.int32) if rows.shape[0]
                else np.zeros(0, np.int32) for j in range(len(vs))]
        results.append((vs, cols))
    raise AssertionError("unreachable")
