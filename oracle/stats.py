"""Column statistics and the greedy left-deep order -- TEST INFRASTRUCTURE
ONLY (see the package header).

* ``sketch``: the distinct count of each column and its largest value
  frequencies, by their definition (a sort-based unique with counts).
* ``greedy_order``: the stand-in for the cost-based optimizer whose binary
  plans Section 4.1 converts.  Textbook estimates (System R style): the
  join of a placed prefix J with a relation R on shared variables v has
  |J| |R| / prod_v max(V(J,v), V(R,v)) tuples, with V(J,v) the smallest
  distinct count of v over the placed atoms, every V capped at |J| (and at
  least 1) after each placement.  The order starts at the largest relation
  (a traditional plan iterates its largest relation, Section 4.4) or at a
  given atom; a relation sharing no variable is placed only when no
  connected one is left, the smallest first; ties go to the lower atom
  index.  The estimate is evaluated as (|J| * |R|) / P with P multiplied
  over R's columns in column order, and rows and distinct counts are taken
  as at least 1.

Pinned by tests/test_oracle_stats.py with hand-worked examples.
"""

from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

TOPK = 8


def column_sketch(col: np.ndarray) -> Dict:
    col = np.asarray(col)
    if col.size == 0:
        return {"distinct": 0, "top": [0] * TOPK}
    _, counts = np.unique(col, return_counts=True)
    top = sorted((int(c) for c in counts), reverse=True)[:TOPK]
    return {"distinct": int(counts.size), "top": top + [0] * (TOPK - len(top))}


def sketch(cols: Sequence[np.ndarray], sel: np.ndarray = None) -> Dict:
    """Sketch of the rows of a relation (restricted to sel when given)."""
    cols = [np.asarray(c) for c in cols]
    if sel is not None:
        cols = [c[np.asarray(sel, dtype=np.int64)] for c in cols]
    per = [column_sketch(c) for c in cols]
    return {"rows": int(cols[0].size) if cols else 0,
            "distinct": [p["distinct"] for p in per], "top": [p["top"] for p in per]}


def greedy_order(atoms: Sequence[Sequence[int]], sketches: Sequence[Dict], first: int = -1) -> List[int]:
    """atoms[a] = the variable of each column of atom a."""
    n = len(atoms)

    def rows(a):
        return max(1.0, float(sketches[a]["rows"]))

    def dist(a, v):
        j = list(atoms[a]).index(v)
        return max(1.0, float(sketches[a]["distinct"][j]))

    if first < 0:
        first = max(range(n), key=lambda a: (sketches[a]["rows"], -a))
    order = [first]
    J = rows(first)
    V = {}
    for v in atoms[first]:
        V[v] = min(dist(first, v), V.get(v, float("inf")))
    V = {v: max(1.0, min(x, J)) for v, x in V.items()}
    while len(order) < n:
        best, best_est = None, None
        for a in range(n):
            if a in order:
                continue
            shared = [v for v in atoms[a] if v in V]
            if not shared:
                continue
            P = 1.0
            for v in atoms[a]:
                if v in V:
                    P *= max(V[v], dist(a, v))
            est = (J * rows(a)) / P
            if best is None or est < best_est:
                best, best_est = a, est
        if best is None:
            rest = [a for a in range(n) if a not in order]
            best = min(rest, key=lambda a: (sketches[a]["rows"], a))
            best_est = J * rows(best)
        order.append(best)
        J = best_est
        for v in atoms[best]:
            d = dist(best, v)
            V[v] = min(V[v], d) if v in V else d
        V = {v: max(1.0, min(x, J)) for v, x in V.items()}
    return order
