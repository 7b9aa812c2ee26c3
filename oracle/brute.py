"""The definition of the query result, enumerated by nested loops (oracle side;
test infrastructure only).

For a full conjunctive query over bags (Section 2.1, eq. "cq"), the result is
the multiset holding the head tuple of nu once for every choice of one row
per atom (rows counted individually, so duplicate rows are distinct choices)
under which all atoms agree on their shared variables; nu is then unique
because every variable occurs in some atom.  Pushed-down selections restrict
an atom to the rows that satisfy ``column < constant``.
"""

from __future__ import annotations

from typing import List, Tuple


def atom_rows(query, a: int) -> List[Tuple[int, ...]]:
    cols = query.atom_cols(a)
    n = query.atom_rows(a)
    f = query.filters[a]
    rows = []
    for i in range(n):
        if f is not None and not (int(cols[f[0]][i]) < f[1]):
            continue
        rows.append(tuple(int(c[i]) for c in cols))
    return rows


def enumerate_result(query) -> List[Tuple[int, ...]]:
    """All result tuples in head order, duplicates kept, sorted."""
    tables = [atom_rows(query, a) for a in range(len(query.atoms))]
    out = []
    nu = {}

    def rec(i):
        if i == len(tables):
            out.append(tuple(nu[v] for v in query.head))
            return
        vars_i = query.atoms[i][1]
        for row in tables[i]:
            added = []
            ok = True
            for v, val in zip(vars_i, row):
                if v in nu:
                    if nu[v] != val:
                        ok = False
                        break
                else:
                    nu[v] = val
                    added.append(v)
            if ok:
                rec(i + 1)
            for v in added:
                del nu[v]

    rec(0)
    out.sort()
    return out


def count(query) -> int:
    return len(enumerate_result(query))
