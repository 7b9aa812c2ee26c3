"""Closed forms for result counts (oracle side; test infrastructure only).

A full conjunctive query counts homomorphisms, so with M_R the multiplicity
matrix of a binary bag relation R (M_R[u, v] = number of rows (u, v)):

* triangle R(x,y), S(y,z), T(z,x):  trace(M_R M_S M_T)
* k-cycle over one edge relation:    trace(A^k)
* chain R1(x0,x1) ... Rk(x_{k-1},x_k): 1^T M_1 ... M_k 1
* star F(k1..kd), D_i(k_i, a_i):      sum over fact rows f of prod_i deg_{D_i}(k_i(f))

These hold for any instance and are computed here with scipy/numpy,
independently of every other tier.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _mult_matrix(src: np.ndarray, dst: np.ndarray, n: int):
    data = np.ones(src.shape[0], dtype=np.int64)
    return sp.csr_matrix((data, (src.astype(np.int64), dst.astype(np.int64))), shape=(n, n))


def _domain(*cols) -> int:
    m = 0
    for c in cols:
        if c.size:
            if int(c.min()) < 0:
                raise ValueError("closed forms expect non-negative vertex ids")
            m = max(m, int(c.max()) + 1)
    return max(m, 1)


def triangle_count(r, s, t) -> int:
    """trace(M_R M_S M_T) for R(x,y), S(y,z), T(z,x); each arg = (col0, col1)."""
    n = _domain(*r, *s, *t)
    mr, ms, mt = (_mult_matrix(a, b, n) for a, b in (r, s, t))
    p = (mr @ ms)
    # trace(P M_T) = sum_{x,z} P[x,z] * M_T[z,x]
    return int(p.multiply(mt.T).sum())


def cycle_count(src, dst, k: int) -> int:
    """trace(A^k) for the k-cycle over one edge relation (k >= 2)."""
    n = _domain(src, dst)
    a = _mult_matrix(src, dst, n)
    half = k // 2
    p = a
    for _ in range(half - 1):
        p = p @ a
    if k % 2 == 0:
        # trace(P P) = sum_{u,v} P[u,v] P[v,u]
        return int(p.multiply(p.T).sum())
    q = p @ a
    return int(q.multiply(p.T).sum())


def cycle4_count_blocked(src, dst, rows_per_block: int = 1 << 14) -> int:
    """trace(A^4) = sum over (u, v) of (A^2)[u, v] (A^2)[v, u], with A^2
    formed one block of rows u at a time: the block's rows A[U, :] A and
    its columns A A[:, U] (transposed) are multiplied elementwise and summed,
    so memory stays bounded for graphs whose A^2 does not fit."""
    n = _domain(src, dst)
    a = _mult_matrix(src, dst, n)
    ac = a.tocsc()
    total = 0
    for u0 in range(0, n, rows_per_block):
        u1 = min(n, u0 + rows_per_block)
        rows = a[u0:u1, :] @ a                # (A^2)[U, :]
        cols = (a @ ac[:, u0:u1]).T.tocsr()   # (A^2)[:, U] transposed
        total += int(rows.multiply(cols).sum())
    return total


def chain_count(rels) -> int:
    """1^T M_1 ... M_k 1 for R1(x0,x1), ..., Rk(x_{k-1},x_k)."""
    n = _domain(*[c for r in rels for c in r])
    v = np.ones(n, dtype=np.int64)
    for a, b in reversed(rels):
        m = _mult_matrix(a, b, n)
        v = m @ v
    return int(v.sum())


def star_count(fact_cols, dims, dim_filters=None) -> int:
    """sum_f prod_i deg_{D_i'}(k_i(f)); dims[i] = (pk, attr), and
    dim_filters[i] = None or c (keep rows with attr < c)."""
    total = None
    for i, (kcol, (pk, attr)) in enumerate(zip(fact_cols, dims)):
        keep = np.ones(pk.shape[0], bool)
        if dim_filters is not None and dim_filters[i] is not None:
            keep = attr < dim_filters[i]
        pk = pk[keep]
        n = _domain(kcol, pk)
        deg = np.bincount(pk.astype(np.int64), minlength=n).astype(np.int64)
        term = deg[kcol.astype(np.int64)]
        total = term if total is None else total * term
    return int(total.sum())


def star_rows(fact_cols, dims, dim_filters=None) -> np.ndarray:
    """The star result for primary-key dimensions (each key at most once per
    dimension), as sorted int32 rows (k1..kd, a1..ad)."""
    d = len(fact_cols)
    nf = fact_cols[0].shape[0]
    alive = np.ones(nf, bool)
    attrs = []
    for i, (kcol, (pk, attr)) in enumerate(zip(fact_cols, dims)):
        keep = np.ones(pk.shape[0], bool)
        if dim_filters is not None and dim_filters[i] is not None:
            keep = attr < dim_filters[i]
        pk_k, at_k = pk[keep].astype(np.int64), attr[keep]
        if np.unique(pk_k).shape[0] != pk_k.shape[0]:
            raise ValueError("star_rows needs unique dimension keys")
        n = _domain(kcol, pk_k)
        lut = np.full(n, -1, np.int64)
        lut[pk_k] = np.arange(pk_k.shape[0])
        idx = lut[kcol.astype(np.int64)]
        alive &= idx >= 0
        attrs.append((idx, at_k))
    rows = [c[alive] for c in fact_cols]
    for idx, at in attrs:
        rows.append(at[idx[alive]])
    out = np.stack(rows, axis=1).astype(np.int32) if rows else np.zeros((0, 2 * d), np.int32)
    return sort_rows(out)


def sort_rows(rows: np.ndarray) -> np.ndarray:
    """Lexicographic sort of int32 rows (signed), first column most significant."""
    if rows.shape[0] == 0:
        return rows
    keys = [rows[:, j] for j in range(rows.shape[1] - 1, -1, -1)]
    return rows[np.lexsort(keys)]
