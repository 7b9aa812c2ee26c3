"""ctypes front end of the C Free Join oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

from . import plans as P

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fj_oracle.c")
LIB = os.path.join(HERE, "libfj_oracle.so")
MAXC = 8
NCTR = 6
CTR_NAMES = ("cover", "probe", "hit", "survivors", "forced", "forced_offsets")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, -O2)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        lib = C.CDLL(LIB)
        f = lib.ofj_execute
        f.restype = C.c_int
        f.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                      C.c_void_p, C.c_void_p,
                      C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                      C.c_int, C.c_int, C.c_void_p,
                      C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]
        _lib = lib
    return _lib


def selection(query, a: int) -> Optional[np.ndarray]:
    """Offsets of the rows of atom a that pass its pushed-down selection."""
    f = query.filters[a]
    if f is None:
        return None
    col = query.atom_cols(a)[f[0]]
    return np.nonzero(col < f[1])[0].astype(np.uint32)


def run(query, plan, batch: int = 1000, materialize: bool = True,
        cap: Optional[int] = None, counters: bool = True):
    """Execute ``plan`` on ``query``.  Returns dict(count, rows, counters).

    ``rows`` are the head-ordered result rows sorted lexicographically
    (signed int32), or None when not materialized."""
    lib = _load()
    P.validate(query, plan)
    na = len(query.atoms)
    keep = []  # keep numpy buffers alive
    arity = np.zeros(na, np.int32)
    avars = np.full(na * MAXC, -1, np.int32)
    colp = (C.c_void_p * (na * MAXC))()
    nrows = np.zeros(na, np.int64)
    selp = (C.c_void_p * na)()
    nsel = np.zeros(na, np.int64)
    for a, (r, vs) in enumerate(query.atoms):
        cols = query.relations[r].cols
        arity[a] = len(vs)
        for j, v in enumerate(vs):
            avars[a * MAXC + j] = v
            c = np.ascontiguousarray(cols[j], dtype=np.int32)
            keep.append(c)
            colp[a * MAXC + j] = c.ctypes.data
        nrows[a] = query.relations[r].nrows
        s = selection(query, a)
        if s is not None:
            s = np.ascontiguousarray(s) if s.size else np.zeros(1, np.uint32)
            keep.append(s)
            selp[a] = s.ctypes.data
            nsel[a] = int((query.atom_cols(a)[query.filters[a][0]] < query.filters[a][1]).sum())
    nnodes = len(plan)
    node_nsub = np.array([len(n) for n in plan], np.int32)
    subs = [sa for n in plan for sa in n]
    sub_atom = np.array([a for a, _ in subs], np.int32)
    sub_nv = np.array([len(vs) for _, vs in subs], np.int32)
    sub_vars = np.full(max(1, len(subs)) * MAXC, -1, np.int32)
    for i, (_, vs) in enumerate(subs):
        sub_vars[i * MAXC:i * MAXC + len(vs)] = vs
    head = np.array(query.head, np.int32)
    nh = len(query.head)
    if materialize and cap is None:
        # count first, then size the buffer exactly
        pre = run(query, plan, batch=batch, materialize=False, counters=False)
        cap = pre["count"]
    cap = int(cap or 0) if materialize else 0
    out = np.zeros((max(cap, 1), max(nh, 1)), np.int32)
    cnt = C.c_uint64(0)
    wr = C.c_uint64(0)
    ctr = np.zeros((nnodes + 1) * NCTR, np.uint64)
    rc = lib.ofj_execute(na, arity.ctypes.data, avars.ctypes.data, C.cast(colp, C.c_void_p),
                         nrows.ctypes.data, C.cast(selp, C.c_void_p), nsel.ctypes.data,
                         query.nvars, nnodes, node_nsub.ctypes.data, sub_atom.ctypes.data,
                         sub_nv.ctypes.data, sub_vars.ctypes.data, int(batch), nh,
                         head.ctypes.data, C.byref(cnt),
                         out.ctypes.data if materialize else None, cap, C.byref(wr),
                         ctr.ctypes.data if counters else None)
    if rc != 0:
        raise RuntimeError(f"oracle failed with status {rc}")
    rows = None
    if materialize:
        rows = out[: wr.value]
        if rows.shape[0]:
            keys = [rows[:, j] for j in range(rows.shape[1] - 1, -1, -1)]
            rows = rows[np.lexsort(keys)]
    res = {"count": int(cnt.value), "rows": rows, "written": int(wr.value)}
    if counters:
        m = ctr.reshape(nnodes + 1, NCTR)
        res["counters"] = [dict(zip(CTR_NAMES, map(int, m[k]))) for k in range(nnodes)]
        res["build"] = dict(zip(CTR_NAMES, map(int, m[nnodes])))
    return res
