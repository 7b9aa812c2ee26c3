"""Run a conjunctive query end to end through libfj.

Uploads column-stored relations with torch, applies pushed-down selections
with the library's filter kernel, builds the plan and the COLTs, and runs the
join.  Only argument marshalling happens here; all join work is in libfj.
"""

from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import fj


class DeviceQuery:
    """Relations of a ``datagen`` query resident on one GPU."""

    def __init__(self, ctx: fj.Context, dq, device: Optional[str] = None):
        import torch
        self.ctx = ctx
        self.dq = dq
        dev = device or f"cuda:{ctx.device}"
        self.rel_cols = [[torch.from_numpy(np.ascontiguousarray(c, dtype=np.int32)).to(dev) for c in r.cols]
                         for r in dq.relations]
        self.q = fj.make_query([vs for _, vs in dq.atoms], dq.nvars, dq.head)
        self.sel: List = [None] * len(dq.atoms)
        self.nsel: List[int] = [0] * len(dq.atoms)
        self._flt = None      # selections' marshalled arguments (the buffers are fixed)
        self._rb = None       # (COLT handles, handle array, relation array) of the last rebuild
        self._sr = None       # the same for select_rebuild, with the selections' arrays
        self.apply_filters()

    def apply_filters(self):
        import torch
        if self._flt is None:
            specs, atoms = [], []
            for a, f in enumerate(self.dq.filters):
                if f is None:
                    continue
                col = self.rel_cols[self.dq.atoms[a][0]][f[0]]
                if self.sel[a] is None:
                    self.sel[a] = torch.empty(max(int(col.shape[0]), 1), dtype=torch.int32, device=col.device)
                specs.append((col, f[1], self.sel[a]))
                atoms.append(a)
            self._flt = (atoms, fj.filter_args(specs) if specs else None)
        atoms, args = self._flt
        if args is None:
            return
        self.ctx.filter_lt_prepared(args)
        counts = args[-1]
        for i, a in enumerate(atoms):
            self.nsel[a] = int(counts[i])

    def atom_cols(self, a: int):
        return self.rel_cols[self.dq.atoms[a][0]]

    def plan_binary(self, order: Sequence[int], factor: bool = True) -> fj.Plan:
        return fj.plan_from_binary(self.q, list(order), factor)

    def plan_nodes(self, nodes) -> fj.Plan:
        return fj.plan_from_nodes(self.q, nodes)

    def sketches(self) -> List[fj.Sketch]:
        """Exact per-atom column statistics of the (selected) rows, on the GPU."""
        return [self.ctx.sketch(self.atom_cols(a), self.sel[a], self.nsel[a]) for a in range(len(self.dq.atoms))]

    def candidates(self, sketches):
        return fj.plan_candidates(self.q, sketches)

    def candidate_plan(self, cand) -> fj.Plan:
        return fj.candidate_plan(self.q, cand)

    def choose(self, mlp, sketches, margin: float = 0.0, gate_rows: int = 0):
        """(plan, candidate index, scores) chosen by the learned chooser."""
        return self.ctx.choose_plan(self.q, sketches, mlp, margin, gate_rows)

    def build(self, plan: fj.Plan):
        return [self.ctx.build_colt(self.q, plan, a, self.atom_cols(a), self.sel[a], self.nsel[a])
                for a in range(len(self.dq.atoms))]

    def rebuild(self, colts):
        """Rebuild every COLT of the query in one grouped pass.  The relation
        array is marshalled once per set of COLTs; later calls only update
        the selection sizes."""
        import ctypes as C
        n = len(colts)
        if n == 0:
            return
        key = tuple(c.h for c in colts)
        if self._rb is None or self._rb[0] != key:
            specs = [(self.atom_cols(a), self.sel[a], self.nsel[a]) for a in range(n)]
            rels = (fj.Relation * n)(*[fj._relation(*sp) for sp in specs])
            self._rb = (key, (C.c_void_p * n)(*key), rels)
            for c, sp in zip(colts, specs):
                c.keep = (sp[0], sp[1])
        else:
            rels = self._rb[2]
            for a in range(n):
                if self.sel[a] is not None:
                    rels[a].nsel = int(self.nsel[a])
        self.ctx.rebuild_colts_prepared(n, self._rb[1], self._rb[2])

    def select_rebuild(self, colts):
        """The query's selections and then one grouped rebuild of its COLTs,
        in one library call with one host wait (apply_filters() followed by
        rebuild(colts)).  The arrays are marshalled once per set of COLTs."""
        import ctypes as C
        n = len(colts)
        key = tuple(c.h for c in colts)
        if self._sr is None or self._sr[0] != key:
            specs = [(self.atom_cols(a), self.sel[a], self.nsel[a]) for a in range(n)]
            rels = (fj.Relation * n)(*[fj._relation(*sp) for sp in specs])
            for c, sp in zip(colts, specs):
                c.keep = (sp[0], sp[1])
            fa = [a for a in range(n) if self.dq.filters[a] is not None]
            m = max(len(fa), 1)
            atoms = (C.c_int32 * m)(*fa)
            cols = (C.c_int32 * m)(*[int(self.dq.filters[a][0]) for a in fa])
            bounds = (C.c_int32 * m)(*[int(self.dq.filters[a][1]) for a in fa])
            self._sr = (key, (C.c_void_p * n)(*key), rels, atoms, cols, bounds, fa)
        _, arr, rels, atoms, cols, bounds, fa = self._sr
        self.ctx.select_rebuild_prepared(len(fa), atoms, cols, bounds, n, arr, rels)
        for a in fa:
            self.nsel[a] = int(rels[a].nsel)

    def run(self, plan: fj.Plan, materialize: bool = True, cap: Optional[int] = None,
            stats: bool = False, colts=None):
        """Returns dict(count, rows (sorted numpy or None), written, stats)."""
        import torch
        if colts is None:
            colts = self.build(plan)
        out = None
        if materialize:
            if cap is None:
                cnt, _, _ = self.ctx.execute(self.q, plan, colts)
                cap = cnt
                self.rebuild(colts)
            out = torch.empty((max(int(cap), 1), self.q.nhead), dtype=torch.int32,
                              device=f"cuda:{self.ctx.device}")
            if cap == 0:
                out = out[:0]
        cnt, written, st = self.ctx.execute(self.q, plan, colts, out=out if materialize and cap else None,
                                            stats=stats)
        rows = None
        if materialize:
            rows = out[:written].cpu().numpy() if written else np.zeros((0, self.q.nhead), np.int32)
            rows = sort_rows(rows)
        return {"count": cnt, "rows": rows, "written": written, "stats": st, "colts": colts}


    def run_factorized(self, plan: fj.Plan, page: Optional[int] = None, colts=None):
        """Run with a factorized result, then expand it page by page (all at
        once when page is None).  Returns dict(count, bindings, rows (sorted
        numpy), pages)."""
        import torch
        if colts is None:
            colts = self.build(plan)
        res = self.ctx.execute_factorized(self.q, plan, colts)
        try:
            n = res.count
            page = max(int(page if page is not None else n), 1)
            out = torch.empty((min(page, max(n, 1)), self.q.nhead), dtype=torch.int32,
                              device=f"cuda:{self.ctx.device}")
            parts, first, pages = [], 0, 0
            while first < n:
                w = res.expand(first, out)
                if w == 0:
                    raise RuntimeError("expansion wrote no rows")
                parts.append(out[:w].cpu().numpy())
                first += w
                pages += 1
            rows = np.concatenate(parts) if parts else np.zeros((0, self.q.nhead), np.int32)
            return {"count": n, "bindings": res.bindings, "rows": sort_rows(rows), "unsorted": rows,
                    "pages": pages}
        finally:
            res.free()

    def run_bushy(self, tree, materialize: bool = True, factor: bool = True):
        """Run a binary plan (nested pairs of atom indices) by its left-deep
        decomposition.  Returns dict(count, rows (sorted numpy or None), written)."""
        import torch
        rels = [(self.atom_cols(a), self.sel[a], self.nsel[a]) for a in range(len(self.dq.atoms))]
        cnt, _ = self.ctx.execute_bushy(self.q, tree, rels, factor=factor)
        if not materialize:
            return {"count": cnt, "rows": None, "written": 0}
        out = torch.empty((max(int(cnt), 1), self.q.nhead), dtype=torch.int32, device=f"cuda:{self.ctx.device}")
        cnt2, written = self.ctx.execute_bushy(self.q, tree, rels, factor=factor, out=out)
        rows = out[:written].cpu().numpy() if written else np.zeros((0, self.q.nhead), np.int32)
        return {"count": cnt2, "rows": sort_rows(rows), "written": written}


def sort_rows(rows: np.ndarray) -> np.ndarray:
    if rows.shape[0] == 0:
        return rows
    keys = [rows[:, j] for j in range(rows.shape[1] - 1, -1, -1)]
    return rows[np.lexsort(keys)]
