"""Python binding of libfj (include/fj.h): argument marshalling only.

Every step of the join runs in the library's HIP kernels; PyTorch provides the
device memory and the stream.  Importing this module fails loudly when
libfj.so has not been built: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfj.so")

MAX_COLS = 8
MAX_ATOMS = 16
MAX_VARS = 32
MAX_NODES = 16
FACTOR = 1
SKETCH_TOPK = 8
CAND_MAX = 32
FEATURES = 128
CAND_BINARY = 0
CAND_GJ = 1

STATUS = {0: "FJ_OK", 1: "FJ_TRUNCATED", -1: "FJ_ERR_ARG", -2: "FJ_ERR_PLAN_INVALID",
          -3: "FJ_ERR_PLAN_NO_PURE_COVER", -4: "FJ_ERR_OOM", -5: "FJ_ERR_HIP", -6: "FJ_ERR_UNSUPPORTED",
          -7: "FJ_ERR_INTERNAL"}
TIMERS = ("filter", "build", "cover", "probe", "probe0", "force", "emit", "scan")


class FJError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Relation(C.Structure):
    _fields_ = [("ncols", C.c_int32), ("nrows", C.c_int64),
                ("cols", C.c_void_p * MAX_COLS), ("sel", C.c_void_p), ("nsel", C.c_int64)]


class Atom(C.Structure):
    _fields_ = [("arity", C.c_int32), ("vars", C.c_int32 * MAX_COLS)]


class QueryS(C.Structure):
    _fields_ = [("natoms", C.c_int32), ("atoms", Atom * MAX_ATOMS), ("nvars", C.c_int32),
                ("nhead", C.c_int32), ("head", C.c_int32 * MAX_VARS)]


class Options(C.Structure):
    _fields_ = [("tile", C.c_int64), ("block", C.c_int32), ("timing", C.c_int32),
                ("tail", C.c_int32), ("generic", C.c_int32), ("trie", C.c_int32), ("no_filter", C.c_int32),
                ("reserved", C.c_int32 * 1)]


class Stats(C.Structure):
    _fields_ = [("cover", C.c_uint64 * MAX_NODES), ("probe", C.c_uint64 * MAX_NODES),
                ("hit", C.c_uint64 * MAX_NODES), ("survivors", C.c_uint64 * MAX_NODES),
                ("forced", C.c_uint64 * MAX_NODES), ("forced_offsets", C.c_uint64 * MAX_NODES),
                ("tail_from", C.c_int32), ("nnodes", C.c_int32), ("tiles", C.c_uint64),
                ("deferred", C.c_uint64), ("filtered", C.c_uint64)]

    def per_node(self):
        n = self.nnodes
        keys = ("cover", "probe", "hit", "survivors", "forced", "forced_offsets")
        return [{k: int(getattr(self, k)[i]) for k in keys} for i in range(n)]


class Sketch(C.Structure):
    _fields_ = [("rows", C.c_int64), ("ncols", C.c_int32), ("distinct", C.c_int64 * MAX_COLS),
                ("top", (C.c_int64 * SKETCH_TOPK) * MAX_COLS)]

    def as_dict(self):
        n = self.ncols
        return {"rows": int(self.rows), "distinct": [int(self.distinct[j]) for j in range(n)],
                "top": [[int(self.top[j][k]) for k in range(SKETCH_TOPK)] for j in range(n)]}


MAX_BUSHY = 2 * MAX_ATOMS - 1


class Bushy(C.Structure):
    """A binary join plan (fj_bushy): node i is a leaf when atom[i] >= 0,
    else the join of nodes left[i] and right[i]."""
    _fields_ = [("n", C.c_int32), ("root", C.c_int32), ("atom", C.c_int32 * MAX_BUSHY),
                ("left", C.c_int32 * MAX_BUSHY), ("right", C.c_int32 * MAX_BUSHY)]


def bushy(tree) -> Bushy:
    """A Bushy from a nested tree: an int is an atom, a pair (l, r) a join."""
    b = Bushy()
    nodes = []

    def add(t):
        if isinstance(t, int):
            nodes.append((int(t), -1, -1))
        else:
            l, r = t
            li = add(l)
            ri = add(r)
            nodes.append((-1, li, ri))
        return len(nodes) - 1

    b.root = add(tree)
    b.n = len(nodes)
    if b.n > MAX_BUSHY:
        raise ValueError("plan too large")
    for i, (a, l, r) in enumerate(nodes):
        b.atom[i] = a
        b.left[i] = l
        b.right[i] = r
    return b


def bushy_decompose(tree) -> List[List[int]]:
    """The left-deep plans of a binary plan, in evaluation order (host only):
    inputs are atom indices, or -(j + 1) for the result of plan j."""
    b = tree if isinstance(tree, Bushy) else bushy(tree)
    n = C.c_int32(0)
    ninp = (C.c_int32 * MAX_BUSHY)()
    inp = (C.c_int32 * (MAX_BUSHY * MAX_ATOMS))()
    _check(lib().fj_bushy_decompose(C.byref(b), C.byref(n), ninp, inp))
    return [[int(inp[k * MAX_ATOMS + i]) for i in range(ninp[k])] for k in range(n.value)]


class Candidate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("order", C.c_int32 * MAX_VARS)]

    def key(self):
        return (int(self.kind), tuple(int(self.order[i]) for i in range(self.n)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2301_10841_amd/build.py "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.fj_last_error.restype = C.c_char_p
        L.fj_ctx_create.argtypes = [C.c_int, vp, P(Options), P(vp)]
        L.fj_ctx_destroy.argtypes = [vp]
        L.fj_ctx_destroy.restype = None
        L.fj_timings.argtypes = [vp, vp, vp]
        L.fj_timings_reset.argtypes = [vp]
        L.fj_set_timing.argtypes = [vp, C.c_int32]
        L.fj_plan_from_binary.argtypes = [P(QueryS), vp, C.c_int32, C.c_uint32, P(vp)]
        L.fj_plan_from_nodes.argtypes = [P(QueryS), C.c_int32, vp, vp, vp, vp, P(vp)]
        L.fj_plan_get.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32]
        L.fj_plan_free.argtypes = [vp]
        L.fj_plan_free.restype = None
        L.fj_filter_lt.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, P(C.c_int64)]
        L.fj_filter_lt_noalloc.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, P(C.c_int64)]
        L.fj_filter_lt_batch.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp]
        L.fj_build_colt.argtypes = [vp, P(QueryS), vp, C.c_int32, P(Relation), P(vp)]
        L.fj_colt_rebuild.argtypes = [vp, vp, P(Relation)]
        L.fj_colt_rebuild_many.argtypes = [vp, C.c_int32, vp, vp]
        L.fj_select_rebuild.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int32, vp, vp]
        L.fj_colt_free.argtypes = [vp]
        L.fj_colt_free.restype = None
        L.fj_execute.argtypes = [vp, P(QueryS), vp, vp, P(C.c_uint64), vp, C.c_uint64,
                                 P(C.c_uint64), P(Stats)]
        L.fj_bushy_decompose.argtypes = [P(Bushy), P(C.c_int32), vp, vp]
        L.fj_execute_bushy.argtypes = [vp, P(QueryS), P(Bushy), vp, C.c_uint32, P(C.c_uint64), vp, C.c_uint64,
                                       P(C.c_uint64)]
        L.fj_execute_factorized.argtypes = [vp, P(QueryS), vp, vp, P(vp), P(C.c_uint64), P(C.c_uint64)]
        L.fj_result_expand.argtypes = [vp, vp, C.c_uint64, vp, C.c_uint64, P(C.c_uint64)]
        L.fj_result_free.argtypes = [vp]
        L.fj_result_free.restype = None
        L.fj_batch_create.argtypes = [vp, C.c_int32, vp, vp, vp, vp, P(vp)]
        L.fj_batch_run.argtypes = [vp, vp]
        L.fj_batch_free.argtypes = [vp]
        L.fj_batch_free.restype = None
        L.fj_sketch_relation.argtypes = [vp, P(Relation), P(Sketch)]
        L.fj_greedy_order.argtypes = [P(QueryS), vp, C.c_int32, vp]
        L.fj_plan_candidates.argtypes = [P(QueryS), vp, C.c_int32, vp, P(C.c_int32), vp]
        L.fj_candidate_plan.argtypes = [P(QueryS), P(Candidate), P(vp)]
        L.fj_mlp_create.argtypes = [vp, C.c_int32, C.c_int32, P(vp)]
        L.fj_mlp_param_count.argtypes = [vp]
        L.fj_mlp_param_count.restype = C.c_int64
        L.fj_mlp_set_params.argtypes = [vp, vp, C.c_int64]
        L.fj_mlp_get_params.argtypes = [vp, vp, C.c_int64]
        L.fj_mlp_forward.argtypes = [vp, vp, C.c_int32, vp]
        L.fj_mlp_gradient.argtypes = [vp, vp, vp, C.c_int32, vp, P(C.c_float)]
        L.fj_mlp_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, vp]
        L.fj_mlp_free.argtypes = [vp]
        L.fj_mlp_free.restype = None
        L.fj_choose_plan.argtypes = [vp, vp, P(QueryS), vp, C.c_float, C.c_uint64, P(vp), P(C.c_int32), vp]
        for name in ("fj_ctx_create", "fj_timings", "fj_timings_reset", "fj_plan_from_binary",
                     "fj_plan_from_nodes", "fj_plan_get", "fj_filter_lt", "fj_filter_lt_batch", "fj_build_colt",
                     "fj_colt_rebuild", "fj_colt_rebuild_many", "fj_select_rebuild", "fj_execute",
                     "fj_execute_factorized",
                     "fj_result_expand", "fj_execute_bushy", "fj_bushy_decompose", "fj_batch_create", "fj_batch_run", "fj_sketch_relation",
                     "fj_greedy_order", "fj_plan_candidates", "fj_candidate_plan", "fj_mlp_create",
                     "fj_mlp_set_params", "fj_mlp_get_params", "fj_mlp_forward", "fj_mlp_gradient",
                     "fj_mlp_train_step", "fj_choose_plan"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int, ok=(0,)):
    if st not in ok:
        raise FJError(st, lib().fj_last_error().decode(errors="replace"))
    return st


# ------------------------------------------------------------------ queries

def make_query(atoms: Sequence[Sequence[int]], nvars: int, head: Optional[Sequence[int]] = None) -> QueryS:
    """atoms[i] = the variable of each column of atom i."""
    q = QueryS()
    if len(atoms) > MAX_ATOMS:
        raise ValueError("too many atoms")
    q.natoms = len(atoms)
    for i, vs in enumerate(atoms):
        q.atoms[i].arity = len(vs)
        for j, v in enumerate(vs):
            q.atoms[i].vars[j] = int(v)
    q.nvars = nvars
    head = list(range(nvars)) if head is None else list(head)
    q.nhead = len(head)
    for j, v in enumerate(head):
        q.head[j] = int(v)
    return q


class Plan:
    def __init__(self, handle: int, query: QueryS):
        self.h = handle
        self.query = query

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fj_plan_free(self.h)
            self.h = None

    def nodes(self) -> List[List[Tuple[int, Tuple[int, ...]]]]:
        cap = MAX_NODES * MAX_ATOMS
        nn = C.c_int32(0)
        nsub = (C.c_int32 * MAX_NODES)()
        sa = (C.c_int32 * cap)()
        snv = (C.c_int32 * cap)()
        sv = (C.c_int32 * (cap * MAX_COLS))()
        _check(lib().fj_plan_get(self.h, C.byref(nn), nsub, sa, snv, sv, cap))
        out, idx = [], 0
        for k in range(nn.value):
            node = []
            for _ in range(nsub[k]):
                node.append((sa[idx], tuple(sv[idx * MAX_COLS + j] for j in range(snv[idx]))))
                idx += 1
            out.append(node)
        return out


def plan_from_binary(q: QueryS, order: Sequence[int], factor: bool = True) -> Plan:
    arr = (C.c_int32 * len(order))(*order)
    h = C.c_void_p()
    _check(lib().fj_plan_from_binary(C.byref(q), arr, len(order), FACTOR if factor else 0, C.byref(h)))
    return Plan(h.value, q)


def plan_from_nodes(q: QueryS, nodes: Sequence[Sequence[Tuple[int, Sequence[int]]]]) -> Plan:
    subs = [s for n in nodes for s in n]
    nsub = (C.c_int32 * max(1, len(nodes)))(*[len(n) for n in nodes])
    sa = (C.c_int32 * max(1, len(subs)))(*[a for a, _ in subs])
    snv = (C.c_int32 * max(1, len(subs)))(*[len(vs) for _, vs in subs])
    sv = (C.c_int32 * (max(1, len(subs)) * MAX_COLS))()
    for i, (_, vs) in enumerate(subs):
        for j, v in enumerate(vs):
            sv[i * MAX_COLS + j] = v
    h = C.c_void_p()
    _check(lib().fj_plan_from_nodes(C.byref(q), len(nodes), nsub, sa, snv, sv, C.byref(h)))
    return Plan(h.value, q)


# ------------------------------------------------------------------ context

class Context:
    """A libfj context bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None, tile: int = 0, block: int = 0,
                 timing=False, tail: int = 0, generic: bool = False, trie: int = 0, no_filter: bool = False):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        opt = Options()
        opt.tile = tile
        opt.block = block
        opt.timing = int(timing)   # True: every kernel class; 2: the node-0 probe only
        opt.tail = tail
        opt.generic = 1 if generic else 0
        opt.trie = int(trie)
        opt.no_filter = 1 if no_filter else 0
        h = C.c_void_p()
        _check(lib().fj_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(opt), C.byref(h)))
        self.h = h.value

    def close(self):
        if getattr(self, "h", None):
            lib().fj_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timings(self):
        ms = (C.c_double * len(TIMERS))()
        n = (C.c_uint64 * len(TIMERS))()
        _check(lib().fj_timings(self.h, ms, n))
        return {k: (ms[i], int(n[i])) for i, k in enumerate(TIMERS)}

    def timings_reset(self):
        _check(lib().fj_timings_reset(self.h))

    def set_timing(self, mode):
        """True / 1: every kernel class; 2: the node-0 probe only; 0: off."""
        _check(lib().fj_set_timing(self.h, int(mode)))

    # ---- selection
    def filter_lt(self, col, bound: int, out_sel=None):
        """Row offsets r with col[r] < bound (device uint32 tensor, unspecified order)."""
        import torch
        n = int(col.shape[0])
        if out_sel is None:
            out_sel = torch.empty(max(n, 1), dtype=torch.int32, device=col.device)
        cnt = C.c_int64(0)
        _check(lib().fj_filter_lt(self.h, C.c_void_p(col.data_ptr()), n, int(bound),
                                  C.c_void_p(out_sel.data_ptr()), C.byref(cnt)))
        return out_sel, int(cnt.value)

    def filter_lt_batch(self, specs):
        """specs: list of (col tensor, bound, out tensor).  Returns the counts."""
        args = filter_args(specs)
        self.filter_lt_prepared(args)
        return [int(args[-1][i]) for i in range(args[0])]

    def filter_lt_prepared(self, args):
        """Run selections whose arguments filter_args() marshalled once; the
        counts land in args[-1]."""
        _check(lib().fj_filter_lt_batch(self.h, *args))

    # ---- COLTs
    def build_colt(self, q: QueryS, plan: Plan, atom: int, cols, sel=None, nsel: int = 0) -> "Colt":
        rel = _relation(cols, sel, nsel)
        h = C.c_void_p()
        _check(lib().fj_build_colt(self.h, C.byref(q), plan.h, atom, C.byref(rel), C.byref(h)))
        return Colt(h.value, cols, sel)

    def rebuild_colt(self, colt: "Colt", cols, sel=None, nsel: int = 0):
        rel = _relation(cols, sel, nsel)
        _check(lib().fj_colt_rebuild(self.h, colt.h, C.byref(rel)))
        colt.keep = (cols, sel)

    def rebuild_colts(self, colts: Sequence["Colt"], specs):
        """Rebuild many COLTs in one grouped pass; specs[k] = (cols, sel, nsel)."""
        n = len(colts)
        if n == 0:
            return
        rels = (Relation * n)(*[_relation(*sp) for sp in specs])
        arr = (C.c_void_p * n)(*[c.h for c in colts])
        self.rebuild_colts_prepared(n, arr, rels)
        for c, sp in zip(colts, specs):
            c.keep = (sp[0], sp[1])

    def select_rebuild_prepared(self, nsel: int, atoms, cols, bounds, n: int, arr, rels):
        """fj_select_rebuild with every array already marshalled: the
        selections' counts land in rels[atoms[i]].nsel."""
        _check(lib().fj_select_rebuild(self.h, nsel, atoms, cols, bounds, n, arr, rels))

    def rebuild_colts_prepared(self, n: int, arr, rels):
        """As rebuild_colts, with the handle and relation arrays already
        marshalled (the caller keeps the buffers alive)."""
        _check(lib().fj_colt_rebuild_many(self.h, n, arr, rels))

    # ---- join
    def execute(self, q: QueryS, plan: Plan, colts: Sequence["Colt"], out=None, stats: bool = False):
        """Returns (count, written, Stats or None).  out: device int32 [cap, nhead] or None."""
        key = tuple(c.h for c in colts)
        if getattr(self, "_exec_key", None) != key:
            self._exec_key = key
            self._exec_arr = (C.c_void_p * len(key))(*key)
        arr = self._exec_arr
        cnt = C.c_uint64(0)
        wr = C.c_uint64(0)
        st = Stats() if stats else None
        cap = int(out.shape[0]) if out is not None else 0
        rc = lib().fj_execute(self.h, C.byref(q), plan.h, arr, C.byref(cnt),
                              C.c_void_p(out.data_ptr()) if out is not None else None, cap,
                              C.byref(wr), C.byref(st) if st is not None else None)
        _check(rc, ok=(0, 1))
        return int(cnt.value), int(wr.value), st


    def execute_factorized(self, q: QueryS, plan: Plan, colts: Sequence["Colt"]) -> "Result":
        """Run the plan but keep its final bindings instead of rows (a
        factorized result); Result.expand writes pages of rows."""
        arr = (C.c_void_p * len(colts))(*[c.h for c in colts])
        h = C.c_void_p()
        cnt = C.c_uint64(0)
        nb = C.c_uint64(0)
        _check(lib().fj_execute_factorized(self.h, C.byref(q), plan.h, arr, C.byref(h), C.byref(cnt),
                                           C.byref(nb)))
        return Result(h.value, self, int(cnt.value), int(nb.value), int(q.nhead), list(colts))

    def execute_bushy(self, q: QueryS, tree, rels, factor: bool = True, out=None):
        """Run a binary plan by its left-deep decomposition; rels: one
        (cols, sel, nsel) per atom.  Returns (count, written)."""
        b = tree if isinstance(tree, Bushy) else bushy(tree)
        ra = (Relation * len(rels))(*[_relation(c, s, n) for c, s, n in rels])
        cnt = C.c_uint64(0)
        wr = C.c_uint64(0)
        cap = int(out.shape[0]) if out is not None else 0
        rc = lib().fj_execute_bushy(self.h, C.byref(q), C.byref(b), ra, FACTOR if factor else 0, C.byref(cnt),
                                    C.c_void_p(out.data_ptr()) if out is not None else None, cap, C.byref(wr))
        _check(rc, ok=(0, 1))
        return int(cnt.value), int(wr.value)

    # ---- statistics and plan choice
    def sketch(self, cols, sel=None, nsel: int = 0) -> Sketch:
        """Exact distinct counts and top frequencies of each column (GPU)."""
        rel = _relation(cols, sel, nsel)
        sk = Sketch()
        _check(lib().fj_sketch_relation(self.h, C.byref(rel), C.byref(sk)))
        return sk

    def choose_plan(self, q: QueryS, sketches: Sequence[Sketch], mlp: Optional["Mlp"], margin: float = 0.0,
                    gate_rows: int = 0):
        """Returns (Plan, chosen candidate index, scores or None)."""
        arr = _sketch_array(sketches)
        h = C.c_void_p()
        chosen = C.c_int32(0)
        scores = (C.c_float * CAND_MAX)()
        _check(lib().fj_choose_plan(self.h, mlp.h if mlp is not None else None, C.byref(q), arr,
                                    float(margin), int(gate_rows), C.byref(h), C.byref(chosen), scores))
        return Plan(h.value, q), int(chosen.value), [float(x) for x in scores]


def _sketch_array(sketches: Sequence[Sketch]):
    return (Sketch * len(sketches))(*sketches)


def greedy_order(q: QueryS, sketches: Sequence[Sketch], first: int = -1) -> List[int]:
    order = (C.c_int32 * MAX_ATOMS)()
    _check(lib().fj_greedy_order(C.byref(q), _sketch_array(sketches), int(first), order))
    return [int(order[i]) for i in range(q.natoms)]


def plan_candidates(q: QueryS, sketches: Sequence[Sketch], cap: int = CAND_MAX):
    """Returns (list of Candidate, numpy float32 features [n, FEATURES])."""
    import numpy as np
    cands = (Candidate * CAND_MAX)()
    n = C.c_int32(0)
    feat = np.zeros((CAND_MAX, FEATURES), dtype=np.float32)
    _check(lib().fj_plan_candidates(C.byref(q), _sketch_array(sketches), int(cap), cands, C.byref(n),
                                    C.c_void_p(feat.ctypes.data)))
    k = int(n.value)
    out = []
    for i in range(k):
        c = Candidate()
        C.pointer(c)[0] = cands[i]
        out.append(c)
    return out, feat[:k].copy()


def candidate_plan(q: QueryS, cand: Candidate) -> Plan:
    h = C.c_void_p()
    _check(lib().fj_candidate_plan(C.byref(q), C.byref(cand), C.byref(h)))
    return Plan(h.value, q)


class Mlp:
    """The chooser's perceptron (in_dim -> hidden -> hidden -> 1, FP32), trained
    and evaluated by libfj's kernels.  Inputs and targets are device float32
    tensors on the context's device."""

    def __init__(self, ctx: Context, in_dim: int = FEATURES, hidden: int = 128):
        h = C.c_void_p()
        _check(lib().fj_mlp_create(ctx.h, int(in_dim), int(hidden), C.byref(h)))
        self.h = h.value
        self.ctx = ctx
        self.in_dim = in_dim
        self.hidden = hidden
        self.n = int(lib().fj_mlp_param_count(self.h))

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != self.n:
            raise ValueError(f"expected {self.n} parameters, got {p.size}")
        _check(lib().fj_mlp_set_params(self.h, C.c_void_p(p.ctypes.data), self.n))

    def get_params(self):
        import numpy as np
        p = np.empty(self.n, dtype=np.float32)
        _check(lib().fj_mlp_get_params(self.h, C.c_void_p(p.ctypes.data), self.n))
        return p

    def forward(self, x, y=None):
        import torch
        b = int(x.shape[0])
        if y is None:
            y = torch.empty(b, dtype=torch.float32, device=x.device)
        _check(lib().fj_mlp_forward(self.h, C.c_void_p(x.data_ptr()), b, C.c_void_p(y.data_ptr())))
        return y

    def gradient(self, x, t):
        import numpy as np
        g = np.empty(self.n, dtype=np.float32)
        loss = C.c_float(0)
        _check(lib().fj_mlp_gradient(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), int(x.shape[0]),
                                     C.c_void_p(g.ctypes.data), C.byref(loss)))
        return g, float(loss.value)

    def train_step(self, x, t, lr: float, want_loss: bool = False):
        loss = C.c_float(0)
        _check(lib().fj_mlp_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                       int(x.shape[0]), float(lr), C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def free(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fj_mlp_free(self.h)
            self.h = None

    def __del__(self):
        self.free()


class BatchOptions(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("block", C.c_int32), ("no_graph", C.c_int32),
                ("no_rebuild", C.c_int32), ("reserved", C.c_int32 * 3), ("query_chunk", C.c_void_p)]


class Batch:
    """Many queries counted by one persistent launch (captured in a hipGraph)."""

    def __init__(self, ctx: "Context", items, chunk: int = 0, block: int = 0, graph: bool = True,
                 rebuild: bool = True, query_chunk=None):
        """items: list of (QueryS, Plan, [Colt per atom])."""
        n = len(items)
        self.ctx = ctx
        self.keep = items
        qs = (C.c_void_p * n)(*[C.addressof(q) for q, _, _ in items])
        ps = (C.c_void_p * n)(*[p.h for _, p, _ in items])
        self._colt_arrays = [(C.c_void_p * len(cs))(*[c.h for c in cs]) for _, _, cs in items]
        cs = (C.c_void_p * n)(*[C.addressof(a) for a in self._colt_arrays])
        opt = BatchOptions()
        opt.chunk = chunk
        opt.block = block
        opt.no_graph = 0 if graph else 1
        opt.no_rebuild = 0 if rebuild else 1
        if query_chunk is not None:
            self._qc = (C.c_int32 * n)(*[int(x) for x in query_chunk])
            opt.query_chunk = C.addressof(self._qc)
        h = C.c_void_p()
        _check(lib().fj_batch_create(ctx.h, n, qs, ps, cs, C.byref(opt), C.byref(h)))
        self.h = h.value
        self.n = n

    def run(self):
        counts = (C.c_uint64 * self.n)()
        _check(lib().fj_batch_run(self.h, counts))
        return [int(x) for x in counts]

    def free(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fj_batch_free(self.h)
            self.h = None

    def __del__(self):
        self.free()


class Result:
    """A factorized result: count rows held as `bindings` final bindings.
    It keeps its COLTs (and through them the relations) alive; they must not
    be rebuilt while the result is in use."""

    def __init__(self, handle: int, ctx: "Context", count: int, bindings: int, nhead: int, colts):
        self.h = handle
        self.ctx = ctx
        self.count = count
        self.bindings = bindings
        self.nhead = nhead
        self.keep = colts

    def expand(self, first: int, out) -> int:
        """Rows [first, first + len(out)) into out (device int32 [cap, nhead]);
        returns how many were written."""
        wr = C.c_uint64(0)
        cap = int(out.shape[0])
        _check(lib().fj_result_expand(self.ctx.h, self.h, int(first),
                                      C.c_void_p(out.data_ptr()) if cap else None, cap, C.byref(wr)))
        return int(wr.value)

    def free(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fj_result_free(self.h)
            self.h = None

    def __del__(self):
        self.free()


class Colt:
    def __init__(self, handle: int, cols, sel):
        self.h = handle
        self.keep = (cols, sel)  # the library borrows these buffers

    def free(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fj_colt_free(self.h)
            self.h = None

    def __del__(self):
        self.free()


def filter_args(specs):
    """fj_filter_lt_batch's arguments for specs = [(col, bound, out)], the
    counts array last."""
    n = len(specs)
    cols = (C.c_void_p * max(n, 1))(*[c.data_ptr() for c, _, _ in specs])
    nrows = (C.c_int64 * max(n, 1))(*[int(c.shape[0]) for c, _, _ in specs])
    bounds = (C.c_int32 * max(n, 1))(*[int(b) for _, b, _ in specs])
    outs = (C.c_void_p * max(n, 1))(*[o.data_ptr() for _, _, o in specs])
    counts = (C.c_int64 * max(n, 1))()
    return (n, cols, nrows, bounds, outs, counts)


def _relation(cols, sel, nsel) -> Relation:
    r = Relation()
    r.ncols = len(cols)
    r.nrows = int(cols[0].shape[0]) if cols else 0
    for j, c in enumerate(cols):
        r.cols[j] = c.data_ptr()
    r.sel = sel.data_ptr() if sel is not None else None
    r.nsel = int(nsel) if sel is not None else 0
    return r
