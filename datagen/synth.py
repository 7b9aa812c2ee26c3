"""Seeded relation generators shaped like the Free Join paper's workloads.

Every generator takes an explicit seed and draws from numpy's PCG64.  The
outputs are plain int32 columns; a query is described by atoms that name a
relation and give one variable per column (all variables of an atom are
distinct, as the paper's query model of Section 2.1 requires), plus optional
pushed-down selections of the form ``column < constant`` (Section 2.1: the
atom may be a selection over a base table).

Nothing here evaluates a join.  The one exception to "no arithmetic over two
relations" is the size bound of ``batch_mix`` (``_two_path_bound`` times
``_max_dup``), a degree product used only to reject oversized random triangle
instances; it is a workload filter and never an expected value.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 0xF7EE0000


def seed_for(config: int, rep: int = 0) -> int:
    """Seed of repetition ``rep`` of workload ``config``."""
    return SEED_BASE + config * 0x100 + rep


@dataclasses.dataclass
class Relation:
    name: str
    cols: List[np.ndarray]  # int32, equal lengths

    @property
    def nrows(self) -> int:
        return int(self.cols[0].shape[0]) if self.cols else 0

    @property
    def arity(self) -> int:
        return len(self.cols)


@dataclasses.dataclass
class Query:
    """A full conjunctive query over bag relations.

    ``atoms[i] = (relation index, var ids, one per relation column)``.
    ``filters[i]`` is ``None`` or ``(column, c)`` meaning the atom ranges over
    ``sigma_{col < c}`` of its relation.  ``head`` lists every variable once,
    in output-column order.
    """

    var_names: List[str]
    relations: List[Relation]
    atoms: List[Tuple[int, Tuple[int, ...]]]
    filters: List[Optional[Tuple[int, int]]]
    head: List[int]
    kind: str = ""

    @property
    def nvars(self) -> int:
        return len(self.var_names)

    def atom_cols(self, i: int) -> List[np.ndarray]:
        return self.relations[self.atoms[i][0]].cols

    def atom_rows(self, i: int) -> int:
        return self.relations[self.atoms[i][0]].nrows


def make_query(var_names, relations, atoms, filters=None, head=None, kind=""):
    names = list(var_names)
    atoms = [(int(r), tuple(int(v) for v in vs)) for r, vs in atoms]
    for r, vs in atoms:
        if len(vs) != relations[r].arity:
            raise ValueError("atom arity does not match its relation")
        if len(set(vs)) != len(vs):
            raise ValueError("variables of one atom must be distinct")
    if filters is None:
        filters = [None] * len(atoms)
    if head is None:
        head = list(range(len(names)))
    return Query(names, list(relations), atoms, list(filters), list(head), kind)


# --------------------------------------------------------------------------
# small fixtures
# --------------------------------------------------------------------------

def clover_instance(n: int) -> Query:
    """The clover query and the adversarial instance of the paper's Section 3
    figure: R, S, T share x; x0 is the only value common to all three, x1 is
    in R and T (n tuples each), x2 in R and S, x3 in S and T.

    Values are encoded as int32: x_j -> j; a_0 = b_0 = c_0 = 0; the left
    family a^l_i / b^l_i / c^l_i -> i; the right family -> 1000 + i.
    """
    if n < 1:
        raise ValueError("n >= 1")
    def rel(name, pairs):
        a = np.array(pairs, dtype=np.int32).reshape(-1, 2)
        return Relation(name, [a[:, 0].copy(), a[:, 1].copy()])
    r = [(0, 0)] + [(1, i) for i in range(1, n + 1)] + [(2, 1000 + i) for i in range(1, n + 1)]
    s = [(0, 0)] + [(2, i) for i in range(1, n + 1)] + [(3, 1000 + i) for i in range(1, n + 1)]
    t = [(0, 0)] + [(3, i) for i in range(1, n + 1)] + [(1, 1000 + i) for i in range(1, n + 1)]
    rels = [rel("R", r), rel("S", s), rel("T", t)]
    # variables: x=0, a=1, b=2, c=3
    return make_query(["x", "a", "b", "c"], rels,
                      [(0, (0, 1)), (1, (0, 2)), (2, (0, 3))], kind="clover")


def clover_u_instance(n: int, u_values) -> Query:
    """The clover instance extended with a unary relation U(b), as in the
    paper's Section 4.2 COLT example: Q(x,a,b,c) :- R(x,a), S(x,b), T(x,c),
    U(b).  R, S, T are ``clover_instance(n)``'s; U holds ``u_values`` (int32,
    duplicates kept).  Variables: x=0, a=1, b=2, c=3; atoms R, S, T, U."""
    base = clover_instance(n)
    u = Relation("U", [np.asarray(list(u_values), dtype=np.int32).reshape(-1)])
    rels = list(base.relations) + [u]
    return make_query(["x", "a", "b", "c"], rels,
                      [(0, (0, 1)), (1, (0, 2)), (2, (0, 3)), (3, (2,))], kind="clover_u")


def triangle_query(edges: Tuple[np.ndarray, np.ndarray], kind="triangle") -> Query:
    """Q(x,y,z) :- E(x,y), E(y,z), E(z,x): three atoms over one edge buffer."""
    e = Relation("E", [edges[0], edges[1]])
    return make_query(["x", "y", "z"], [e],
                      [(0, (0, 1)), (0, (1, 2)), (0, (2, 0))], kind=kind)


def four_cycle_query(edges: Tuple[np.ndarray, np.ndarray]) -> Query:
    """Q(w,x,y,z) :- E(w,x), E(x,y), E(y,z), E(z,w)."""
    e = Relation("E", [edges[0], edges[1]])
    return make_query(["w", "x", "y", "z"], [e],
                      [(0, (0, 1)), (0, (1, 2)), (0, (2, 3)), (0, (3, 0))], kind="4cycle")


# --------------------------------------------------------------------------
# distributions
# --------------------------------------------------------------------------

def _dedupe_first(keys: np.ndarray) -> np.ndarray:
    """Indices of the first occurrence of each distinct key, in draw order."""
    _, first = np.unique(keys, return_index=True)
    first.sort()
    return first


def zipf_keys(rng: np.random.Generator, n: int, domain: int, s: float,
              perm: Optional[np.ndarray] = None) -> np.ndarray:
    """n draws of a bounded Zipf(s) over ranks 1..domain by inverse CDF,
    mapped to keys 0..domain-1 through ``perm`` (rank r -> perm[r-1]).
    s = 0 is the uniform distribution."""
    if domain <= 0:
        raise ValueError("domain must be positive")
    if s == 0.0:
        ranks = rng.integers(0, domain, size=n, dtype=np.int64)
    else:
        w = np.arange(1, domain + 1, dtype=np.float64) ** (-float(s))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        u = rng.random(n)
        ranks = np.searchsorted(cdf, u, side="right")
        np.minimum(ranks, domain - 1, out=ranks)
    if perm is None:
        return ranks.astype(np.int32)
    return perm[ranks].astype(np.int32)


def triangle_edges(seed: int, n_edges: int = 10_000, n_vertices: int = 2_000):
    """Uniform directed edges over [0, n_vertices)^2 with self-loops and
    duplicates rejected until exactly ``n_edges`` distinct edges remain."""
    if n_edges > n_vertices * (n_vertices - 1):
        raise ValueError("more edges requested than exist")
    rng = np.random.Generator(np.random.PCG64(seed))
    src = np.empty(0, np.int64)
    dst = np.empty(0, np.int64)
    while True:
        need = n_edges - src.shape[0]
        k = max(1024, int(need * 1.3) + 16)
        u = rng.integers(0, n_vertices, size=k, dtype=np.int64)
        v = rng.integers(0, n_vertices, size=k, dtype=np.int64)
        keep = u != v
        src = np.concatenate([src, u[keep]])
        dst = np.concatenate([dst, v[keep]])
        first = _dedupe_first(src * n_vertices + dst)
        src, dst = src[first], dst[first]
        if src.shape[0] >= n_edges:
            return src[:n_edges].astype(np.int32), dst[:n_edges].astype(np.int32)


def rmat_edges(seed: int, scale: int, n_edges: int,
               abcd=(0.57, 0.19, 0.19, 0.05), chunk: int = 1 << 22):
    """R-MAT power-law edges over 2^scale vertices: per edge and level a
    quadrant is drawn with probabilities (a, b, c, d); vertex labels are then
    permuted by a seeded permutation; self-loops are dropped and the first
    ``n_edges`` distinct edges in draw order are kept."""
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("quadrant probabilities must sum to 1")
    nv = 1 << scale
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(nv).astype(np.int64)
    t1, t2, t3 = a, a + b, a + b + c
    src_all, dst_all = [], []
    have = 0
    seen_keys = np.empty(0, np.int64)
    while have < n_edges:
        k = chunk
        u = np.zeros(k, np.int64)
        v = np.zeros(k, np.int64)
        for _ in range(scale):
            r = rng.random(k)
            ub = (r >= t2).astype(np.int64)              # quadrants c, d: src bit
            vb = (((r >= t1) & (r < t2)) | (r >= t3)).astype(np.int64)  # b, d: dst bit
            u = (u << 1) | ub
            v = (v << 1) | vb
        u = perm[u]
        v = perm[v]
        keep = u != v
        keys = u[keep] * nv + v[keep]
        first = _dedupe_first(keys)
        keys = keys[first]
        # drop keys seen in earlier chunks, keep draw order
        if seen_keys.size:
            fresh = ~np.isin(keys, seen_keys, assume_unique=False)
            keys = keys[fresh]
        keys = keys[: n_edges - have]
        seen_keys = np.union1d(seen_keys, keys) if have + keys.size < n_edges else seen_keys
        src_all.append((keys // nv).astype(np.int32))
        dst_all.append((keys % nv).astype(np.int32))
        have += keys.size
    return np.concatenate(src_all), np.concatenate(dst_all)


def star_schema(seed: int, n_fact: int = 10_000_000, n_dim: int = 1_000_000,
                n_fk: int = 4, s: float = 1.1, attr_range: int = 100,
                attr_lt: int = 10, filter_dims: Sequence[int] = None) -> Query:
    """Star join: fact F(k1..kd) with Zipf(s) foreign keys (one independent
    rank->key permutation per dimension), dimensions D_i(k_i, a_i) with
    primary key 0..n_dim-1 and attribute uniform over [0, attr_range), and a
    pushed-down selection a_i < attr_lt on the dimensions in ``filter_dims``
    (all of them by default).

    Query: Q(k1..kd, a1..ad) :- F(k1..kd), D1(k1,a1), ..., Dd(kd,ad)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fcols = []
    for _ in range(n_fk):
        perm = rng.permutation(n_dim).astype(np.int64)
        fcols.append(zipf_keys(rng, n_fact, n_dim, s, perm))
    rels = [Relation("F", fcols)]
    for i in range(n_fk):
        pk = np.arange(n_dim, dtype=np.int32)
        attr = rng.integers(0, attr_range, size=n_dim, dtype=np.int64).astype(np.int32)
        rels.append(Relation(f"D{i+1}", [pk, attr]))
    names = [f"k{i+1}" for i in range(n_fk)] + [f"a{i+1}" for i in range(n_fk)]
    atoms = [(0, tuple(range(n_fk)))]
    for i in range(n_fk):
        atoms.append((i + 1, (i, n_fk + i)))
    if filter_dims is None:
        filter_dims = range(n_fk)
    filters = [None] + [((1, attr_lt) if i in set(filter_dims) else None) for i in range(n_fk)]
    return make_query(names, rels, atoms, filters, kind="star")


# --------------------------------------------------------------------------
# tiny random instances (brute-force checks) and the batched mix
# --------------------------------------------------------------------------

_SHAPES = ("triangle", "clover", "chain3", "chain4", "star3", "cycle4", "clover_u", "pair", "single")


def fanout_chain(seed: int, n_left: int = 1_000_000, n_keys: int = 100_000, fanout: int = 20) -> Query:
    """R(x, y) join S(y, z): R has n_left rows with y uniform over n_keys; S
    holds `fanout` rows for every key y (z uniform), so each R row meets
    `fanout` S rows.  The result has n_left * fanout rows but only n_left
    bindings before the last variable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.integers(0, 1 << 30, n_left, dtype=np.int32)
    y = rng.integers(0, n_keys, n_left, dtype=np.int32)
    sy = np.repeat(np.arange(n_keys, dtype=np.int32), fanout)
    sy = sy[rng.permutation(sy.shape[0])]
    z = rng.integers(-(1 << 30), 1 << 30, sy.shape[0], dtype=np.int32)
    return make_query(["x", "y", "z"], [Relation("R", [x, y]), Relation("S", [sy, z])],
                      [(0, (0, 1)), (1, (1, 2))], kind="fanout_chain")


def random_tiny_query(seed: int, shape: str, max_rows: int = 10, domain: int = 4) -> Query:
    """Small bag instances over a tiny domain so that duplicates, skew and
    hash collisions all occur; used against nested-loop enumeration."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def rel(name, arity):
        n = int(rng.integers(0, max_rows + 1))
        return Relation(name, [rng.integers(0, domain, size=n).astype(np.int32) for _ in range(arity)])

    if shape == "triangle":
        rels = [rel("R", 2), rel("S", 2), rel("T", 2)]
        return make_query(["x", "y", "z"], rels, [(0, (0, 1)), (1, (1, 2)), (2, (2, 0))], kind=shape)
    if shape == "clover":
        rels = [rel("R", 2), rel("S", 2), rel("T", 2)]
        return make_query(["x", "a", "b", "c"], rels, [(0, (0, 1)), (1, (0, 2)), (2, (0, 3))], kind=shape)
    if shape == "clover_u":
        rels = [rel("R", 2), rel("S", 2), rel("T", 2), rel("U", 1)]
        return make_query(["x", "a", "b", "c"], rels,
                          [(0, (0, 1)), (1, (0, 2)), (2, (0, 3)), (3, (2,))], kind=shape)
    if shape == "chain3":
        rels = [rel("R", 2), rel("S", 2), rel("T", 2)]
        return make_query(["x", "y", "z", "u"], rels, [(0, (0, 1)), (1, (1, 2)), (2, (2, 3))], kind=shape)
    if shape == "chain4":
        rels = [rel("R", 2), rel("S", 2), rel("T", 2), rel("W", 2)]
        return make_query(["x", "y", "z", "u", "v"], rels,
                          [(0, (0, 1)), (1, (1, 2)), (2, (2, 3)), (3, (3, 4))], kind=shape)
    if shape == "star3":
        rels = [rel("F", 3), rel("A", 2), rel("B", 2), rel("C", 2)]
        return make_query(["k1", "k2", "k3", "a", "b", "c"], rels,
                          [(0, (0, 1, 2)), (1, (0, 3)), (2, (1, 4)), (3, (2, 5))], kind=shape)
    if shape == "cycle4":
        rels = [rel("R", 2), rel("S", 2), rel("T", 2), rel("W", 2)]
        return make_query(["w", "x", "y", "z"], rels,
                          [(0, (0, 1)), (1, (1, 2)), (2, (2, 3)), (3, (3, 0))], kind=shape)
    if shape == "pair":
        rels = [rel("R", 2), rel("S", 3)]
        return make_query(["x", "y", "z"], rels, [(0, (0, 1)), (1, (0, 1, 2))], kind=shape)
    if shape == "single":
        rels = [rel("R", 2)]
        return make_query(["x", "y"], rels, [(0, (0, 1))], kind=shape)
    raise ValueError(f"unknown shape {shape}")


def _two_path_bound(a_dst: np.ndarray, b_src: np.ndarray, domain: int) -> int:
    """sum_v deg_a(v) * deg_b(v): the number of joined row pairs (the 2-path
    relation of two bag relations)."""
    da = np.bincount(a_dst, minlength=domain).astype(np.int64)
    db = np.bincount(b_src, minlength=domain).astype(np.int64)
    return int(np.dot(da, db))


def _max_dup(c0: np.ndarray, c1: np.ndarray, domain: int) -> int:
    """Largest number of identical rows (c0, c1) of a bag relation."""
    if c0.size == 0:
        return 0
    _, counts = np.unique(c0.astype(np.int64) * domain + c1.astype(np.int64), return_counts=True)
    return int(counts.max())


def _pk_sample(rng, n: int, domain: int) -> np.ndarray:
    return rng.choice(domain, size=n, replace=False).astype(np.int32)


def batch_mix(seed: int, n_queries: int = 256, min_rows: int = 1_000,
              max_rows: int = 2_000_000, max_bound: int = 1 << 26,
              frac_chain: float = 0.3, frac_star: float = 0.3):
    """The batched workload: 30% chains, 30% stars (3 to 6 relations), 40%
    triangles; rows per relation log-uniform in [min_rows, max_rows]; a
    per-query Zipf exponent s ~ U[0, 1.5].  Query i is ``batch_query(seed,
    i, ...)``.

    Returns (queries, redraws)."""
    out = []
    redraws = 0
    for qi in range(n_queries):
        q, r = batch_query(seed, qi, min_rows, max_rows, max_bound, frac_chain, frac_star)
        out.append(q)
        redraws += r
    return out, redraws


def batch_query(seed: int, qi: int, min_rows: int = 1_000, max_rows: int = 2_000_000,
                max_bound: int = 1 << 26, frac_chain: float = 0.3, frac_star: float = 0.3):
    """Query qi of the batched workload, drawn from its own seeded stream.

    Acyclic queries are primary-key/foreign-key joins: the referenced column
    holds distinct keys sampled from a domain of twice the referenced
    relation's size (so about half of the foreign keys find no partner), and
    the referencing column is Zipf(s) over the same domain through the rank
    permutation shared with the referenced side.  Triangles use three
    distinct bag relations with Zipf(s) endpoints over D = ceil(rows^(2/3));
    a triangle whose result-size upper bound (joined pairs of two relations
    times the largest row multiplicity of the third) exceeds ``max_bound`` is
    redrawn.

    Returns (query, redraws)."""
    redraws = 0
    rng = np.random.Generator(np.random.PCG64(seed * 1_000_003 + qi))
    u = rng.random()
    s = float(rng.uniform(0.0, 1.5))
    lr = lambda: int(round(math.exp(rng.uniform(math.log(min_rows), math.log(max_rows)))))
    if u < frac_chain:
        m = int(rng.integers(3, 7))
        rows = [lr() for _ in range(m)]
        # R_i(x_i, x_{i+1}); for i >= 1 the column x_i of R_i is a key
        # (distinct values from a domain of 2 * rows[i]) and the column
        # x_i of R_{i-1} references it with Zipf(s) skew.
        doms = [0] + [2 * rows[i] for i in range(1, m)]
        perms = [None] + [rng.permutation(doms[i]).astype(np.int64) for i in range(1, m)]
        rels = []
        for i in range(m):
            n = rows[i]
            if i == 0:
                first = rng.integers(0, max(2, n), size=n).astype(np.int32)
            else:
                first = rng.choice(doms[i], size=n, replace=False).astype(np.int32)
            if i == m - 1:
                last = rng.integers(0, max(2, n), size=n).astype(np.int32)
            else:
                last = zipf_keys(rng, n, doms[i + 1], s, perms[i + 1])
            rels.append(Relation(f"R{i}", [first, last]))
        names = [f"x{i}" for i in range(m + 1)]
        atoms = [(i, (i, i + 1)) for i in range(m)]
        return make_query(names, rels, atoms, kind=f"chain{m}"), redraws
    elif u < frac_chain + frac_star:
        m = int(rng.integers(3, 7))
        d = m - 1
        nf = lr()
        rels = [None]
        fcols = []
        for i in range(d):
            nd = lr()
            dom = 2 * nd
            perm = rng.permutation(dom).astype(np.int64)
            pk = perm[rng.choice(dom, size=nd, replace=False)].astype(np.int32)
            attr = rng.integers(0, 100, size=nd).astype(np.int32)
            rels.append(Relation(f"D{i}", [pk, attr]))
            fcols.append(zipf_keys(rng, nf, dom, s, perm))
        rels[0] = Relation("F", fcols)
        names = [f"k{i}" for i in range(d)] + [f"a{i}" for i in range(d)]
        atoms = [(0, tuple(range(d)))] + [(i + 1, (i, d + i)) for i in range(d)]
        return make_query(names, rels, atoms, kind=f"star{m}"), redraws
    else:
        while True:
            rows = [lr() for _ in range(3)]
            dom = int(math.ceil(max(rows) ** (2.0 / 3.0)))
            perm = rng.permutation(dom).astype(np.int64)
            cols = []
            for n in rows:
                cols.append((zipf_keys(rng, n, dom, s, perm), zipf_keys(rng, n, dom, s, perm)))
            (rx, ry), (sy, sz), (tz, tx) = cols
            # every joined pair of two relations extends through at most
            # the largest multiplicity of a row of the third
            b = min(_two_path_bound(ry, sy, dom) * _max_dup(tz, tx, dom),
                    _two_path_bound(sz, tz, dom) * _max_dup(rx, ry, dom),
                    _two_path_bound(tx, rx, dom) * _max_dup(sy, sz, dom))
            if b <= max_bound:
                break
            redraws += 1
            s = float(rng.uniform(0.0, 1.5))
        rels = [Relation("R", [rx, ry]), Relation("S", [sy, sz]), Relation("T", [tz, tx])]
        return make_query(["x", "y", "z"], rels, [(0, (0, 1)), (1, (1, 2)), (2, (2, 0))],
                          kind="triangle"), redraws
