"""Pins of the oracle's join results: nested-loop enumeration, closed forms,
the paper's clover instance and probe counts derived by hand from it."""

import itertools

import numpy as np
import pytest

import datagen
from oracle import brute, cfj, closed
from oracle import plans as P


def all_plans(q, max_orders=None):
    """Converted and factored plans of every left-deep order, plus the
    Generic Join plans of every variable order."""
    out = []
    orders = list(itertools.permutations(range(len(q.atoms))))
    if max_orders:
        orders = orders[:max_orders]
    for order in orders:
        b = P.binary2fj(q, order)
        out.append(b)
        f = P.factor(b)
        if f != b:
            out.append(f)
    for vo in itertools.permutations(range(q.nvars)):
        out.append(P.gj_plan(q, vo))
        if len(out) > 60:
            break
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_clover_instance_single_output(n):
    # Section 3 clover instance: the only result is (x0, a0, b0, c0)
    q = datagen.clover_instance(n)
    for plan in all_plans(q):
        r = cfj.run(q, plan, batch=3)
        assert r["count"] == 1
        assert r["rows"].tolist() == [[0, 0, 0, 0]]


@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_clover_probe_counts(n):
    # Section 4.1: the naive plan probes T once per (x2, a_i, b_j): n^2 + 1
    # lookups; after factoring T is probed once per R-tuple that hits S: n + 1.
    q = datagen.clover_instance(n)
    naive = P.binary2fj(q, [0, 1, 2])
    r = cfj.run(q, naive, batch=4)
    c = r["counters"]
    assert c[0]["probe"] == 2 * n + 1          # S probed by every R tuple
    assert c[1]["probe"] == n * n + 1          # T probed inside the loop over S[x]
    fac = P.factor(naive)
    r2 = cfj.run(q, fac, batch=4)
    c2 = r2["counters"]
    assert c2[0]["probe"] == (2 * n + 1) + (n + 1)
    assert c2[1]["probe"] == 0 and c2[2]["probe"] == 0


SHAPES = ["triangle", "clover", "chain3", "chain4", "star3", "cycle4", "clover_u", "pair", "single"]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_enumeration(shape, seed):
    q = datagen.random_tiny_query(seed * 31 + 7, shape, max_rows=9, domain=3)
    expect = brute.enumerate_result(q)
    plans = all_plans(q, max_orders=24)
    for i, plan in enumerate(plans):
        batch = (1, 2, 3, 1000)[i % 4]
        r = cfj.run(q, plan, batch=batch)
        assert r["count"] == len(expect), P.plan_str(q, plan)
        assert [tuple(x) for x in r["rows"].tolist()] == expect


def test_oracle_with_selection_matches_enumeration():
    q = datagen.star_schema(11, n_fact=40, n_dim=12, n_fk=3, attr_range=10, attr_lt=6)
    expect = brute.enumerate_result(q)
    plan = P.factor(P.binary2fj(q, [0, 1, 2, 3]))
    r = cfj.run(q, plan, batch=5)
    assert [tuple(x) for x in r["rows"].tolist()] == expect


# ---- closed forms: pinned against enumeration first, then used at scale

@pytest.mark.parametrize("seed", range(5))
def test_closed_forms_match_enumeration(seed):
    t = datagen.random_tiny_query(seed, "triangle", max_rows=12, domain=4)
    (r, s, u) = [tuple(t.relations[i].cols) for i in range(3)]
    assert closed.triangle_count(r, s, u) == brute.count(t)
    c = datagen.random_tiny_query(seed, "chain4", max_rows=10, domain=4)
    assert closed.chain_count([tuple(rel.cols) for rel in c.relations]) == brute.count(c)
    e = datagen.triangle_edges(seed, n_edges=14, n_vertices=5)
    assert closed.cycle_count(e[0], e[1], 3) == brute.count(datagen.synth.triangle_query(e))
    assert closed.cycle_count(e[0], e[1], 4) == brute.count(datagen.synth.four_cycle_query(e))
    st = datagen.star_schema(seed, n_fact=25, n_dim=8, n_fk=2, attr_range=4, attr_lt=2)
    dims = [tuple(st.relations[i + 1].cols) for i in range(2)]
    assert closed.star_count(st.relations[0].cols, dims, [2, 2]) == brute.count(st)
    rows = closed.star_rows(st.relations[0].cols, dims, [2, 2])
    assert [tuple(x) for x in rows.tolist()] == brute.enumerate_result(st)


def test_triangle_full_size_small_graph():
    # 10,000 distinct edges over 2,000 vertices: count = trace(A^3)
    for rep in range(2):
        e = datagen.triangle_edges(datagen.seed_for(1, rep))
        q = datagen.synth.triangle_query(e)
        want = closed.cycle_count(e[0], e[1], 3)
        for plan in (P.factor(P.binary2fj(q, [0, 1, 2])), P.gj_plan(q, [0, 1, 2])):
            assert cfj.run(q, plan, materialize=False)["count"] == want


def test_gj_triangle_node2_probe_count():
    # dynamic cover (Section 4.4) on [[R(x),T(x)],[R(y),S(y)],[S(z),T(z)]]:
    # node 2 iterates the smaller of S[y] (out-degree of y) and T[x]
    # (in-degree of x), ties to S, and probes the other once per element.
    e = datagen.triangle_edges(5, n_edges=3000, n_vertices=300)
    q = datagen.synth.triangle_query(e)
    src, dst = e[0].astype(np.int64), e[1].astype(np.int64)
    outdeg = np.bincount(src, minlength=300)
    indeg = np.bincount(dst, minlength=300)
    x, y = src, dst
    live = (indeg[x] > 0) & (outdeg[y] > 0)
    want = int(np.minimum(outdeg[y[live]], indeg[x[live]]).sum())
    r = cfj.run(q, P.gj_plan(q, [0, 1, 2]), materialize=False)
    assert r["counters"][2]["probe"] == want
    assert r["count"] == closed.cycle_count(e[0], e[1], 3)


def test_star_and_chain_closed_forms_medium():
    st = datagen.star_schema(2, n_fact=200_000, n_dim=20_000)
    plan = P.factor(P.binary2fj(st, [0, 1, 2, 3, 4]))
    r = cfj.run(st, plan, batch=1000)
    dims = [tuple(st.relations[i + 1].cols) for i in range(4)]
    rows = closed.star_rows(st.relations[0].cols, dims, [10] * 4)
    assert r["count"] == rows.shape[0] == closed.star_count(st.relations[0].cols, dims, [10] * 4)
    assert np.array_equal(r["rows"], rows)
    qs, _ = datagen.batch_mix(3, n_queries=8, max_rows=20_000)
    for q in qs:
        if q.kind.startswith("chain"):
            want = closed.chain_count([tuple(rel.cols) for rel in q.relations])
            got = cfj.run(q, P.factor(P.binary2fj(q, list(range(len(q.atoms))))), materialize=False)
            assert got["count"] == want


def test_plan_invariance_rmat_small():
    e = datagen.rmat_edges(9, scale=10, n_edges=6000)
    q4 = datagen.synth.four_cycle_query(e)
    want = closed.cycle_count(e[0], e[1], 4)
    for plan in (P.factor(P.binary2fj(q4, [0, 1, 2, 3])), P.gj_plan(q4, [0, 1, 2, 3]),
                 P.gj_plan(q4, [1, 3, 0, 2])):
        assert cfj.run(q4, plan, materialize=False)["count"] == want


def test_fanout_chain_counts_and_rows():
    # R(x, y) join S(y, z) where S holds exactly `fanout` rows per key: the
    # count is |R| * fanout for every plan, and the rows are each R row
    # paired with its key's S rows (written out here by a dictionary join)
    q = datagen.fanout_chain(datagen.seed_for(9, 7), n_left=400, n_keys=30, fanout=7)
    rx, ry = q.relations[0].cols
    sy, sz = q.relations[1].cols
    assert np.bincount(sy, minlength=30).tolist() == [7] * 30
    by_key = {}
    for y, z in zip(sy.tolist(), sz.tolist()):
        by_key.setdefault(y, []).append(z)
    want = np.array(sorted((x, y, z) for x, y in zip(rx.tolist(), ry.tolist()) for z in by_key[y]),
                    np.int32)
    for plan in all_plans(q):
        r = cfj.run(q, plan, batch=97)
        assert r["count"] == 400 * 7
        assert np.array_equal(r["rows"], want)
