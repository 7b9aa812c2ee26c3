"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, the
closed forms and the paper's worked examples.  Counts and sorted tuples must
match bit for bit."""

import itertools
import sys

import numpy as np
import pytest

import datagen
from oracle import closed
from tests.gpu_util import assert_same_rows, gj_nodes, oracle_plan_binary, oracle_run

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def fjm(torch_mod):
    from paper_2301_10841_amd import fj, runner
    fj.lib()
    return fj, runner


@pytest.fixture(scope="module")
def ctx_small(fjm):
    fj, _ = fjm
    c = fj.Context(0, tile=7)          # tiny frontiers: many tiles, deep recursion
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx(fjm):
    fj, _ = fjm
    c = fj.Context(0, tile=1 << 20)
    yield c
    c.close()


def gpu_run(fjm, ctx, dq, order=None, factor=True, nodes=None, materialize=True, stats=False, cap=None):
    _, runner = fjm
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_nodes(nodes) if nodes is not None else d.plan_binary(order, factor)
    r = d.run(plan, materialize=materialize, stats=stats, cap=cap)
    r["plan_nodes"] = plan.nodes()
    for c in r["colts"]:
        c.free()
    return r


# --------------------------------------------------------------- worked examples

@pytest.mark.parametrize("n", [1, 3, 6])
def test_clover_instance(fjm, ctx_small, n):
    dq = datagen.clover_instance(n)
    _say("clover", n)
    for order in itertools.permutations(range(3)):
        for factor in (False, True):
            r = gpu_run(fjm, ctx_small, dq, order, factor, stats=True)
            assert r["count"] == 1
            assert r["rows"].tolist() == [[0, 0, 0, 0]]
    # Section 4.1 probe counts: naive plan probes T n^2+1 times, factored n+1
    naive = gpu_run(fjm, ctx_small, dq, [0, 1, 2], False, stats=True)["stats"].per_node()
    assert naive[0]["probe"] == 2 * n + 1
    assert naive[1]["probe"] == n * n + 1
    fac = gpu_run(fjm, ctx_small, dq, [0, 1, 2], True, stats=True)["stats"].per_node()
    assert fac[0]["probe"] == (2 * n + 1) + (n + 1)
    gj = gpu_run(fjm, ctx_small, dq, nodes=gj_nodes(dq, [0, 1, 2, 3]))
    assert gj["count"] == 1


def test_clover_u_random_rows(fjm, ctx_small):
    # Section 4.2's plan [[R(x,a),S(x),T(x)],[U(b),S(b)],[T(c)]] on a random
    # bag instance: count and rows against the oracle (which tries get
    # forced is checked in test_gpu_laziness.py)
    dq = datagen.random_tiny_query(4, "clover_u", max_rows=12, domain=4)
    nodes = [[(0, (0, 1)), (1, (0,)), (2, (0,))], [(3, (2,)), (1, (2,))], [(2, (3,))]]
    want = oracle_run(dq, nodes)
    got = gpu_run(fjm, ctx_small, dq, nodes=nodes, stats=True)
    assert got["count"] == want["count"]
    assert_same_rows(got["rows"], want["rows"])


# ----------------------------------------------------------- random tiny bags

SHAPES = ["triangle", "clover", "chain3", "chain4", "star3", "cycle4", "clover_u", "pair", "single"]


@pytest.mark.parametrize("shape", SHAPES)
def test_tiny_vs_oracle(fjm, ctx_small, ctx, shape):
    for seed in range(4):
        dq = datagen.random_tiny_query(seed * 13 + 5, shape, max_rows=10, domain=3)
        _say("tiny", shape, seed)
        orders = list(itertools.permutations(range(len(dq.atoms))))[:6]
        plans = []
        for o in orders:
            plans.append(("bin", o, False))
            plans.append(("bin", o, True))
        for vo in list(itertools.permutations(range(dq.nvars)))[:4]:
            plans.append(("gj", vo, None))
        for i, (kind, arg, factor) in enumerate(plans):
            if kind == "bin":
                onodes = oracle_plan_binary(dq, arg, factor)
                want = oracle_run(dq, onodes, batch=(1, 2, 1000)[i % 3])
                got = gpu_run(fjm, ctx_small if i % 2 else ctx, dq, arg, factor)
            else:
                nodes = gj_nodes(dq, arg)
                want = oracle_run(dq, nodes, batch=2)
                got = gpu_run(fjm, ctx_small if i % 2 else ctx, dq, nodes=nodes)
            assert got["count"] == want["count"], (shape, seed, kind, arg)
            assert_same_rows(got["rows"], want["rows"])


def test_tail_products_match_full_execution(fjm):
    fj, _ = fjm
    c_full = fj.Context(0, tile=5, tail=1)
    try:
        for shape in ("clover", "star3", "chain4", "triangle"):
            dq = datagen.random_tiny_query(21, shape, max_rows=10, domain=3)
            order = list(range(len(dq.atoms)))
            want = oracle_run(dq, oracle_plan_binary(dq, order, True))
            got = gpu_run(fjm, c_full, dq, order, True)
            assert got["count"] == want["count"]
            assert_same_rows(got["rows"], want["rows"])
    finally:
        c_full.close()


def test_static_cover_counters_match_oracle(fjm, ctx):
    # nodes with one pure cover: the set of get() calls is fixed by the plan
    for shape in ("clover", "chain4", "star3"):
        dq = datagen.random_tiny_query(8, shape, max_rows=12, domain=3)
        for factor in (False, True):
            order = list(range(len(dq.atoms)))
            want = oracle_run(dq, oracle_plan_binary(dq, order, factor))
            got = gpu_run(fjm, ctx, dq, order, factor, stats=True)
            gs = got["stats"].per_node()
            for k in range(got["stats"].tail_from):
                assert gs[k]["probe"] == want["counters"][k]["probe"], (shape, factor, k)
                assert gs[k]["hit"] == want["counters"][k]["hit"], (shape, factor, k)


# -------------------------------------------------------------- workloads

@pytest.mark.parametrize("rep", [0, 1, 2])
def test_triangle_10k_edges(fjm, ctx, rep):
    e = datagen.triangle_edges(datagen.seed_for(1, rep))
    dq = datagen.synth.triangle_query(e)
    trace = closed.cycle_count(e[0], e[1], 3)
    _say("triangle", rep, trace)
    conv = oracle_plan_binary(dq, [0, 1, 2], True)
    want = oracle_run(dq, conv)
    assert want["count"] == trace
    got = gpu_run(fjm, ctx, dq, [0, 1, 2], True)
    assert got["count"] == trace
    assert_same_rows(got["rows"], want["rows"])
    gj = gpu_run(fjm, ctx, dq, nodes=gj_nodes(dq, [0, 1, 2]), stats=True)
    assert gj["count"] == trace
    assert_same_rows(gj["rows"], want["rows"])


def test_triangle_small_tiles(fjm, ctx_small):
    e = datagen.triangle_edges(77, n_edges=600, n_vertices=60)
    dq = datagen.synth.triangle_query(e)
    want = oracle_run(dq, gj_nodes(dq, [0, 1, 2]))
    got = gpu_run(fjm, ctx_small, dq, nodes=gj_nodes(dq, [0, 1, 2]))
    assert got["count"] == want["count"] == closed.cycle_count(e[0], e[1], 3)
    assert_same_rows(got["rows"], want["rows"])


def test_star_medium_vs_oracle(fjm, ctx):
    dq = datagen.star_schema(datagen.seed_for(2, 9), n_fact=300_000, n_dim=30_000)
    want = oracle_run(dq, oracle_plan_binary(dq, [0, 1, 2, 3, 4], True))
    got = gpu_run(fjm, ctx, dq, [0, 1, 2, 3, 4], True)
    assert got["count"] == want["count"]
    assert_same_rows(got["rows"], want["rows"])


def test_star_one_filter_large_output(fjm, ctx):
    # filter on D1 only: about 10% of the fact rows survive, all materialized
    dq = datagen.star_schema(datagen.seed_for(2, 3), n_fact=2_000_000, n_dim=200_000, filter_dims=[0])
    dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
    want = closed.star_rows(dq.relations[0].cols, dims, [10, None, None, None])
    got = gpu_run(fjm, ctx, dq, [0, 1, 2, 3, 4], True)
    assert got["count"] == want.shape[0]
    assert_same_rows(got["rows"], want)


def test_star_full_size(fjm):
    # 10M fact rows x 4 Zipf(1.1) keys, 4 x 1M dimension rows, attr < 10 on each
    fj, _ = fjm
    c = fj.Context(0)
    try:
        dq = datagen.star_schema(datagen.seed_for(2, 0))
        dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
        want = closed.star_rows(dq.relations[0].cols, dims, [10] * 4)
        got = gpu_run(fjm, c, dq, [0, 1, 2, 3, 4], True, stats=True)
        _say("star full", got["count"], want.shape[0])
        assert got["count"] == want.shape[0]
        assert_same_rows(got["rows"], want)
    finally:
        c.close()


@pytest.mark.parametrize("scale,edges", [(10, 8_000), (13, 60_000)])
def test_rmat_cycles(fjm, ctx, scale, edges):
    e = datagen.rmat_edges(datagen.seed_for(3, scale), scale, edges)
    tq = datagen.synth.triangle_query(e)
    t3 = closed.cycle_count(e[0], e[1], 3)
    for nodes in (None, gj_nodes(tq, [0, 1, 2]), gj_nodes(tq, [2, 0, 1])):
        r = gpu_run(fjm, ctx, tq, [0, 1, 2], True, nodes=nodes, materialize=False)
        assert r["count"] == t3
    cq = datagen.synth.four_cycle_query(e)
    t4 = closed.cycle_count(e[0], e[1], 4)
    for nodes in (None, gj_nodes(cq, [0, 1, 2, 3]), gj_nodes(cq, [0, 2, 1, 3])):
        r = gpu_run(fjm, ctx, cq, [0, 1, 2, 3], True, nodes=nodes, materialize=False)
        assert r["count"] == t4


def test_batch_mix_queries(fjm, ctx):
    qs, _ = datagen.batch_mix(11, n_queries=10, max_rows=30_000)
    for dq in qs:
        order = list(range(len(dq.atoms)))
        want = oracle_run(dq, oracle_plan_binary(dq, order, True))
        got = gpu_run(fjm, ctx, dq, order, True)
        assert got["count"] == want["count"], dq.kind
        assert_same_rows(got["rows"], want["rows"])


# -------------------------------------------------------------- edge cases

def test_truncation_keeps_exact_count(fjm, ctx):
    dq = datagen.random_tiny_query(3, "chain3", max_rows=10, domain=2)
    want = oracle_run(dq, oracle_plan_binary(dq, [0, 1, 2], True))
    assert want["count"] > 5
    got = gpu_run(fjm, ctx, dq, [0, 1, 2], True, cap=5)
    assert got["count"] == want["count"]
    assert got["written"] == 5
    # the written rows are a sub-multiset of the result
    from collections import Counter
    w = Counter(map(tuple, want["rows"].tolist()))
    g = Counter(map(tuple, got["rows"].tolist()))
    assert all(g[k] <= w[k] for k in g)


def test_empty_inputs(fjm, ctx):
    e = (np.zeros(0, np.int32), np.zeros(0, np.int32))
    dq = datagen.synth.triangle_query(e)
    assert gpu_run(fjm, ctx, dq, [0, 1, 2], True)["count"] == 0
    assert gpu_run(fjm, ctx, dq, nodes=gj_nodes(dq, [0, 1, 2]))["count"] == 0
    st = datagen.star_schema(5, n_fact=1000, n_dim=100, attr_lt=0)   # empty selections
    assert gpu_run(fjm, ctx, st, [0, 1, 2, 3, 4], True)["count"] == 0


def test_negative_and_sentinel_keys(fjm, ctx):
    # -1 is the empty marker of the 32-bit maps and (-1, -1) of the 64-bit ones
    r = np.array([-1, -1, 5, 0, -1], np.int32)
    s = np.array([-1, 3, 5, -1, 7], np.int32)
    dq = datagen.synth.make_query(
        ["x", "y", "z"],
        [datagen.Relation("R", [r, s]), datagen.Relation("S", [s, r]), datagen.Relation("T", [r, r])],
        [(0, (0, 1)), (1, (1, 2)), (2, (2, 0))])
    for order in itertools.permutations(range(3)):
        want = oracle_run(dq, oracle_plan_binary(dq, order, True))
        got = gpu_run(fjm, ctx, dq, order, True)
        assert got["count"] == want["count"]
        assert_same_rows(got["rows"], want["rows"])


def test_repeat_and_rebuild(fjm, ctx):
    _, runner = fjm
    e = datagen.triangle_edges(5, n_edges=2000, n_vertices=200)
    dq = datagen.synth.triangle_query(e)
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_nodes(gj_nodes(dq, [0, 1, 2]))
    colts = d.build(plan)
    want = closed.cycle_count(e[0], e[1], 3)
    c1, _, _ = ctx.execute(d.q, plan, colts)
    c2, _, _ = ctx.execute(d.q, plan, colts)     # inner levels already forced
    d.rebuild(colts)
    c3, _, _ = ctx.execute(d.q, plan, colts)
    assert c1 == c2 == c3 == want
    for c in colts:
        c.free()


def test_grouped_rebuild_matches_single_rebuilds(fjm, ctx):
    # one grouped pass over the COLTs of several queries (built and
    # directly iterated roots, an empty relation, inner levels forced lazily
    # afterwards) gives the same results as rebuilding them one by one
    fj, runner = fjm
    e = datagen.triangle_edges(7, n_edges=3000, n_vertices=300)
    tri = datagen.synth.triangle_query(e)
    empty = datagen.synth.triangle_query((np.zeros(0, np.int32), np.zeros(0, np.int32)))
    star = datagen.star_schema(11, n_fact=60_000, n_dim=6_000)
    chain = datagen.batch_mix(31, n_queries=4, max_rows=30_000)[0]
    runs = []
    for dq, nodes in [(tri, gj_nodes(tri, [0, 1, 2])), (tri, None), (empty, None), (star, None)] + \
            [(q, None) for q in chain]:
        d = runner.DeviceQuery(ctx, dq)
        plan = d.plan_nodes(nodes) if nodes else d.plan_binary(list(range(len(dq.atoms))), True)
        colts = d.build(plan)
        want = oracle_run(dq, plan.nodes(), materialize=False, counters=False)["count"]
        runs.append((d, plan, colts, want))
    for rep in range(3):
        allc, specs = [], []
        for d, plan, colts, _ in runs:
            for a, c in enumerate(colts):
                allc.append(c)
                specs.append((d.atom_cols(a), d.sel[a], d.nsel[a]))
        ctx.rebuild_colts(allc, specs)
        for d, plan, colts, want in runs:
            assert ctx.execute(d.q, plan, colts)[0] == want, (rep, d.dq.kind)
        # single rebuilds in between
        for d, plan, colts, want in runs:
            for a, c in enumerate(colts):
                ctx.rebuild_colt(c, d.atom_cols(a), d.sel[a], d.nsel[a])
            assert ctx.execute(d.q, plan, colts)[0] == want
    d, plan, colts, _ = runs[0]
    with pytest.raises(fj.FJError) as ex:
        ctx.rebuild_colts([colts[0], colts[0]], [(d.atom_cols(0), None, 0)] * 2)
    assert ex.value.status == -1
    for _, _, colts, _ in runs:
        for c in colts:
            c.free()


def test_scan_path_matches_generic_kernel(fjm, ctx):
    # the specialised first-node kernel and the generic one give the same
    # results and the same lookup counts
    fj, _ = fjm
    gen = fj.Context(0, tile=1 << 20, generic=True)
    try:
        cases = [datagen.star_schema(7, n_fact=50_000, n_dim=5_000),
                 datagen.synth.triangle_query(datagen.triangle_edges(3, n_edges=3000, n_vertices=400))]
        cases += [q for q in datagen.batch_mix(5, n_queries=6, max_rows=20_000)[0]]
        for dq in cases:
            order = list(range(len(dq.atoms)))
            a = gpu_run(fjm, ctx, dq, order, True, stats=True)
            b = gpu_run(fjm, gen, dq, order, True, stats=True)
            assert a["count"] == b["count"], dq.kind
            assert_same_rows(a["rows"], b["rows"])
            assert a["stats"].per_node()[0]["probe"] == b["stats"].per_node()[0]["probe"]
            assert a["stats"].per_node()[0]["hit"] == b["stats"].per_node()[0]["hit"]
    finally:
        gen.close()


def test_filters_match_numpy(fjm, ctx, torch_mod):
    # the pushed-down selection returns the passing row offsets in row order
    torch = torch_mod
    rng = np.random.default_rng(4)
    specs, want = [], []
    for n, bound in ((1, 5), (1023, 50), (4097, 0), (100_003, 10), (1_000_000, 37)):
        col = rng.integers(-20, 100, size=n).astype(np.int32)
        want.append(np.nonzero(col < bound)[0].astype(np.int32))
        specs.append((torch.from_numpy(col).cuda(), bound, torch.empty(n, dtype=torch.int32, device="cuda")))
    counts = ctx.filter_lt_batch(specs)
    for (c, b, out), w, k in zip(specs, want, counts):
        assert k == w.shape[0]
        assert np.array_equal(out[:k].cpu().numpy(), w)
        out2, k2 = ctx.filter_lt(c, b)
        assert k2 == k and np.array_equal(out2[:k2].cpu().numpy(), w)


@pytest.mark.parametrize("n_left,n_keys,fanout", [(500, 50, 20), (800, 10, 100), (3000, 50, 40)],
                         ids=["fused", "rows_apart", "many_bindings"])
def test_last_tile_emit_paths(fjm, ctx, n_left, n_keys, fanout):
    # the node-0 scan's last emit is enqueued before its binding count is
    # known: few bindings and rows are written by one workgroup, few bindings
    # with many rows by a second launch, many bindings by the general path
    dq = datagen.fanout_chain(datagen.seed_for(9, 2), n_left=n_left, n_keys=n_keys, fanout=fanout)
    want = oracle_run(dq, oracle_plan_binary(dq, [0, 1], True), counters=False)
    got = gpu_run(fjm, ctx, dq, [0, 1], True)
    assert got["count"] == want["count"] == n_left * fanout
    assert_same_rows(got["rows"], want["rows"])
    cut = gpu_run(fjm, ctx, dq, [0, 1], True, cap=777)
    assert cut["count"] == n_left * fanout and cut["written"] == 777
    from collections import Counter
    w = Counter(map(tuple, want["rows"].tolist()))
    g = Counter(map(tuple, cut["rows"].tolist()))
    assert all(g[k] <= w[k] for k in g)


def test_star_rows_written_by_the_probe_kernel(fjm, ctx):
    # the star's first node is its last probing node: the probe kernel writes
    # the result rows itself (four tails, one row per binding); a cap below
    # the count keeps the count exact and writes a sub-multiset of the rows
    dq = datagen.star_schema(datagen.seed_for(2, 5), n_fact=400_000, n_dim=20_000, attr_lt=40)
    want = oracle_run(dq, oracle_plan_binary(dq, [0, 1, 2, 3, 4], True), counters=False)
    assert want["count"] > 1000
    got = gpu_run(fjm, ctx, dq, [0, 1, 2, 3, 4], True)
    assert got["count"] == want["count"]
    assert_same_rows(got["rows"], want["rows"])
    cap = want["count"] // 3
    cut = gpu_run(fjm, ctx, dq, [0, 1, 2, 3, 4], True, cap=cap)
    assert cut["count"] == want["count"] and cut["written"] == cap
    from collections import Counter
    w = Counter(map(tuple, want["rows"].tolist()))
    g = Counter(map(tuple, cut["rows"].tolist()))
    assert all(g[k] <= w[k] for k in g)


@pytest.mark.parametrize("bound", [1 << 30, 500])
def test_range_build_long_slices(fjm, ctx, bound):
    # S(y, z) of 1.6M rows is the probed root, built range by range: with all
    # rows selected its place slices span two 1,024-item chunks each (the
    # pass reads its items twice), with about half of them one chunk; keys
    # are skewed (a few keys own many rows) and include the maps' empty
    # marker (-1).  Rows equal a plain merge of the two relations.
    _, runner = fjm
    rng = np.random.default_rng(17)
    ns, nk = 1_600_000, 100_000
    ys = np.minimum(rng.zipf(1.5, ns) - 1, nk - 1).astype(np.int32)   # 0 .. nk - 1, skewed
    ys[rng.choice(ns, 1000, replace=False)] = -1
    zs = rng.integers(0, 1000, ns).astype(np.int32)
    nr = 2_000
    xr = np.arange(nr, dtype=np.int32)
    yr = rng.integers(1, 5000, nr).astype(np.int32)   # not the hottest key: a bounded result
    yr[:3] = -1
    r = datagen.Relation("R", [xr, yr])
    s = datagen.Relation("S", [ys, zs])
    dq = datagen.synth.make_query(["x", "y", "z"], [r, s], [(0, (0, 1)), (1, (1, 2))],
                                  filters=[None, (1, bound)])
    keep = zs < bound
    # the expected rows: every R row with every selected S row of its key
    order = np.argsort(ys[keep], kind="stable")
    sy, sz = ys[keep][order], zs[keep][order]
    lo = np.searchsorted(sy, yr, "left")
    hi = np.searchsorted(sy, yr, "right")
    cnt = hi - lo
    want = np.empty((int(cnt.sum()), 3), dtype=np.int32)
    want[:, 0] = np.repeat(xr, cnt)
    want[:, 1] = np.repeat(yr, cnt)
    idx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]) if cnt.sum() else np.zeros(0, np.int64)
    want[:, 2] = sz[idx]
    want = runner.sort_rows(want)
    assert (ys[keep] == -1).any() and 0 < want.shape[0] < 3_000_000
    _say("long slices", bound, int(keep.sum()), "S rows,", want.shape[0], "result rows")
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary([0, 1], True)
    got = d.run(plan, materialize=True)
    assert got["count"] == want.shape[0]
    assert_same_rows(got["rows"], want)
    for c in got["colts"]:
        c.free()
