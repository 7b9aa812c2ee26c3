"""GPU parity of the batched persistent executor: every query's count equals
the oracle's and the single-query path's, on every graph replay."""

import numpy as np
import pytest

import datagen
from oracle import closed
from tests.gpu_util import oracle_plan_binary, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10841_amd import fj, runner
    ctx = fj.Context(0, tile=1 << 20)
    yield fj, runner, ctx
    ctx.close()


def _queries():
    qs, _ = datagen.batch_mix(17, n_queries=24, max_rows=40_000)
    qs.append(datagen.star_schema(3, n_fact=200_000, n_dim=20_000))
    qs.append(datagen.synth.triangle_query(datagen.triangle_edges(datagen.seed_for(1, 1))))
    qs.append(datagen.random_tiny_query(2, "chain4", max_rows=10, domain=3))
    qs.append(datagen.synth.triangle_query((np.zeros(0, np.int32), np.zeros(0, np.int32))))
    return qs


def test_batch_counts_match_oracle_and_single(env):
    fj, runner, ctx = env
    qs = _queries()
    devs, items, want, single = [], [], [], []
    for dq in qs:
        order = list(range(len(dq.atoms)))
        want.append(oracle_run(dq, oracle_plan_binary(dq, order, True), materialize=False, counters=False)["count"])
        d = runner.DeviceQuery(ctx, dq)
        plan = d.plan_binary(order, True)
        colts = d.build(plan)
        single.append(ctx.execute(d.q, plan, colts)[0])
        d.rebuild(colts)
        devs.append(d)
        items.append((d.q, plan, colts))
    assert single == want
    b = fj.Batch(ctx, items, chunk=512)
    for rep in range(3):
        got = b.run()
        assert got == want, rep
        # eager work between replays
        ctx.execute(devs[0].q, items[0][1], items[0][2])
    b.free()
    b2 = fj.Batch(ctx, items, chunk=2048, block=128, graph=False)
    assert b2.run() == want
    b2.free()
    qc = [64 + 64 * (i % 7) for i in range(len(items))]
    b3 = fj.Batch(ctx, items, query_chunk=qc)
    assert b3.run() == want
    b3.free()
    for _, _, cs in items:
        for c in cs:
            c.free()


def test_batch_refuses_plans_with_inner_probes(env):
    fj, runner, ctx = env
    dq = datagen.synth.triangle_query(datagen.triangle_edges(5, n_edges=500, n_vertices=60))
    d = runner.DeviceQuery(ctx, dq)
    gj = d.plan_nodes([[(0, (0,)), (2, (0,))], [(0, (1,)), (1, (1,))], [(1, (2,)), (2, (2,))]])
    colts = d.build(gj)
    with pytest.raises(fj.FJError) as e:
        fj.Batch(ctx, [(d.q, gj, colts)])
    assert e.value.status == -6
    for c in colts:
        c.free()


def _golden_batch_counts():
    import os
    f = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_seed4_counts.txt")
    out = {}
    for ln in open(f):
        if ln.startswith("#") or not ln.strip():
            continue
        i, kind, n = ln.split()
        out[int(i)] = (kind, int(n))
    return out


def test_batch_full_workload_matches_oracle(env):
    # the batched workload at its real shape: the 256 queries of
    # batch_mix(seed_for(4, 0)) (relations of 1K-2M rows) in one persistent
    # launch, against the oracle's counts (tests/golden/make_batch_counts.py),
    # on two replays, with the default and with autotuned-style chunks
    fj, runner, ctx = env
    from paper_2301_10841_amd import autotune
    golden = _golden_batch_counts()
    n = len(golden)
    assert n == 256
    seed = datagen.seed_for(4, 0)
    items, rows = [], []
    for i in range(n):
        dq, _ = datagen.batch_query(seed, i)
        assert dq.kind == golden[i][0]
        d = runner.DeviceQuery(ctx, dq)
        plan = d.plan_binary(list(range(len(dq.atoms))), True)
        items.append((d.q, plan, d.build(plan)))
        rows.append(dq.relations[dq.atoms[0][0]].nrows)
    want = [golden[i][1] for i in range(n)]
    print("loaded", n, "queries,", sum(rows), "first-node rows", flush=True)
    b = fj.Batch(ctx, items)
    assert b.run() == want
    assert b.run() == want
    b.free()
    # a tuner-shaped setting: small chunks for short queries, large for long
    setting = {"block": 128, "chunk_by_bucket": {"0": 64, "1": 256, "2": 1024, "3": 4096, "4": 4096}}
    b2 = fj.Batch(ctx, items, block=setting["block"], query_chunk=autotune.chunks_for(setting, rows))
    assert b2.run() == want
    b2.free()
    for _, _, cs in items:
        for c in cs:
            c.free()
