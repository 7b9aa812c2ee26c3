"""Parity at the workloads' full sizes: R-MAT with 2^22 vertices and 50M
edges (the triangle count against the oracle's, summed over disjoint parts
of x by a committed script, plan invariance, and the triangles through
sampled vertices against the oracle and the closed form),
and batched-mix queries at full relation sizes (counts against the oracle)."""

import os
import sys

import numpy as np
import pytest

import datagen
from datagen import synth
from oracle import cfj, closed
from oracle import plans as P
from tests.gpu_util import gj_nodes

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10841_amd import fj, runner
    ctx = fj.Context(0)
    yield fj, runner, ctx
    ctx.close()


def _count(runner, ctx, dq, order=None, nodes=None):
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_nodes(nodes) if nodes is not None else d.plan_binary(order, True)
    r = d.run(plan, materialize=False)
    for c in r["colts"]:
        c.free()
    return r["count"]


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat_s22_triangles.txt")


def golden_triangles():
    """The oracle's count for the full graph (tests/golden/make_rmat_triangles.py)."""
    lines = [ln for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    return int(lines[0])


def test_rmat_full_scale_triangles(env):
    fj, runner, ctx = env
    src, dst = datagen.rmat_edges(datagen.seed_for(3, 1), 22, 50_000_000)
    _say("R-MAT edges", src.size)
    assert src.size == 50_000_000
    tq = synth.triangle_query((src, dst))
    gj = _count(runner, ctx, tq, nodes=gj_nodes(tq, [0, 1, 2]))
    conv = _count(runner, ctx, tq, order=[0, 1, 2])
    _say("triangles", gj, conv)
    assert gj == conv == golden_triangles()
    # the triangles through 256 sampled x vertices use exactly the R rows
    # leaving the sample, the S rows those reach and the T rows closing back
    rng = np.random.default_rng(99)
    xs = rng.choice(np.unique(src), size=256, replace=False)
    kr = np.isin(src, xs)
    ks = np.isin(src, np.unique(dst[kr]))
    kt = np.isin(dst, xs)
    rels = [synth.Relation("R", [src[kr], dst[kr]]), synth.Relation("S", [src[ks], dst[ks]]),
            synth.Relation("T", [src[kt], dst[kt]])]
    sq = synth.make_query(["x", "y", "z"], rels, [(0, (0, 1)), (1, (1, 2)), (2, (2, 0))])
    got = _count(runner, ctx, sq, order=[0, 1, 2])
    want = cfj.run(sq, P.factor(P.binary2fj(sq, [0, 1, 2])), materialize=False, counters=False)["count"]
    tr = closed.triangle_count((src[kr], dst[kr]), (src[ks], dst[ks]), (src[kt], dst[kt]))
    _say("sampled triangles", got, want, tr)
    assert got == want == tr
    assert 0 < got < gj


def test_batch_queries_at_full_size(env):
    fj, runner, ctx = env
    seed = datagen.seed_for(4, 0)
    for i in range(16):
        dq, _ = datagen.batch_query(seed, i)
        order = list(range(len(dq.atoms)))
        got = _count(runner, ctx, dq, order=order)
        want = cfj.run(dq, P.factor(P.binary2fj(dq, order)), materialize=False, counters=False)["count"]
        _say(i, dq.kind, [r.nrows for r in dq.relations], got)
        assert got == want, (i, dq.kind)


def _golden_cycle4():
    f = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat_cycle4_counts.txt")
    out = {}
    for ln in open(f):
        if ln.strip() and not ln.startswith("#"):
            s, e, n = ln.split()
            out[int(s)] = (int(e), int(n))
    return out


@pytest.mark.parametrize("scale", [16, 18])
def test_rmat_cycle4_reduced_scales(env, scale):
    # the directed 4-cycle Q(w,x,y,z) :- E(w,x),E(x,y),E(y,z),E(z,w) with
    # Generic Join's plan, counted without materializing (the last node's
    # intersections are counted, not emitted), against trace(A^4)
    # (tests/golden/make_rmat_cycle4.py)
    fj, runner, ctx = env
    n_edges, want = _golden_cycle4()[scale]
    src, dst = datagen.rmat_edges(datagen.seed_for(3, 1), scale, n_edges)
    assert src.size == n_edges
    q4 = synth.four_cycle_query((src, dst))
    nodes = [[(0, (0,)), (3, (0,))], [(0, (1,)), (1, (1,))], [(1, (2,)), (2, (2,))], [(2, (3,)), (3, (3,))]]
    got = _count(runner, ctx, q4, nodes=nodes)
    _say("4-cycles", scale, got, want)
    assert got == want
