"""GPU parity of the laziness and dynamic-cover counters: which tries the
HIP path forces (Section 4.2) and which cover each binding iterates
(Section 4.4), against the oracle's counters and against values derived by
hand or from vertex degrees (the same pins the oracle is held to).

A kernel that forced every sub-trie up front, forced a root nobody probes,
or always iterated a node's first pure cover would fail here: the per-node
probe, hit, forced and forced-offset counts would differ."""

import sys

import numpy as np
import pytest

import datagen
from oracle import closed
from tests.gpu_util import gj_nodes, oracle_run
from tests.test_oracle_laziness import CLOVER_U_PLAN, gj_triangle_counters

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fjm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10841_amd import fj, runner
    fj.lib()
    return fj, runner


@pytest.fixture(scope="module", params=[7, 1 << 20], ids=["tile7", "tile1M"])
def ctx(fjm, request):
    fj, _ = fjm
    c = fj.Context(0, tile=request.param)
    yield c
    c.close()


def _gpu(fjm, ctx, dq, nodes, materialize=True):
    _, runner = fjm
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_nodes(nodes)
    r = d.run(plan, materialize=materialize, stats=True)
    for c in r["colts"]:
        c.free()
    return r


def _assert_counters(stats, want):
    """Per node: forced tries and offsets everywhere; cover tuples, get()
    calls and hits on the probing nodes; survivors where they feed another
    probing node (the last probing node's survivors are the output)."""
    gs = stats.per_node()
    tf = stats.tail_from
    for k, w in enumerate(want):
        g = gs[k]
        assert (g["forced"], g["forced_offsets"]) == (w["forced"], w["forced_offsets"]), (k, g, w)
        if k < tf:
            assert (g["cover"], g["probe"], g["hit"]) == (w["cover"], w["probe"], w["hit"]), (k, g, w)
        if k < tf - 1:
            assert g["survivors"] == w["survivors"], (k, g, w)


@pytest.mark.parametrize("n", [1, 3])
def test_clover_u_cover_is_u(fjm, ctx, n):
    # |U| = 1 ties with |S[x0]| = 1 and U, first in node order, is the cover:
    # U is iterated over its base table and never forced; its one lookup
    # forces S[x0] (one trie of one offset) and nothing else
    dq = datagen.clover_u_instance(n, [0])
    _say("clover+U, U covers", n)
    want = oracle_run(dq, CLOVER_U_PLAN, batch=4)
    got = _gpu(fjm, ctx, dq, CLOVER_U_PLAN)
    assert got["count"] == want["count"] == 1
    assert got["rows"].tolist() == [[0, 0, 0, 0]]
    c1 = {"cover": 1, "probe": 1, "hit": 1, "survivors": 1, "forced": 1, "forced_offsets": 1}
    assert want["counters"][1] == c1
    _assert_counters(got["stats"], want["counters"])
    g0 = got["stats"].per_node()[0]
    assert (g0["cover"], g0["probe"], g0["hit"], g0["forced"]) == (2 * n + 1, 3 * n + 2, n + 2, 0)


@pytest.mark.parametrize("extra", [1, 5])
def test_clover_u_cover_is_s(fjm, ctx, extra):
    # |U| > |S[x0]|: S[x0] is iterated by offset and never forced; U's root
    # map is built by its one probe, over all of U's rows, during node 1
    dq = datagen.clover_u_instance(2, [0] + [5000 + j for j in range(extra)])
    _say("clover+U, S covers", extra)
    want = oracle_run(dq, CLOVER_U_PLAN, batch=4)
    got = _gpu(fjm, ctx, dq, CLOVER_U_PLAN)
    assert got["count"] == want["count"] == 1
    assert want["counters"][1]["forced_offsets"] == 1 + extra
    _assert_counters(got["stats"], want["counters"])


def test_clover_u_duplicates_and_misses(fjm, ctx):
    # U = {b0, b0}: an unforced vector's size is its length (2), so S[x0]
    # covers and the result counts the duplicate; U = {7}: U covers, its
    # lookup forces S[x0] and misses; U empty: nothing is iterated or forced
    for u, count in (([0, 0], 2), ([7], 0), ([], 0)):
        dq = datagen.clover_u_instance(3, u)
        _say("clover+U", u)
        want = oracle_run(dq, CLOVER_U_PLAN, batch=4)
        got = _gpu(fjm, ctx, dq, CLOVER_U_PLAN)
        assert got["count"] == want["count"] == count
        _assert_counters(got["stats"], want["counters"])


@pytest.mark.parametrize("seed,ne,nv", [(11, 800, 40), (5, 3000, 300)])
def test_gj_triangle_counters_small(fjm, ctx, seed, ne, nv):
    e = datagen.triangle_edges(seed, n_edges=ne, n_vertices=nv)
    dq = datagen.synth.triangle_query(e)
    _say("gj triangle counters", seed, ne, nv)
    nodes = gj_nodes(dq, [0, 1, 2])
    want = gj_triangle_counters(e[0], e[1], nv)
    # node 2's hits are the triangles: each output is one hit
    want[2]["hit"] = closed.cycle_count(e[0], e[1], 3)
    got = _gpu(fjm, ctx, dq, nodes, materialize=False)
    assert got["count"] == want[2]["hit"]
    _assert_counters(got["stats"], want)


@pytest.mark.parametrize("rep", [0, 1])
def test_gj_triangle_10k_counters(fjm, ctx, rep):
    # the triangle workload (10,000 distinct edges over 2,000 vertices):
    # node 2 iterates min(|S[y]|, |T[x]|) per binding and forces the other
    # trie at its first probe, so its get() count is that sum
    e = datagen.triangle_edges(datagen.seed_for(1, rep))
    dq = datagen.synth.triangle_query(e)
    _say("gj triangle 10k counters", rep)
    nodes = gj_nodes(dq, [0, 1, 2])
    want = oracle_run(dq, nodes, materialize=False)
    pinned = gj_triangle_counters(e[0], e[1], 2000)
    for k in range(3):
        for name in ("cover", "probe", "forced", "forced_offsets"):
            assert want["counters"][k][name] == pinned[k][name]
    got = _gpu(fjm, ctx, dq, nodes, materialize=False)
    assert got["count"] == want["count"]
    _assert_counters(got["stats"], want["counters"])
    # a kernel always iterating the node's first cover, S[y], would probe
    # sum |S[y]| over node 2's bindings: strictly more on this instance
    src, dst = np.asarray(e[0], np.int64), np.asarray(e[1], np.int64)
    outdeg, indeg = np.bincount(src, minlength=2000), np.bincount(dst, minlength=2000)
    live = (outdeg[src] > 0) & (indeg[src] > 0) & (outdeg[dst] > 0)
    first_cover = int(outdeg[dst[live]].sum())
    assert got["stats"].per_node()[2]["probe"] == pinned[2]["probe"] < first_cover
