"""Pins of the oracle's laziness and dynamic-cover counters: which tries COLT
forces (Section 4.2) and which cover each binding iterates (Section 4.4).

The expected counters are derived by hand from the instances (the clover
instance of Section 3 extended with U(b) as in Section 4.2's COLT example) or
computed with numpy from vertex degrees (Generic Join's triangle plan), never
by the oracle itself.  A force charged to the wrong node, a root built when
the paper leaves it unbuilt, an iterated last-level vector that gets forced,
or a cover chosen by the wrong size or tie rule fails one of them.
"""

import numpy as np
import pytest

import datagen
from oracle import cfj, closed
from oracle import plans as P

# Section 4.2's plan for Q(x,a,b,c) :- R(x,a), S(x,b), T(x,c), U(b):
# [[R(x,a), S(x), T(x)], [U(b), S(b)], [T(c)]]  (atoms R=0, S=1, T=2, U=3;
# variables x=0, a=1, b=2, c=3)
CLOVER_U_PLAN = [[(0, (0, 1)), (1, (0,)), (2, (0,))], [(3, (2,)), (1, (2,))], [(2, (3,))]]


def _clover_u(n, u_values):
    q = datagen.clover_u_instance(n, u_values)
    return q, cfj.run(q, CLOVER_U_PLAN, batch=4)


def _node0_and_build(r, n):
    # R is the only pure cover of node 0 and has one level: iterated over the
    # base table, never built.  S and T are probed there: their roots (every
    # row, 2n + 1 each) are the build phase's two forces.
    b = r["build"]
    assert (b["forced"], b["forced_offsets"]) == (2, 2 * (2 * n + 1))
    c0 = r["counters"][0]
    # 2n + 1 R rows; S(x) probed by each, hit by x0 and the n x2 rows; T(x)
    # probed by those n + 1, hit by x0 only
    assert c0 == {"cover": 2 * n + 1, "probe": (2 * n + 1) + (n + 1), "hit": (n + 1) + 1,
                  "survivors": 1, "forced": 0, "forced_offsets": 0}


@pytest.mark.parametrize("n", [1, 2, 5])
def test_colt_u_is_cover(n):
    # U = {b0}: |U| = 1 = |S[x0]| (the instance has one S row for x0), the
    # tie goes to U, first in node order.  U is iterated over its base
    # table (never forced); the first lookup in S[x0] forces x0's subtrie
    # of S, one offset, and nothing else: the paper's first reading of the
    # example.  T[x0] at the last node is iterated by offset: never forced.
    q, r = _clover_u(n, [0])
    assert r["count"] == 1 and r["rows"].tolist() == [[0, 0, 0, 0]]
    _node0_and_build(r, n)
    c1, c2 = r["counters"][1], r["counters"][2]
    assert c1 == {"cover": 1, "probe": 1, "hit": 1, "survivors": 1, "forced": 1, "forced_offsets": 1}
    assert c2 == {"cover": 1, "probe": 0, "hit": 0, "survivors": 1, "forced": 0, "forced_offsets": 0}


@pytest.mark.parametrize("n", [1, 3])
@pytest.mark.parametrize("extra", [1, 4])
def test_colt_s_is_cover(n, extra):
    # U = {b0} plus `extra` values no S row holds: |U| > |S[x0]| = 1, so S(b)
    # is the cover (the paper's "more realistic" reading).  S[x0] is
    # iterated by offset and never forced; U's map is built by its one get,
    # over all of U's rows, charged to node 1.
    u = [0] + [5000 + j for j in range(extra)]
    q, r = _clover_u(n, u)
    assert r["count"] == 1
    _node0_and_build(r, n)
    c1, c2 = r["counters"][1], r["counters"][2]
    assert c1 == {"cover": 1, "probe": 1, "hit": 1, "survivors": 1, "forced": 1,
                  "forced_offsets": 1 + extra}
    assert (c2["forced"], c2["probe"]) == (0, 0)


def test_colt_unforced_size_is_length():
    # U = {b0, b0}: one distinct key but two rows.  An unforced vector's size
    # is its length (2) against S[x0]'s 1, so S is the cover, and the result
    # counts the duplicate: two rows (x0, a0, b0, c0)
    q, r = _clover_u(2, [0, 0])
    assert r["count"] == 2
    c1 = r["counters"][1]
    assert (c1["cover"], c1["probe"], c1["forced"], c1["forced_offsets"]) == (1, 1, 1, 2)


def test_colt_empty_u():
    # U empty: size 0 wins, nothing is iterated, nothing forced at node 1
    q, r = _clover_u(3, [])
    assert r["count"] == 0
    c1 = r["counters"][1]
    assert (c1["cover"], c1["probe"], c1["forced"]) == (0, 0, 0)


def test_colt_u_cover_miss():
    # U = {7}: a b-value S[x0] lacks; size 1 ties with S[x0] and U is the
    # cover.  The one lookup still forces S[x0], then misses.
    q, r = _clover_u(2, [7])
    assert r["count"] == 0
    c1 = r["counters"][1]
    assert c1 == {"cover": 1, "probe": 1, "hit": 0, "survivors": 0, "forced": 1, "forced_offsets": 1}
    assert r["counters"][2]["cover"] == 0


def test_colt_independent_of_batch():
    # the set of get() calls, hence the forced set, does not depend on the
    # vector batch (Section 4.3)
    q = datagen.clover_u_instance(4, [0, 9, 9])
    ref = cfj.run(q, CLOVER_U_PLAN, batch=1)
    for b in (2, 3, 1000):
        r = cfj.run(q, CLOVER_U_PLAN, batch=b)
        assert r["counters"] == ref["counters"] and r["build"] == ref["build"]


def gj_triangle_counters(src, dst, nv):
    """Counters of Generic Join's triangle plan [[R(x),T(x)],[R(y),S(y)],
    [S(z),T(z)]] over R = S = T = E with distinct edges, from degrees alone.

    Roots are keyed by x (R: sources; T(z,x): destinations) and by y (S:
    sources), all built up front.  Node 0 iterates the root with fewer keys
    (ties to R).  Node 1 iterates R[x] (out-degree of x) against S's root.
    Node 2 iterates the smaller of S[y] (out-degree of y) and T[x]
    (in-degree of x), ties to S, and probes the other, which forces it at
    its first probe: one force per distinct losing trie, of its length."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    outdeg = np.bincount(src, minlength=nv)
    indeg = np.bincount(dst, minlength=nv)
    nsrc = int((outdeg > 0).sum())
    ndst = int((indeg > 0).sum())
    xs = np.nonzero((outdeg > 0) & (indeg > 0))[0]
    c = [dict(cover=0, probe=0, hit=0, survivors=0, forced=0, forced_offsets=0) for _ in range(3)]
    if nsrc <= ndst:
        c[0]["cover"], c[0]["probe"] = nsrc, nsrc
    else:
        c[0]["cover"], c[0]["probe"] = ndst, ndst
    c[0]["hit"] = c[0]["survivors"] = len(xs)
    # node 1: bindings x; R[x] has out-degree keys; S root has nsrc keys
    assert (outdeg[xs] <= nsrc).all()
    live1 = np.isin(src, xs)
    c[1]["cover"] = c[1]["probe"] = int(live1.sum())
    b_x, b_y = src[live1], dst[live1]
    hit = outdeg[b_y] > 0
    c[1]["hit"] = c[1]["survivors"] = int(hit.sum())
    x2, y2 = b_x[hit], b_y[hit]
    s_cover = outdeg[y2] <= indeg[x2]
    c[2]["cover"] = int(np.where(s_cover, outdeg[y2], indeg[x2]).sum())
    c[2]["probe"] = c[2]["cover"]
    t_forced = np.unique(x2[s_cover])
    s_forced = np.unique(y2[~s_cover])
    c[2]["forced"] = len(t_forced) + len(s_forced)
    c[2]["forced_offsets"] = int(indeg[t_forced].sum() + outdeg[s_forced].sum())
    return c


@pytest.mark.parametrize("seed,ne,nv", [(5, 3000, 300), (11, 800, 40), (1, 10_000, 2_000)])
def test_gj_triangle_counters(seed, ne, nv):
    e = datagen.triangle_edges(seed, n_edges=ne, n_vertices=nv)
    q = datagen.synth.triangle_query(e)
    r = cfj.run(q, P.gj_plan(q, [0, 1, 2]), materialize=False, batch=(7 if ne < 1000 else 1000))
    want = gj_triangle_counters(e[0], e[1], nv)
    got = r["counters"]
    for k in range(3):
        for name in ("cover", "probe", "forced", "forced_offsets"):
            assert got[k][name] == want[k][name], (k, name, got[k], want[k])
    for k in range(2):
        assert got[k]["hit"] == want[k]["hit"]
    # node 2's hits are the triangles: each output is one hit
    assert got[2]["hit"] == r["count"] == closed.cycle_count(e[0], e[1], 3)
    # roots of R (sources), S (sources) and T (destinations): every row each
    assert r["build"]["forced"] == 3 and r["build"]["forced_offsets"] == 3 * ne
