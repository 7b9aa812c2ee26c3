"""The first-node scan with a key filter: the range-by-range root build
writes a membership filter of each root map's keys (two bits of one word
per key), and the first node's scan keeps the first lookup's filter in LDS,
so most misses of a selective join never load a bucket.  Results, emitted
rows and lookup counts must equal the same scan without the filter, the
generic probe kernel and the closed form or the oracle: on a selective star,
on an unselective one whose hits overflow a batch, on ragged tiles, with a
selection on the cover, and with keys equal to the maps' empty marker."""

import sys

import numpy as np
import pytest

import datagen
from oracle import closed
from tests.gpu_util import assert_same_rows, oracle_plan_binary, oracle_run

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


@pytest.fixture(scope="module")
def ctxs(fjm):
    fj, _ = fjm
    cs = {"filter": fj.Context(0, tile=1 << 22),
          "plain": fj.Context(0, tile=1 << 22, no_filter=True),
          "generic": fj.Context(0, tile=1 << 22, generic=True)}
    yield cs
    for c in cs.values():
        c.close()


def _run(fjm, ctx, dq, cap=None):
    _, runner = fjm
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary(list(range(len(dq.atoms))), True)
    r = d.run(plan, materialize=True, stats=True, cap=cap)
    for c in r["colts"]:
        c.free()
    return r


def _all_three(fjm, ctxs, dq, want_rows):
    """Runs dq in the three contexts; returns the filtered run's stats."""
    got = {k: _run(fjm, c, dq) for k, c in ctxs.items()}
    for k, g in got.items():
        assert g["count"] == want_rows.shape[0], k
        assert_same_rows(g["rows"], want_rows)
    f, p, g = (got[k]["stats"].per_node() for k in ("filter", "plain", "generic"))
    assert f[0]["probe"] == p[0]["probe"] == g[0]["probe"]
    assert f[0]["hit"] == p[0]["hit"] == g[0]["hit"]
    assert got["plain"]["stats"].filtered == 0 and got["generic"]["stats"].filtered == 0
    return got["filter"]["stats"]


def test_selective_star_filter_settles_most_misses(fjm, ctxs):
    # attr < 10 on every dimension: about 90% of the fact rows miss lookup 0
    dq = datagen.star_schema(datagen.seed_for(2, 11), n_fact=1_000_003, n_dim=100_000)
    dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
    want = closed.star_rows(dq.relations[0].cols, dims, [10] * 4)
    st = _all_three(fjm, ctxs, dq, want)
    node0 = st.per_node()[0]
    misses0 = dq.relations[0].cols[0].shape[0] - int(np.isin(
        dq.relations[0].cols[0], dims[0][0][dims[0][1] < 10]).sum())
    _say("filtered", st.filtered, "of", misses0, "first-lookup misses")
    assert 0 < st.filtered <= misses0
    assert st.filtered >= misses0 // 2          # two bits a key, about six keys a word
    assert node0["probe"] >= dq.relations[0].cols[0].shape[0]


def test_unselective_lookup_overflows_the_batch(fjm, ctxs):
    # every dimension row passes, so every fact row hits every lookup: a
    # tile's hits exceed a batch and are added a row per thread at a time
    dq = datagen.star_schema(datagen.seed_for(2, 12), n_fact=200_001, n_dim=20_000, attr_lt=100)
    dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
    want = closed.star_rows(dq.relations[0].cols, dims, [100] * 4)
    assert want.shape[0] == 200_001
    st = _all_three(fjm, ctxs, dq, want)
    assert st.filtered == 0


@pytest.mark.parametrize("n_fact", [1, 777, 8192, 3 * 8192 + 17])
def test_ragged_tiles(fjm, ctxs, n_fact):
    dq = datagen.star_schema(datagen.seed_for(2, 13), n_fact=n_fact, n_dim=3_000, attr_lt=30)
    dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
    want = closed.star_rows(dq.relations[0].cols, dims, [30] * 4)
    _all_three(fjm, ctxs, dq, want)


def test_selection_on_the_cover(fjm, ctxs):
    # the cover relation has a selection of its own: its rows are read
    # through the selection's offsets
    rng = np.random.default_rng(5)
    n, nd = 100_000, 5_000
    f = datagen.Relation("F", [rng.integers(0, nd, n).astype(np.int32), rng.integers(0, nd, n).astype(np.int32),
                               rng.integers(0, 1000, n).astype(np.int32)])
    d1 = datagen.Relation("D1", [np.arange(nd, dtype=np.int32), rng.integers(0, 100, nd).astype(np.int32)])
    d2 = datagen.Relation("D2", [rng.permutation(nd).astype(np.int32), rng.integers(0, 100, nd).astype(np.int32)])
    dq = datagen.synth.make_query(["k1", "k2", "f", "a1", "a2"], [f, d1, d2],
                                  [(0, (0, 1, 2)), (1, (0, 3)), (2, (1, 4))],
                                  filters=[(2, 400), (1, 20), None])
    want = oracle_run(dq, oracle_plan_binary(dq, [0, 1, 2], True), counters=False)
    assert 0 < want["count"] < n
    _all_three(fjm, ctxs, dq, want["rows"])


def test_empty_marker_keys(fjm, ctxs):
    # -1 is the 32-bit maps' empty marker, kept in their reserved slot and
    # not in the filter: such keys bypass it
    rng = np.random.default_rng(6)
    n, nd = 50_000, 2_000
    k1 = rng.integers(-1, nd, n).astype(np.int32)
    k2 = rng.integers(-1, nd, n).astype(np.int32)
    pk1 = np.arange(-1, nd - 1, dtype=np.int32)
    pk2 = np.arange(0, nd, dtype=np.int32)   # no -1 key: the reserved slot stays empty
    f = datagen.Relation("F", [k1, k2])
    a1 = rng.integers(0, 100, nd).astype(np.int32)
    a1[0] = 0                                 # the row keyed -1 passes D1's selection
    d1 = datagen.Relation("D1", [pk1, a1])
    d2 = datagen.Relation("D2", [pk2, rng.integers(0, 100, nd).astype(np.int32)])
    dq = datagen.synth.make_query(["k1", "k2", "a1", "a2"], [f, d1, d2],
                                  [(0, (0, 1)), (1, (0, 2)), (2, (1, 3))],
                                  filters=[None, (1, 15), (1, 60)])
    want = oracle_run(dq, oracle_plan_binary(dq, [0, 1, 2], True), counters=False)
    assert (want["rows"][:, 0] == -1).any()
    _all_three(fjm, ctxs, dq, want["rows"])


def test_select_rebuild_matches_two_calls(fjm, ctxs):
    # fj_select_rebuild (the selections and the grouped rebuild in one call)
    # gives the same selection counts, rows and lookup counts as
    # fj_filter_lt_batch followed by fj_colt_rebuild_many, step after step
    fj, runner = fjm
    ctx = ctxs["filter"]
    dq = datagen.star_schema(datagen.seed_for(2, 14), n_fact=300_007, n_dim=30_000)
    dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
    want = closed.star_rows(dq.relations[0].cols, dims, [10] * 4)
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary([0, 1, 2, 3, 4], True)
    colts = d.build(plan)
    import torch
    out = torch.empty((want.shape[0] + 5, dq.nvars), dtype=torch.int32, device="cuda:0")
    two = list(d.nsel)
    for rep in range(3):
        d.nsel = [0] * len(d.nsel)
        d.select_rebuild(colts)
        assert d.nsel == two, rep
        cnt, written, st = ctx.execute(d.q, plan, colts, out=out, stats=True)
        assert cnt == written == want.shape[0]
        assert_same_rows(runner.sort_rows(out[:written].cpu().numpy()), want)
        d.apply_filters()
        d.rebuild(colts)
        _, _, st2 = ctx.execute(d.q, plan, colts, stats=True)
        assert st.per_node() == st2.per_node()
    # argument errors are refused before any device work
    import ctypes as C
    key = tuple(c.h for c in colts)
    arr = (C.c_void_p * len(key))(*key)
    rels = (fj.Relation * len(colts))(*[fj._relation(d.atom_cols(a), d.sel[a], d.nsel[a])
                                         for a in range(len(colts))])
    for atoms, cols in [([1, 1], [1, 1]), ([7], [1]), ([1], [5])]:
        at = (C.c_int32 * len(atoms))(*atoms)
        co = (C.c_int32 * len(cols))(*cols)
        bo = (C.c_int32 * len(atoms))(*([10] * len(atoms)))
        with pytest.raises(fj.FJError) as ex:
            ctx.select_rebuild_prepared(len(atoms), at, co, bo, len(colts), arr, rels)
        assert ex.value.status == -1, (atoms, cols)
    for c in colts:
        c.free()
