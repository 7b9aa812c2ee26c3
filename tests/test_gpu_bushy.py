"""GPU parity of bushy plans (Section 2.2): the HIP path runs the left-deep
decomposition through fj_execute_bushy (intermediates materialized on the
device); results must equal the oracle's decomposition run and the query's
own result, bit for bit."""

import sys

import numpy as np
import pytest

import datagen
from oracle import brute
from oracle import bushy as B
from tests.gpu_util import assert_same_rows
from tests.test_oracle_bushy import random_tree

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


def _check(fjm, ctx, dq, tree, want=None):
    _, runner = fjm
    d = runner.DeviceQuery(ctx, dq)
    got = d.run_bushy(tree)
    if want is None:
        want = B.evaluate(dq, tree)
    assert got["count"] == want["count"], (tree, got["count"], want["count"])
    assert_same_rows(got["rows"], want["rows"])
    return got


@pytest.mark.parametrize("shape", ["triangle", "chain3", "chain4", "star3", "cycle4", "clover", "pair"])
def test_tiny_random_trees(fjm, ctx, shape):
    rng = np.random.Generator(np.random.PCG64(17))
    for rep in range(8):
        dq = datagen.random_tiny_query(datagen.seed_for(8, rep), shape)
        tree = random_tree(range(len(dq.atoms)), rng)
        _say("tiny", shape, rep, tree)
        want = B.evaluate(dq, tree)
        assert want["count"] == brute.count(dq)
        _check(fjm, ctx, dq, tree, want)


def test_paper_example_tree_on_chains(fjm, ctx):
    # (R join S) join (T join U) on seeded 4-chains of a few thousand rows
    fj, _ = fjm
    n = 0
    for qi in range(40):
        dq, _ = datagen.batch_query(datagen.seed_for(8, 50), qi, min_rows=200, max_rows=4_000,
                                    frac_chain=1.0, frac_star=0.0)
        if len(dq.atoms) < 4:
            continue
        tree = ((0, 1), (2, 3))
        for a in range(4, len(dq.atoms)):
            tree = (tree, a)
        _say("chain", qi, len(dq.atoms), tree)
        _check(fjm, ctx, dq, tree)
        n += 1
        if n == 4:
            break
    assert n == 4


def test_right_deep_triangle_and_stars(fjm, ctx):
    fj, _ = fjm
    from oracle import closed
    e = datagen.triangle_edges(datagen.seed_for(1, 0))
    dq = datagen.synth.triangle_query(e)
    got = _check(fjm, ctx, dq, (0, (1, 2)))          # the 2-paths S join T materialized first
    assert got["count"] == closed.cycle_count(e[0], e[1], 3)
    for qi in range(60):
        dq, _ = datagen.batch_query(datagen.seed_for(8, 51), qi, min_rows=100, max_rows=3_000,
                                    frac_chain=0.0, frac_star=1.0)
        m = len(dq.atoms)
        if m > 4:
            continue
        # the dimensions joined together first, then with the fact table
        tree = 1
        for a in range(2, m):
            tree = (tree, a)
        tree = (0, tree)
        _say("star", qi, m, tree)
        _check(fjm, ctx, dq, tree)
        break


def test_empty_intermediate_and_selections(fjm, ctx):
    dq = datagen.random_tiny_query(datagen.seed_for(8, 90), "chain4")
    for a in range(len(dq.atoms)):
        dq.filters[a] = None
    dq.filters[3] = (0, -(1 << 30))     # atom 3 keeps no row: P1 = [2, 3] is empty
    got = _check(fjm, ctx, dq, ((0, 1), (2, 3)))
    assert got["count"] == 0
    dq.filters[3] = (1, 3)              # a real selection under an intermediate
    _check(fjm, ctx, dq, ((0, 1), (2, 3)))
    _check(fjm, ctx, dq, (0, ((1, 2), 3)))


def test_wide_intermediate_is_refused(fjm, ctx):
    fj, runner = fjm
    # a star of six dimensions: an intermediate holding the fact table and
    # five dimensions has more variables than a relation has columns
    names = [f"v{i}" for i in range(12)]
    rels = [datagen.synth.Relation("F", [np.arange(4, dtype=np.int32)] * 6)]
    for i in range(6):
        rels.append(datagen.synth.Relation(f"D{i}", [np.arange(4, dtype=np.int32), np.arange(4, dtype=np.int32)]))
    atoms = [(0, tuple(range(6)))] + [(i + 1, (i, 6 + i)) for i in range(6)]
    dq = datagen.synth.make_query(names, rels, atoms)
    d = runner.DeviceQuery(ctx, dq)
    # the right child (0, ..., 5) holds the fact table's 6 variables and
    # five attributes: 11 > 8 columns for its materialized result
    tree = (6, (0, (1, (2, (3, (4, 5))))))
    with pytest.raises(fj.FJError):
        d.run_bushy(tree)
