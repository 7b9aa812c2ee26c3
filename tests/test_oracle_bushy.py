"""Pins of the oracle's bushy-plan decomposition (Section 2.2) and of its
evaluation, plus the library's host-side decomposition (no GPU needed)."""

import numpy as np
import pytest

import datagen
from oracle import brute
from oracle import bushy as B


def random_tree(atoms, rng):
    """A uniformly split binary tree over the given atoms (shuffled)."""
    atoms = list(atoms)
    rng.shuffle(atoms)

    def split(xs):
        if len(xs) == 1:
            return int(xs[0])
        k = int(rng.integers(1, len(xs)))
        return (split(xs[:k]), split(xs[k:]))

    return split(atoms)


def test_paper_example():
    # Section 2.2: (R join S) join (T join U) runs as P1 = [T, U], then
    # P2 = [R, S, P1]; R, S, T, U are atoms 0..3
    assert B.decompose(((0, 1), (2, 3))) == [[2, 3], [0, 1, -1]]


def test_left_deep_is_one_plan():
    assert B.decompose((((0, 1), 2), 3)) == [[0, 1, 2, 3]]
    assert B.decompose(0) == [[0]]


def test_right_deep_nests():
    # every right child that is a join is its own plan, innermost first
    assert B.decompose((0, (1, (2, 3)))) == [[2, 3], [1, -1], [0, -2]]
    steps = B.decompose(((0, (1, 2)), (3, 4)))
    assert steps == [[1, 2], [3, 4], [0, -1, -2]]


def test_every_atom_once_per_decomposition():
    rng = np.random.Generator(np.random.PCG64(11))
    for n in range(1, 8):
        for _ in range(20):
            t = random_tree(range(n), rng)
            steps = B.decompose(t)
            seen = [x for s in steps for x in s if x >= 0]
            assert sorted(seen) == list(range(n))
            # each intermediate is used exactly once, by a later plan
            used = [-x - 1 for s in steps for x in s if x < 0]
            assert sorted(used) == list(range(len(steps) - 1))
            for k, s in enumerate(steps):
                assert all(-x - 1 < k for x in s if x < 0)


@pytest.mark.parametrize("shape", ["triangle", "chain4", "star3", "cycle4", "clover"])
def test_bushy_result_is_the_query_result(shape):
    # whatever the tree, the result is the query's (plan invariance), checked
    # against nested-loop enumeration of the definition
    rng = np.random.Generator(np.random.PCG64(5))
    for rep in range(6):
        q = datagen.random_tiny_query(datagen.seed_for(7, rep), shape)
        want = sorted(brute.enumerate_result(q))
        t = random_tree(range(len(q.atoms)), rng)
        got = B.evaluate(q, t)
        assert got["count"] == len(want)
        assert sorted(map(tuple, got["rows"].tolist())) == want


def test_empty_intermediate():
    # a right subtree with no result: the whole plan is empty
    q = datagen.random_tiny_query(datagen.seed_for(7, 99), "chain4")
    for a in range(len(q.atoms)):
        q.filters[a] = None
    q.filters[3] = (0, -(1 << 30))   # atom 3 keeps no row
    got = B.evaluate(q, ((0, 1), (2, 3)))
    assert got["count"] == 0 == brute.count(q)


def test_library_decomposition_matches_oracle():
    from paper_2301_10841_amd import fj
    rng = np.random.Generator(np.random.PCG64(3))
    for n in range(1, 10):
        for _ in range(25):
            t = random_tree(range(n), rng)
            assert fj.bushy_decompose(t) == B.decompose(t)


def test_library_rejects_bad_trees():
    from paper_2301_10841_amd import fj
    for bad in [((0, 1), (1, 2))]:
        with pytest.raises(fj.FJError):
            fj.bushy_decompose(bad)
    b = fj.bushy(((0, 1), 2))
    b.root = 0   # nodes left outside the tree
    with pytest.raises(fj.FJError):
        fj.bushy_decompose(b)
