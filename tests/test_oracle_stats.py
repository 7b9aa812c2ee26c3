"""Pins of the statistics oracle (oracle/stats.py): a sketch counted by hand
and greedy orders worked out by hand from the textbook estimate."""

from oracle import stats as S


def test_column_sketch_by_hand():
    sk = S.column_sketch([5, 5, 5, 2, 2, 9, -1])
    assert sk["distinct"] == 4
    assert sk["top"] == [3, 2, 1, 1, 0, 0, 0, 0]
    assert S.column_sketch([])["distinct"] == 0


def test_sketch_with_selection():
    sk = S.sketch([[1, 1, 2, 3], [7, 7, 7, 7]], sel=[0, 1, 3])
    assert sk["rows"] == 3 and sk["distinct"] == [2, 1] and sk["top"][1][0] == 3


def mk(rows, distinct):
    return {"rows": rows, "distinct": distinct, "top": [[0] * 8 for _ in distinct]}


def test_greedy_chain_by_hand():
    # R0(x0,x1) 1000 rows, R1(x1,x2) 100, R2(x2,x3) 10.  Start at R0 (largest).
    # R1 is the only connected atom: est 1000 * 100 / max(10, 100) = 1000.
    # Then R2: V(J,x2) = 50, est 1000 * 10 / max(50, 10) = 200.
    atoms = [(0, 1), (1, 2), (2, 3)]
    sks = [mk(1000, [1000, 10]), mk(100, [100, 50]), mk(10, [10, 10])]
    assert S.greedy_order(atoms, sks) == [0, 1, 2]
    # from R2: R1 next (est 10 * 100 / max(10, 50) = 20), then R0
    assert S.greedy_order(atoms, sks, first=2) == [2, 1, 0]


def test_greedy_star_prefers_the_more_selective_dimension():
    # F(k1,k2) 10000 rows (V 100, 1000); D1(k1,a) 100 rows (V 100, 100);
    # D2(k2,b) 500 rows (V 500, 500).
    # est D1 = 10000 * 100 / max(100, 100) = 10000
    # est D2 = 10000 * 500 / max(1000, 500) = 5000  -> D2 first
    atoms = [(0, 1), (0, 2), (1, 3)]
    sks = [mk(10000, [100, 1000]), mk(100, [100, 100]), mk(500, [500, 500])]
    assert S.greedy_order(atoms, sks) == [0, 2, 1]


def test_greedy_ties_and_disconnected():
    # equal estimates go to the lower atom index
    atoms = [(0, 1), (0,), (1,)]
    sks = [mk(100, [10, 10]), mk(10, [10]), mk(10, [10])]
    assert S.greedy_order(atoms, sks) == [0, 1, 2]
    # R0(x) shares nothing with R1(y), R2(y): start at the largest (R2), then
    # the connected R1, then R0; from R0 nothing is connected, so the
    # smallest (R1) comes next
    atoms = [(0,), (1,), (1,)]
    sks = [mk(5, [5]), mk(3, [3]), mk(7, [7])]
    assert S.greedy_order(atoms, sks) == [2, 1, 0]
    assert S.greedy_order(atoms, sks, first=0) == [0, 1, 2]
    # largest-rows tie goes to the lower index
    sks = [mk(7, [5]), mk(3, [3]), mk(7, [7])]
    assert S.greedy_order(atoms, sks)[0] == 0
