"""The scripts that write stored expected values, checked at small sizes
against what they must equal: the R-MAT triangle count summed over parts
of x equals trace(A^3) of the whole graph."""

import os
import sys

import pytest

import datagen
from oracle import cfj, closed

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_rmat_triangles as MT  # noqa: E402


@pytest.mark.parametrize("parts", [1, 3, 8])
def test_triangle_parts_sum_to_trace(parts):
    src, dst = datagen.rmat_edges(datagen.seed_for(3, 7), 10, 6000)
    total = 0
    for p in range(parts):
        q = MT.part_query(src, dst, parts, p)
        total += cfj.run(q, MT.GJ, materialize=False, counters=False)["count"]
    assert total == closed.cycle_count(src, dst, 3) > 0


def test_golden_file_is_a_count():
    lines = [ln for ln in open(MT.OUT) if ln.strip() and not ln.startswith("#")]
    assert len(lines) == 1 and int(lines[0]) > 0


@pytest.mark.parametrize("scale,block", [(8, 16), (10, 1000), (11, 1 << 11)])
def test_blocked_trace4_equals_whole(scale, block):
    # the row-blocked trace(A^4) of the 4-cycle golden equals the unblocked
    # closed form, whatever the block size (ragged last block included)
    src, dst = datagen.rmat_edges(datagen.seed_for(3, 5), scale, 12 * (1 << scale))
    assert closed.cycle4_count_blocked(src, dst, block) == closed.cycle_count(src, dst, 4) > 0


def test_blocked_trace4_brute_force():
    # closed 4-walks on a tiny graph, enumerated
    import numpy as np
    rng = np.random.default_rng(3)
    e = {(int(a), int(b)) for a, b in rng.integers(0, 7, (30, 2)) if a != b}
    src = np.array([a for a, _ in e], np.int32)
    dst = np.array([b for _, b in e], np.int32)
    adj = {}
    for a, b in e:
        adj.setdefault(a, []).append(b)
    walks = 0
    for w in range(7):
        for x in adj.get(w, []):
            for y in adj.get(x, []):
                for z in adj.get(y, []):
                    walks += w in adj.get(z, [])
    assert closed.cycle4_count_blocked(src, dst, 3) == walks
