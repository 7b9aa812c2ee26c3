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
