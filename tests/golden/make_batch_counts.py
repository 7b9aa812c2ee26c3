"""Write the oracle's result count of every query of the batched workload
(the 256 queries of ``datagen.batch_mix(seed_for(4, 0))``: chains and stars
of 3-6 relations and triangles, 1K-2M rows per relation) to
``batch_seed4_counts.txt`` beside this script, one line per query:
``index kind count``.

Each query runs through the C oracle with the plan of its left-deep order
[0, 1, ..., m-1], converted and factored (Section 4.1), count only, in a
pool of processes.  Only ``datagen`` and ``oracle`` are used.

    python tests/golden/make_batch_counts.py [--queries 256] [--procs 8]
"""

import argparse
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import cfj  # noqa: E402
from oracle import plans as P  # noqa: E402

OUT = os.path.join(HERE, "batch_seed4_counts.txt")
SEED = datagen.seed_for(4, 0)


def count_query(i):
    t = time.perf_counter()
    q, _ = datagen.batch_query(SEED, i)
    plan = P.factor(P.binary2fj(q, list(range(len(q.atoms)))))
    n = cfj.run(q, plan, materialize=False, counters=False)["count"]
    return i, q.kind, n, time.perf_counter() - t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--queries", type=int, default=256)
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    a = ap.parse_args()
    cfj.build(force=False)
    rows = {}
    with mp.get_context("fork").Pool(a.procs) as pool:
        for i, kind, n, s in pool.imap_unordered(count_query, range(a.queries)):
            rows[i] = (kind, n)
            print(f"query {i} ({kind}): {n} in {s:.1f}s", flush=True)
    with open(OUT, "w") as f:
        f.write("# Result counts of the batched workload's queries (datagen.batch_query(seed_for(4, 0), i)),\n")
        f.write("# C oracle, left-deep order [0..m-1] converted and factored, count only.\n")
        f.write("# Written by tests/golden/make_batch_counts.py.  Columns: index kind count\n")
        for i in sorted(rows):
            f.write(f"{i} {rows[i][0]} {rows[i][1]}\n")


if __name__ == "__main__":
    main()
