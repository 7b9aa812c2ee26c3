"""Write the oracle's triangle count of the full-scale R-MAT graph
(2^22 vertices, the first 50,000,000 distinct edges drawn with seed
seed_for(3, 1)) to ``rmat_s22_triangles.txt`` beside this script.

The count of Q(x,y,z) :- E(x,y), E(y,z), E(z,x) splits over disjoint sets of
x: every triangle is counted once, in the part holding its x.  Part p keeps
the R rows whose x is in the part, the S rows whose y such an R row reaches
and the T rows closing back into the part, which are exactly the rows the
part's triangles use.  Each part runs through the C oracle (Generic Join's
plan [[R(x),T(x)],[R(y),S(y)],[S(z),T(z)]], count only) in its own
process; the parts' counts are summed.  Only ``datagen`` and ``oracle``
are used.

    python tests/golden/make_rmat_triangles.py [--parts 64] [--procs 8]
"""

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from datagen import synth  # noqa: E402
from oracle import cfj  # noqa: E402

SCALE, EDGES = 22, 50_000_000
OUT = os.path.join(HERE, "rmat_s22_triangles.txt")
GJ = [[(0, (0,)), (2, (0,))], [(0, (1,)), (1, (1,))], [(1, (2,)), (2, (2,))]]

_E = None


def part_query(src, dst, parts, p):
    """The rows the triangles whose x lies in part p (x mod parts == p) use."""
    kr = (src % parts) == p
    reach = np.zeros(1 << SCALE, bool)
    reach[dst[kr]] = True
    ks = reach[src]
    kt = (dst % parts) == p
    rels = [synth.Relation("R", [src[kr], dst[kr]]), synth.Relation("S", [src[ks], dst[ks]]),
            synth.Relation("T", [src[kt], dst[kt]])]
    return synth.make_query(["x", "y", "z"], rels, [(0, (0, 1)), (1, (1, 2)), (2, (2, 0))])


def run_part(args):
    parts, p = args
    src, dst = _E
    t = time.perf_counter()
    q = part_query(src, dst, parts, p)
    n = cfj.run(q, GJ, materialize=False, counters=False)["count"]
    return p, n, time.perf_counter() - t


def main():
    global _E
    ap = argparse.ArgumentParser()
    ap.add_argument("--parts", type=int, default=64)
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    a = ap.parse_args()
    cfj.build(force=False)
    t0 = time.perf_counter()
    _E = datagen.rmat_edges(datagen.seed_for(3, 1), SCALE, EDGES)
    print(f"edges {_E[0].size} in {time.perf_counter() - t0:.0f}s", flush=True)
    total = 0
    with mp.get_context("fork").Pool(a.procs) as pool:
        for p, n, s in pool.imap_unordered(run_part, [(a.parts, p) for p in range(a.parts)]):
            total += n
            print(f"part {p}: {n} triangles in {s:.0f}s", flush=True)
    with open(OUT, "w") as f:
        f.write("# Triangles of the R-MAT graph: 2^22 vertices, (a,b,c,d) = (0.57,0.19,0.19,0.05),\n")
        f.write("# the first 50,000,000 distinct edges of seed seed_for(3, 1), self-loops dropped.\n")
        f.write(f"# Written by tests/golden/make_rmat_triangles.py: C oracle, Generic Join plan,\n")
        f.write(f"# {a.parts} parts of x (x mod {a.parts}), summed.\n")
        f.write(f"{total}\n")
    print(f"total {total} in {time.perf_counter() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
