"""Write trace(A^4), the directed 4-cycle count Q(w,x,y,z) :- E(w,x),
E(x,y), E(y,z), E(z,w), of the reduced-scale R-MAT graphs (2^S vertices,
round(11.92 * 2^S) distinct edges, the full-scale graph's edges per vertex,
seed seed_for(3, 1)) to ``rmat_cycle4_counts.txt`` beside this script, one
line per scale: ``S edges count``.  The count is the closed form of
``oracle.closed`` computed in row blocks (A^2 is too large to hold at once
beyond S = 16).  Only ``datagen`` and ``oracle`` are used.

    python tests/golden/make_rmat_cycle4.py [16 18 20]
"""

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import closed  # noqa: E402

OUT = os.path.join(HERE, "rmat_cycle4_counts.txt")


def edges_for(scale):
    return int(round(11.92 * (1 << scale)))


def main():
    scales = [int(a) for a in sys.argv[1:]] or [16, 18, 20]
    lines = []
    for S in scales:
        t = time.perf_counter()
        src, dst = datagen.rmat_edges(datagen.seed_for(3, 1), S, edges_for(S))
        n = closed.cycle4_count_blocked(src, dst, 1 << max(10, S - 8))
        print(f"scale {S}: {src.size} edges, {n} 4-cycles in {time.perf_counter() - t:.0f}s", flush=True)
        lines.append(f"{S} {src.size} {n}\n")
    with open(OUT, "w") as f:
        f.write("# trace(A^4) of R-MAT graphs: 2^S vertices, (a,b,c,d) = (0.57,0.19,0.19,0.05),\n")
        f.write("# round(11.92 * 2^S) distinct edges of seed seed_for(3, 1), self-loops dropped.\n")
        f.write("# Written by tests/golden/make_rmat_cycle4.py.  Columns: S edges count\n")
        f.writelines(lines)


if __name__ == "__main__":
    main()
