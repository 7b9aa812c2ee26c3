"""CPU oracle for the Free Join executor -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or run anything in this package.  The
product path (``paper_2301_10841_amd``) never does, and shares no code with it:
the two meet only at the seeded inputs drawn by ``datagen``.

Tiers
-----
* ``plans``   -- the plan pipeline written from the paper: binary-to-Free-Join
  conversion (Section 4.1 figure "bj2fj"), conservative factoring (Section 4.1
  figure "factorize-plan"), validity and covers (Section 3.2 definitions),
  GHT/COLT schemas (Section 3.3 build phase), Generic Join plans (Section 3.2,
  equation "gj-plan").
* ``brute``   -- the definition of a full conjunctive query over bags
  (Section 2.1, equation "cq"): every combination of one row per atom that
  agrees on shared variables, by nested loops.  Tiny inputs only.
* ``closed``  -- closed forms that hold for any instance: trace identities for
  cycles, matrix products for chains, degree products for stars.
* ``fj_oracle.c`` (via ``cfj``) -- a plain C Free Join following Section 3.3
  (figure "fj-algo"), COLT (Section 4.2 figure "colt-impl"), vectorized
  batches (Section 4.3) and dynamic covers (Section 4.4), with work counters.
* ``bushy``   -- bushy binary plans run as a series of left-deep plans with
  materialized intermediates (Section 2.2), each plan through ``plans`` and
  ``cfj``; pinned by the paper's decomposition example and by nested-loop
  enumeration of the query result.

* ``stats``   -- per-relation sketches (row count, distinct counts, top-k
  frequencies) and the greedy left-deep order of the plain baseline plan.
* ``mlp``     -- a float64 perceptron (forward, backward, Adam) that the
  learned plan chooser's kernels are checked against.

Pins: see ``tests/test_oracle_*.py``.  The join tiers are pinned by the
paper's worked plans, brute force, closed forms, the clover instance's probe
counts and its Section 4.2 extension's forced tries, and Generic Join's
triangle counters derived from vertex degrees.  ``mlp`` is pinned by a
hand-worked forward and backward pass, central finite differences, the
all-active ReLU closed form and the closed form of Adam's first two steps;
``stats`` by hand-counted sketches and hand-worked greedy orders.  Parity
unpinned: the chooser's estimate features (this library's own definition;
they change speed, never results).
"""
