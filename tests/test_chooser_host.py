"""Host-side checks of the plan chooser's C-ABI (no GPU needed): the greedy
left-deep order equals the oracle's, and every candidate plan equals the
oracle's conversion of the same order (binary candidates: Section 4.1
conversion then factoring) or its Generic Join plan (Section 3.2)."""

import math

import numpy as np
import pytest

import datagen
from datagen import synth
from oracle import plans as P
from oracle import stats as S
from paper_2301_10841_amd import fj


def shape_query(shape):
    """A query of the batched workload's shapes (relation contents unused)."""
    z = lambda k: synth.Relation("R", [np.zeros(1, np.int32)] * k)
    if shape.startswith("chain"):
        m = int(shape[5:])
        return synth.make_query([f"x{i}" for i in range(m + 1)], [z(2) for _ in range(m)],
                                  [(i, (i, i + 1)) for i in range(m)])
    if shape.startswith("star"):
        m = int(shape[4:])
        d = m - 1
        rels = [z(d)] + [z(2) for _ in range(d)]
        return synth.make_query([f"k{i}" for i in range(d)] + [f"a{i}" for i in range(d)], rels,
                                  [(0, tuple(range(d)))] + [(i + 1, (i, d + i)) for i in range(d)])
    return datagen.random_tiny_query(1, shape, max_rows=3)


SHAPES = ["triangle", "chain3", "chain4", "chain6", "star3", "star4", "star6", "cycle4", "clover"]


def random_sketches(rng, dq):
    out = []
    for _, vs in dq.atoms:
        rows = int(math.exp(rng.uniform(0, math.log(2_000_000))))
        dist = [int(rng.integers(1, rows + 1)) for _ in vs]
        top = [sorted(rng.integers(1, max(2, rows // 4), size=8).tolist(), reverse=True) for _ in vs]
        out.append({"rows": rows, "distinct": dist, "top": top})
    return out


def to_c(sks):
    res = []
    for sk in sks:
        s = fj.Sketch()
        s.rows = sk["rows"]
        s.ncols = len(sk["distinct"])
        for j, d in enumerate(sk["distinct"]):
            s.distinct[j] = d
            for k, t in enumerate(sk["top"][j]):
                s.top[j][k] = t
        res.append(s)
    return res


def fjq(dq):
    return fj.make_query([vs for _, vs in dq.atoms], dq.nvars, dq.head)


def atoms_of(dq):
    return [vs for _, vs in dq.atoms]


@pytest.mark.parametrize("shape", SHAPES)
def test_greedy_order_matches_oracle(shape):
    dq = shape_query(shape)
    rng = np.random.default_rng(abs(hash(shape)) % (1 << 32))
    for _ in range(25):
        sks = random_sketches(rng, dq)
        for first in range(-1, len(dq.atoms)):
            want = S.greedy_order(atoms_of(dq), sks, first)
            assert fj.greedy_order(fjq(dq), to_c(sks), first) == want


def test_greedy_order_hand_examples():
    mk = lambda rows, d: {"rows": rows, "distinct": d, "top": [[0] * 8 for _ in d]}
    dq = shape_query("star3")   # F(k0,k1), D0(k0,a0), D1(k1,a1)
    sks = [mk(10000, [100, 1000]), mk(100, [100, 100]), mk(500, [500, 500])]
    assert fj.greedy_order(fjq(dq), to_c(sks)) == [0, 2, 1]


def var_order_of(dq, order):
    vo = []
    for a in order:
        for v in dq.atoms[a][1]:
            if v not in vo:
                vo.append(v)
    return vo


@pytest.mark.parametrize("shape", SHAPES)
def test_candidates_match_oracle_plans(shape):
    dq = shape_query(shape)
    rng = np.random.default_rng(7 + len(shape))
    for _ in range(10):
        sks = random_sketches(rng, dq)
        cands, feat = fj.plan_candidates(fjq(dq), to_c(sks))
        assert feat.shape == (len(cands), fj.FEATURES) and np.all(np.isfinite(feat))
        keys = [c.key() for c in cands]
        assert len(set(keys)) == len(keys), "duplicate candidates"
        # candidate 0: the plain plan, the greedy order from the largest atom
        assert keys[0] == (fj.CAND_BINARY, tuple(S.greedy_order(atoms_of(dq), sks)))
        binaries = [k for k in keys if k[0] == fj.CAND_BINARY]
        # every start atom's greedy order is there (deduplicated)
        want_orders = []
        for first in [-1] + list(range(len(dq.atoms))):
            o = tuple(S.greedy_order(atoms_of(dq), sks, first))
            if o not in want_orders:
                want_orders.append(o)
        assert [k[1] for k in binaries] == want_orders
        want_gj = []
        for o in want_orders:
            vo = tuple(var_order_of(dq, o))
            if vo not in want_gj and len(vo) <= fj.MAX_NODES:
                want_gj.append(vo)
        assert [k[1] for k in keys if k[0] == fj.CAND_GJ] == want_gj
        for c, f in zip(cands, feat):
            kind, order = c.key()
            got = fj.candidate_plan(fjq(dq), c).nodes()
            if kind == fj.CAND_BINARY:
                want = P.factor(P.binary2fj(dq, order))
            else:
                want = P.gj_plan(dq, order)
            assert got == [[(a, tuple(vs)) for a, vs in node] for node in want]
            # directly defined features: the kind flags, the node count and
            # the rows of the first atom in plan order
            assert f[0] == (kind == fj.CAND_BINARY) and f[1] == (kind == fj.CAND_GJ)
            assert f[2] == pytest.approx(len(want) / 16)
            a0 = want[0][0][0]
            assert f[16] == 1.0
            assert f[17] == pytest.approx(math.log2(1 + sks[a0]["rows"]) / 32, rel=1e-6)


def test_candidate_cap_and_errors():
    dq = shape_query("star6")
    sks = random_sketches(np.random.default_rng(1), dq)
    cands, feat = fj.plan_candidates(fjq(dq), to_c(sks), cap=3)
    assert len(cands) == 3 and feat.shape == (3, fj.FEATURES)
    bad = to_c(sks)
    bad[0].ncols = 1
    with pytest.raises(fj.FJError) as e:
        fj.plan_candidates(fjq(dq), bad)
    assert e.value.status == -1
    with pytest.raises(fj.FJError):
        fj.greedy_order(fjq(dq), to_c(sks), first=99)
