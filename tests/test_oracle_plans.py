"""Pins of the oracle's plan pipeline against the paper's worked examples."""

import os

import pytest

import datagen
from oracle import plans as P
from tests.plan_text import atom_index, load_golden, parse_plan, plan_str, subatom_str

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_plans.txt")
CASES = load_golden(GOLDEN)


def _query(shape):
    return datagen.random_tiny_query(1, shape, max_rows=3)


def _order(q, arg):
    return [atom_index(q, n) for n in arg.split(",")]


def _vars(q, arg):
    return [q.var_names.index(v) for v in arg.split(",")]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{i}" for i, c in enumerate(CASES)])
def test_paper_example(case):
    shape, op, arg, expected = case
    q = _query(shape)
    if op == "binary2fj":
        assert plan_str(q, P.binary2fj(q, _order(q, arg))) == expected
    elif op == "factor_binary":
        assert plan_str(q, P.factor(P.binary2fj(q, _order(q, arg)))) == expected
    elif op == "gj":
        assert plan_str(q, P.gj_plan(q, _vars(q, arg))) == expected
    elif op in ("covers_binary", "covers_gj"):
        plan = P.binary2fj(q, _order(q, arg)) if op == "covers_binary" else P.gj_plan(q, _vars(q, arg))
        got = ";".join(",".join(subatom_str(q, plan[k][i]) for i in P.covers(plan, k))
                       for k in range(len(plan)))
        assert got == expected
    elif op in ("schemas_binary", "schemas_explicit"):
        plan = P.binary2fj(q, _order(q, arg)) if op == "schemas_binary" else parse_plan(q, arg)
        sch = P.schemas(q, plan)
        got = ";".join(
            f"{q.relations[q.atoms[a][0]].name}=[" + ",".join("[" + ",".join(q.var_names[v] for v in lv) + "]" for lv in sch[a]) + "]"
            for a in range(len(q.atoms)))
        assert got == expected
    elif op == "invalid":
        with pytest.raises(P.PlanError):
            P.validate(q, parse_plan(q, arg))
    elif op == "valid":
        P.validate(q, parse_plan(q, arg))
    else:
        raise AssertionError(op)


def test_binary2fj_triangle_keeps_empty_remainder():
    # reading of figure bj2fj: T's remainder after probing T(z,x) is T()
    q = _query("triangle")
    assert plan_str(q, P.binary2fj(q, [0, 1, 2])) == "[[R(x,y),S(y)],[S(z),T(z,x)],[T()]]"


def test_factor_star_hoists_every_lookup():
    q = datagen.star_schema(3, n_fact=10, n_dim=5)
    got = plan_str(q, P.factor(P.binary2fj(q, [0, 1, 2, 3, 4])))
    assert got == "[[F(k1,k2,k3,k4),D1(k1),D2(k2),D3(k3),D4(k4)],[D1(a1)],[D2(a2)],[D3(a3)],[D4(a4)]]"


def test_pure_covers_and_root_rule():
    q = _query("triangle")
    conv = P.binary2fj(q, [0, 1, 2])
    # node 1 [S(z),T(z,x)]: T(z,x) is a cover but binds x again; only S(z) is pure
    assert P.covers(conv, 1) == [0, 1]
    assert P.pure_covers(conv, 1) == [0]
    # R is iterated directly; S and T roots are probed and therefore built
    assert [P.root_is_built(q, conv, a) for a in range(3)] == [False, True, True]
    gj = P.gj_plan(q, [0, 1, 2])
    assert [P.root_is_built(q, gj, a) for a in range(3)] == [True, True, True]


def test_plans_from_all_orders_are_valid():
    for shape in ("triangle", "clover", "chain4", "star3", "cycle4", "clover_u", "pair"):
        q = _query(shape)
        import itertools
        for order in itertools.permutations(range(len(q.atoms))):
            for plan in (P.binary2fj(q, order), P.factor(P.binary2fj(q, order))):
                P.validate(q, plan)
