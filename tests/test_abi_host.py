"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function declared in include/fj.h, and its plan pipeline matches the
oracle's and the paper's worked examples."""

import ctypes
import itertools
import os
import re

import pytest

import datagen
from oracle import plans as P
from paper_2301_10841_amd import fj
from tests.plan_text import atom_index, load_golden, plan_str

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fj.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fj_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fj.lib()
    names = declared_functions()
    assert "fj_execute" in names and "fj_build_colt" in names and "fj_plan_from_binary" in names
    for n in names:
        assert hasattr(lib, n), n


def _fjq(dq):
    return fj.make_query([vs for _, vs in dq.atoms], dq.nvars, dq.head)


SHAPES = ["triangle", "clover", "chain3", "chain4", "star3", "cycle4", "clover_u", "pair"]


@pytest.mark.parametrize("shape", SHAPES)
def test_plan_pipeline_matches_oracle(shape):
    dq = datagen.random_tiny_query(3, shape, max_rows=3)
    q = _fjq(dq)
    for order in itertools.permutations(range(len(dq.atoms))):
        for factor in (False, True):
            want = P.binary2fj(dq, order)
            if factor:
                want = P.factor(want)
            got = fj.plan_from_binary(q, order, factor).nodes()
            assert got == [[(a, tuple(vs)) for a, vs in node] for node in want]


def test_plan_examples_from_paper():
    golden = load_golden(os.path.join(ROOT, "tests", "golden", "paper_plans.txt"))
    for shape, op, arg, expected in golden:
        if op not in ("binary2fj", "factor_binary"):
            continue
        dq = datagen.random_tiny_query(1, shape, max_rows=3)
        order = [atom_index(dq, n) for n in arg.split(",")]
        plan = fj.plan_from_binary(_fjq(dq), order, op == "factor_binary").nodes()
        assert plan_str(dq, plan) == expected


def test_invalid_plans_are_refused():
    dq = datagen.random_tiny_query(1, "clover", max_rows=3)
    q = _fjq(dq)
    # Section 3.2: one node with all three atoms is invalid
    with pytest.raises(fj.FJError) as e:
        fj.plan_from_nodes(q, [[(0, (0, 1)), (1, (0, 2)), (2, (0, 3))]])
    assert e.value.status == -2
    # not a partition: atom 0 misses variable a
    with pytest.raises(fj.FJError) as e:
        fj.plan_from_nodes(q, [[(0, (0,)), (1, (0,)), (2, (0,))], [(1, (2,))], [(2, (3,))]])
    assert e.value.status == -2
    # an atom twice in a node (validity (a))
    with pytest.raises(fj.FJError) as e:
        fj.plan_from_nodes(q, [[(0, (0,)), (0, (1,))], [(1, (0, 2))], [(2, (0, 3))]])
    assert e.value.status == -2
    # the only cover of node 1 rebinds x: T(z,x) after x is bound
    tq = datagen.random_tiny_query(1, "triangle", max_rows=3)
    with pytest.raises(fj.FJError) as e:
        fj.plan_from_nodes(_fjq(tq), [[(0, (0, 1)), (1, (1,))], [(2, (2, 0))], [(1, (2,))]])
    assert e.value.status == -3
    # the GJ plan is accepted
    gj = fj.plan_from_nodes(q, [[(0, (0,)), (1, (0,)), (2, (0,))], [(0, (1,))], [(1, (2,))], [(2, (3,))]])
    assert len(gj.nodes()) == 4


def test_bad_query_and_order():
    dq = datagen.random_tiny_query(1, "triangle", max_rows=3)
    q = _fjq(dq)
    with pytest.raises(fj.FJError):
        fj.plan_from_binary(q, [0, 1], True)
    with pytest.raises(fj.FJError):
        fj.plan_from_binary(q, [0, 0, 1], True)
    bad = fj.make_query([(0, 0)], 1)  # repeated variable in an atom
    with pytest.raises(fj.FJError):
        fj.plan_from_binary(bad, [0], True)


def test_context_without_gpu_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = fj.lib().fj_ctx_create(0, None, None, ctypes.byref(h))
    assert st in (-1, -5)


def test_factorized_entry_points_refuse_null_arguments():
    # argument checks happen before any device call
    L = fj.lib()
    out = ctypes.c_void_p(123)
    cnt = ctypes.c_uint64(7)
    st = L.fj_execute_factorized(None, None, None, None, ctypes.byref(out), ctypes.byref(cnt), None)
    assert st == -1 and out.value is None
    assert L.fj_execute_factorized(None, None, None, None, None, None, None) == -1
    wr = ctypes.c_uint64(5)
    assert L.fj_result_expand(None, None, 0, None, 0, ctypes.byref(wr)) == -1
    assert wr.value == 5 or wr.value == 0
    L.fj_result_free(None)   # a no-op
