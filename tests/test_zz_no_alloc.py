"""The allocation-free selection entry point (fj_filter_lt_noalloc) through
the C-ABI against fj_filter_lt on the same inputs: offsets in row order and
counts equal, on calls in a row whose inputs shrink (the fixed scratch
array keeps the last call's contents), up to the stated row limit."""

import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LIMIT = 65536 * 1024


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10841_amd import fj
    ctx = fj.Context(0)
    yield torch, fj, ctx
    ctx.close()


def _noalloc(fj, ctx, col, bound, out):
    n = C.c_int64(-1)
    st = fj.lib().fj_filter_lt_noalloc(ctx.h, C.c_void_p(col.data_ptr()), int(col.shape[0]), int(bound),
                                       C.c_void_p(out.data_ptr()), C.byref(n))
    return st, int(n.value)


def _check(torch, fj, ctx, col, bound):
    print("rows", int(col.shape[0]), "bound", bound, flush=True)
    want, nw = ctx.filter_lt(col, bound)
    out = torch.full((max(int(col.shape[0]), 1),), -7, dtype=torch.int32, device=col.device)
    st, n = _noalloc(fj, ctx, col, bound, out)
    assert st == 0
    assert n == nw
    assert torch.equal(out[:n], want[:n])
    # the definition: the rows with col < bound, in row order
    ref = torch.nonzero(col < bound).flatten().to(torch.int32)
    assert torch.equal(out[:n], ref)
    assert bool((out[n:] == -7).all())


def test_noalloc_matches_filter_shrinking_inputs(env):
    torch, fj, ctx = env
    g = torch.Generator(device="cuda:0").manual_seed(1234)
    big = torch.randint(0, 100, (LIMIT,), generator=g, dtype=torch.int32, device="cuda:0")
    _check(torch, fj, ctx, big, 10)           # the largest input allowed
    _check(torch, fj, ctx, big[:3_000_001], 37)   # then a smaller one (ragged tail)
    _check(torch, fj, ctx, big[5:1029], 50)   # a misaligned start, one block
    _check(torch, fj, ctx, big[:1], 100)
    st, n = _noalloc(fj, ctx, big[:0], 10, big)
    assert (st, n) == (0, 0)


def test_noalloc_refuses_rows_above_limit(env):
    torch, fj, ctx = env
    col = torch.zeros(LIMIT + 1, dtype=torch.int32, device="cuda:0")
    out = torch.empty(1, dtype=torch.int32, device="cuda:0")
    st, n = _noalloc(fj, ctx, col, 1, out)
    assert st == -6 and n == 0   # FJ_ERR_UNSUPPORTED, before any device work
    assert b"allocation-free limit" in fj.lib().fj_last_error()
