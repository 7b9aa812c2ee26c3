"""GPU parity of the learned plan chooser's kernels, through the C-ABI:
column sketches equal the oracle's exactly; the perceptron's forward pass,
gradient and Adam step match the FP64 oracle (oracle/mlp.py) within the
stated tolerances; every candidate plan of a query gives the oracle's result
(the plan never changes the answer); the choice falls back to the plain
converted plan when told to."""

import math

import numpy as np
import pytest

import datagen
from oracle import mlp as OM
from oracle import stats as OS
from tests.gpu_util import assert_same_rows, oracle_run

pytestmark = pytest.mark.gpu

# FP32 kernels against the FP64 oracle.  Each output is a sum of at most
# max(in_dim, hidden, batch) <= 512 products of O(1) terms, so its float32
# rounding error is far below 1e-4 of the tensor's largest magnitude.
TOL = 1e-4


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10841_amd import fj, runner
    ctx = fj.Context(0)
    yield fj, runner, ctx, torch
    ctx.close()


def _close(got, want, tol=TOL):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = max(1e-30, float(np.max(np.abs(want))) if want.size else 1.0)
    err = float(np.max(np.abs(got - want))) if want.size else 0.0
    assert err <= tol * scale, (err, scale)


def _columns():
    rng = np.random.default_rng(11)
    perm = rng.permutation(50_000).astype(np.int64)
    yield "uniform", rng.integers(0, 1000, 100_000).astype(np.int32), None
    yield "zipf1.5", datagen.zipf_keys(rng, 300_000, 50_000, 1.5, perm), None
    yield "minus_one", np.where(rng.random(70_000) < 0.3, -1, rng.integers(-5, 5, 70_000)).astype(np.int32), None
    yield "constant", np.full(4097, 7, np.int32), None
    yield "distinct", rng.permutation(65_536).astype(np.int32), None
    yield "one_row", np.array([123], np.int32), None
    yield "empty", np.zeros(0, np.int32), None
    col = rng.integers(0, 50, 20_000).astype(np.int32)
    yield "selected", col, np.flatnonzero(rng.random(20_000) < 0.2).astype(np.uint32)
    yield "extremes", np.array([2**31 - 1, -2**31, -1, 0, -1, 2**31 - 1] * 999, np.int32), None


@pytest.mark.parametrize("case", [c[0] for c in _columns()])
def test_sketch_matches_oracle(env, case):
    fj, _, ctx, torch = env
    name, col, sel = next(c for c in _columns() if c[0] == case)
    other = np.arange(col.size, dtype=np.int32) % 3
    dcols = [torch.from_numpy(col).cuda(), torch.from_numpy(other).cuda()]
    dsel = torch.from_numpy(sel.astype(np.int32)).cuda() if sel is not None else None
    sk = ctx.sketch(dcols, dsel, sel.size if sel is not None else 0).as_dict()
    want = OS.sketch([col, other], sel)
    assert sk == want


def _mlp_case(fj, ctx, torch, d, h, b, seed):
    rng = np.random.default_rng(seed)
    p = OM.init_params(rng, d, h) + rng.normal(0, 0.05, OM.param_count(d, h))
    x = rng.uniform(0, 1, (b, d))
    t = rng.normal(0, 1, b)
    m = fj.Mlp(ctx, d, h)
    assert m.n == OM.param_count(d, h)
    m.set_params(p.astype(np.float32))
    p32 = p.astype(np.float32).astype(np.float64)  # what the GPU holds
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    x32 = x.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    return m, p32, xd, td, x32, t32


@pytest.mark.parametrize("d,h,b", [(128, 128, 256), (128, 128, 1), (17, 33, 70), (5, 128, 513)])
def test_mlp_forward_and_gradient_match_oracle(env, d, h, b):
    fj, _, ctx, torch = env
    m, p, xd, td, x, t = _mlp_case(fj, ctx, torch, d, h, b, seed=d * 1000 + b)
    y = m.forward(xd).cpu().numpy()
    want_y, _ = OM.forward(p, x, d, h)
    _close(y, want_y)
    g, loss = m.gradient(xd, td)
    want_g, want_loss = OM.gradient(p, x, t, d, h)
    assert abs(loss - want_loss) <= TOL * max(1.0, want_loss)
    for got_part, want_part in zip(OM.unpack(g, d, h), OM.unpack(want_g, d, h)):
        _close(got_part, want_part)
    # the parameters come back unchanged
    assert np.array_equal(m.get_params(), p.astype(np.float32))
    m.free()


def test_adam_steps_match_oracle(env):
    fj, _, ctx, torch = env
    d, h, b = 128, 128, 64
    m, p, xd, td, x, t = _mlp_case(fj, ctx, torch, d, h, b, seed=3)
    mom = np.zeros_like(p)
    vel = np.zeros_like(p)
    lr = 1e-3
    for step in (1, 2, 3):
        g, _ = m.gradient(xd, td)          # the GPU's own gradient at the current point
        loss = m.train_step(xd, td, lr, want_loss=True)
        p, mom, vel = OM.adam_step(p, g.astype(np.float64), mom, vel, step, lr)
        got = m.get_params().astype(np.float64)
        # float32 parameter update: |error| <= a few ulps of the parameter
        # plus float32 rounding of the step (<= 1e-5 lr)
        assert np.max(np.abs(got - p) - (4 * np.finfo(np.float32).eps * np.abs(p) + 1e-5 * lr)) <= 0, step
        p = got
        assert math.isfinite(loss)
    m.free()


def test_training_reduces_loss(env):
    fj, _, ctx, torch = env
    rng = np.random.default_rng(9)
    d, h, n = 128, 128, 4096
    x = rng.uniform(0, 1, (n, d)).astype(np.float32)
    w = rng.normal(0, 1, d)
    t = (2.0 * (x - 0.5) @ w / math.sqrt(d) + 0.5 * np.sin(3.0 * x[:, 0])).astype(np.float32)
    m = fj.Mlp(ctx, d, h)
    m.set_params(OM.init_params(rng, d, h).astype(np.float32))
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    _, l0 = m.gradient(xd, td)
    for epoch in range(30):
        perm = torch.randperm(n, device="cuda")
        for i in range(0, n, 256):
            idx = perm[i:i + 256]
            m.train_step(xd[idx].contiguous(), td[idx].contiguous(), 1e-3)
    _, l1 = m.gradient(xd, td)
    assert l1 < 0.2 * l0, (l0, l1)
    m.free()


def _small_mix():
    qs, _ = datagen.batch_mix(23, n_queries=12, max_rows=20_000)
    qs.append(datagen.synth.triangle_query(datagen.triangle_edges(datagen.seed_for(1, 0))))
    qs.append(datagen.star_schema(5, n_fact=100_000, n_dim=10_000))
    return qs


def test_every_candidate_plan_gives_the_oracle_result(env):
    fj, runner, ctx, torch = env
    for qi, dq in enumerate(_small_mix()):
        d = runner.DeviceQuery(ctx, dq)
        sks = d.sketches()
        cands, feat = d.candidates(sks)
        assert feat.shape[0] == len(cands) >= 1
        want = None
        for c in cands:
            plan = d.candidate_plan(c)
            got = d.run(plan, materialize=True)
            for t in got["colts"]:
                t.free()
            if want is None:
                w = oracle_run(dq, plan.nodes(), materialize=True, counters=False)
                want = (w["count"], w["rows"])
            assert got["count"] == want[0], (qi, c.key())
            assert_same_rows(got["rows"], want[1])


def test_choice_and_fallback(env):
    fj, runner, ctx, torch = env
    dq = _small_mix()[0]
    d = runner.DeviceQuery(ctx, dq)
    sks = d.sketches()
    cands, _ = d.candidates(sks)
    plain = fj.plan_from_binary(d.q, list(cands[0].order)[:cands[0].n], True)
    # no model: the plain converted plan
    p, k, _ = d.choose(None, sks)
    assert k == 0 and p.nodes() == plain.nodes()
    m = fj.Mlp(ctx)
    m.set_params(OM.init_params(np.random.default_rng(1), fj.FEATURES, 128).astype(np.float32))
    p, k, scores = d.choose(m, sks)
    assert 0 <= k < len(cands)
    assert p.nodes() == d.candidate_plan(cands[k]).nodes()
    # the scores are the perceptron's outputs on the candidates' features
    _, feat = d.candidates(sks)
    y = m.forward(torch.from_numpy(feat).cuda()).cpu().numpy()
    assert np.allclose(scores[:len(cands)], y, rtol=1e-6, atol=1e-6)
    # a margin no prediction can reach keeps the plain plan
    p, k, _ = d.choose(m, sks, margin=1e30)
    assert k == 0 and p.nodes() == plain.nodes()
    # a query below the row gate gets the plain plan unscored; at the gate
    # it is scored as without one
    rows = sum(int(s.rows) for s in sks)
    p, k, _ = d.choose(m, sks, gate_rows=rows + 1)
    assert k == 0 and p.nodes() == plain.nodes()
    p, k2, _ = d.choose(m, sks, gate_rows=rows)
    assert scores[k2] == min(scores[:len(cands)])
    m.free()
