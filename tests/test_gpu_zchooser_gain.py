"""What the trained chooser gives against the plain converted plan, measured
on the GPU: 64 queries of the batched generator from a seed disjoint from
the training and held-out sets, each run with the plain plan (greedy
left-deep order converted and factored) and with the plan the committed
network picks.  End-to-end time = choice (host + GPU inference, median of
15 alternating repetitions) + root builds + join (median of 5 runs).

The network is consulted only where its fitted gate and margin let it
(queries of at least gate_rows rows, and a predicted score at least margin
below the plain plan's; both fitted on the training run's validation
queries): everywhere else the choice is the plain plan itself.  So both
plans must give the same count, a gated query must get the plain plan, and
the learned end-to-end total must stay within 2% of the plain total (the
timing noise of the few switched queries; the 512 held-out queries of the
training run, profiles/chooser_heldout_512.md, are the measurement of the
gain).  The file name sorts it after the parity tests."""

import os
import statistics

import pytest

import datagen

pytestmark = pytest.mark.gpu

N = 64


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10841_amd import fj, learn, runner
    ctx = fj.Context(0)
    yield fj, learn, runner, ctx
    ctx.close()


def test_learned_choice_against_plain_plan(env):
    fj, learn, runner, ctx = env
    assert os.path.exists(learn.DEFAULT_WEIGHTS)
    m, info = learn.load(ctx)
    assert info["features"] == fj.FEATURES and info["hidden"] == 128
    seed = datagen.seed_for(5, 2)
    tot_plain = tot_learned = 0.0
    switched = 0
    for i in range(N):
        dq, _ = datagen.batch_query(seed, i)
        d = runner.DeviceQuery(ctx, dq)
        sks = d.sketches()
        gate, margin = int(info.get("gate_rows", 0)), float(info.get("margin", 0.0))
        tp, tl = learn.choice_times(fj, d, m, sks, margin, gate, learn.CHOICE_REPS)
        p_plain = fj.plan_from_binary(d.q, fj.greedy_order(d.q, sks), True)
        p_learn, k, _ = d.choose(m, sks, margin, gate)
        rows = sum(int(sk.rows) for sk in sks)   # the gate's measure: the atoms' rows
        if rows < gate:
            assert k == 0 and p_learn.nodes() == p_plain.nodes(), i
        s_plain, c_plain = learn.time_plan(ctx, d, p_plain, 5)
        if k == 0:
            s_learn, c_learn = s_plain, c_plain
        else:
            switched += 1
            s_learn, c_learn = learn.time_plan(ctx, d, p_learn, 5)
        assert c_learn == c_plain, (i, dq.kind)
        tot_plain += statistics.median(tp) + s_plain
        tot_learned += statistics.median(tl) + s_learn
    ratio = tot_learned / tot_plain
    print(f"learned/plain end-to-end over {N} queries: {ratio:.3f} "
          f"({tot_learned * 1e3:.2f} ms vs {tot_plain * 1e3:.2f} ms, {switched} switched)")
    assert ratio <= 1.02
    m.free()
