"""Benchmark: the acyclic star join on one MI355X.

Workload (star, 10M facts): fact table F of 10,000,000 rows x 4 int32 foreign
keys, each Zipf(s=1.1) over its dimension; 4 dimension tables of 1,000,000
rows (int32 key 0..N-1, int32 attribute uniform in 0..99) with the selection
attribute < 10 pushed down on each.  Query
    Q(k1..k4, a1..a4) :- F(k1..k4), D1(k1,a1), ..., D4(k4,a4)
with the plan converted and factored from the left-deep order [F, D1..D4].

One step is the whole hot path on resident inputs: the four selections, the
COLT root builds of the four dimensions, the join (the fact table is iterated
directly and probed into the four dimension maps) and the materialization of
min(count, 1M) result rows.  ``value`` is fact tuples probed per second over
whole steps.

Prints one JSON line.  Extra fields: the dominant kernel's roofline (live
HIP-event timing inside the library), per-phase times and the CPU oracle timed
on the host (the ``cpu_baseline`` leg, the only part that runs the oracle).
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
OUT_CAP = 1_000_000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--seed-rep", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    from paper_2301_10841_amd import fj, runner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    dq = datagen.star_schema(datagen.seed_for(2, args.seed_rep))
    n_fact = dq.relations[0].nrows
    log(f"generated star workload in {time.time() - t0:.1f}s")

    ctx = fj.Context(0, timing=True)
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary([0, 1, 2, 3, 4], True)
    colts = d.build(plan)
    out = torch.empty((OUT_CAP, dq.nvars), dtype=torch.int32, device="cuda:0")

    def step():
        d.apply_filters()
        d.rebuild(colts)
        return ctx.execute(d.q, plan, colts, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timings_reset()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    counts = []
    for _ in range(args.steps):
        cnt, written, _ = step()
        counts.append(cnt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    tim = ctx.timings()
    assert len(set(counts)) == 1, counts
    count = counts[0]

    ms_step = 1e3 * elapsed / args.steps
    probe_tps = n_fact * args.steps / elapsed
    out_tps = count * args.steps / elapsed
    ms0, n0 = tim["probe0"]
    avg_probe0_ms = ms0 / max(n0, 1)
    # algorithmic bytes of one node-0 probe launch: the four int32 fact
    # columns streamed once (16 B per fact row) plus the survivors written
    # to the next frontier (4 keys, 4 handles, one 8-byte multiplicity)
    alg_bytes = 16 * n_fact + written * (4 * 4 + 4 * 4 + 8)
    achieved = alg_bytes / (avg_probe0_ms * 1e-3) / 1e9
    phases = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
              for k, v in tim.items() if v[1]}

    # sanity: exact count against the closed form (numpy, not the GPU)
    from oracle import closed
    dims = [tuple(dq.relations[i + 1].cols) for i in range(4)]
    want = closed.star_count(dq.relations[0].cols, dims, [10] * 4)
    if want != count:
        raise SystemExit(f"count mismatch: GPU {count} vs closed form {want}")

    cpu = None
    if not args.no_cpu:
        from oracle import cfj
        from oracle import plans as P
        oplan = P.factor(P.binary2fj(dq, [0, 1, 2, 3, 4]))
        times = []
        for _ in range(args.cpu_reps):
            tc = time.perf_counter()
            r = cfj.run(dq, oplan, materialize=True, cap=OUT_CAP, counters=False)
            times.append(time.perf_counter() - tc)
            assert r["count"] == count
        tmed = statistics.median(times)
        cpu = {"value": n_fact / tmed, "unit": "probe tuples/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload ({n_fact} fact rows, selections, builds, join, "
                         f"materialization), median of {args.cpu_reps} runs, single-threaded C oracle",
               "s_per_run": tmed, "host_cpus": os.cpu_count()}

    res = {
        "metric": "probe tuples/sec + output tuples/sec, achieved HBM GB/s; learned vs plain plan time",
        "value": probe_tps,
        "unit": "probe tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded Zipf star schema)",
        "config": {"workload": "star join: 10M-row fact x 4 Zipf(1.1) int32 FKs, 4 x 1M-row dimensions, "
                               "attr<10 on each, count + up to 1M materialized rows",
                   "fact_rows": n_fact, "dim_rows": dq.relations[1].nrows, "plan": "factored [F,D1,D2,D3,D4]"},
        "count": count,
        "output_tuples_per_s": out_tps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_probe (node 0)", "avg_launch_ms": avg_probe0_ms,
                     "alg_bytes_per_launch": alg_bytes},
        "phases": phases,
        "cpu_baseline": cpu,
    }
    for c in colts:
        c.free()
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
