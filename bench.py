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
HIP-event timing inside the library, around the node-0 probe alone), the
one-filter variant, the learned chooser's leg and the CPU oracle timed on the
host (the ``cpu_baseline`` leg, the only part that runs the oracle).
"""

import argparse
import gc
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
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 for the star, whose step is a fraction of a ms; 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default: 20 for the star; 3)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--seed-rep", type=int, default=0)
    ap.add_argument("--workload", choices=("star", "batch", "rmat", "bushy", "ablation", "factorized"), default="star")
    ap.add_argument("--rmat-scale", type=int, default=22)
    ap.add_argument("--rmat-edges", type=int, default=50_000_000)
    ap.add_argument("--cycle4-scale", type=int, default=20, help="rmat workload: scale of the 4-cycle run")
    ap.add_argument("--cycle4-parts", type=int, default=16, help="rmat workload: the 4-cycle counted in parts by w")
    ap.add_argument("--rmat-cache", default=None, help="rmat workload: directory keeping the drawn graph")
    ap.add_argument("--queries", type=int, default=256, help="batch workload: number of queries")
    ap.add_argument("--tune-queries", type=int, default=48, help="batch workload: calibration batch size")
    ap.add_argument("--no-extras", action="store_true",
                    help="star: skip the one-filter variant and the learned-vs-plain leg; rmat: time the "
                         "triangle steps only (profiling)")
    ap.add_argument("--chooser-queries", type=int, default=48,
                    help="star workload: held-out queries for the learned-vs-plain leg (0: skip)")
    ap.add_argument("--no-filter", action="store_true",
                    help="star: the node-0 scan without the first lookup's key filter (for comparison)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    star = args.workload == "star"
    if args.steps is None:
        args.steps = 200 if star else 20
    if args.warmup is None:
        args.warmup = 20 if star else 3
    # Python's cyclic garbage collector stays off: one collection of this
    # process's heap (torch's objects) takes tens of milliseconds and lands
    # inside whichever timed step triggers it (reference counting still
    # frees everything the steps create)
    gc.collect()
    gc.disable()
    if args.calibrate_copy:
        return calibrate_copy()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "factorized":
        return bench_factorized(args)
    if args.workload == "bushy":
        return bench_bushy(args)
    if args.workload == "ablation":
        return bench_ablation(args)
    if args.workload == "rmat":
        return bench_rmat(args)

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

    ctx = fj.Context(0, timing=2, no_filter=args.no_filter)   # events around the node-0 probe only
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary([0, 1, 2, 3, 4], True)
    colts = d.build(plan)
    out = torch.empty((OUT_CAP, dq.nvars), dtype=torch.int32, device="cuda:0")

    def step():
        # the selections and the root builds in one library call, then the join
        d.select_rebuild(colts)
        return ctx.execute(d.q, plan, colts, out=out)

    for _ in range(args.warmup):
        step()
    # which node-0 kernel runs: the key filter's count says
    d.select_rebuild(colts)
    _, _, st0 = ctx.execute(d.q, plan, colts, out=out, stats=True)
    filtered = int(st0.filtered)
    probe0_lookups = int(st0.per_node()[0]["probe"])
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
    warm_probe0_ms = ms0 / max(n0, 1)
    # The timed steps run back to back, and one step's inputs (160 MB of
    # fact columns, about 40 MB of dimensions and maps) fit in the 256 MB
    # Infinity Cache.  The roofline takes the same steps started cold: a
    # 512 MiB buffer is read and written before each, outside the probe's
    # events, so the fact stream comes from HBM.
    flush = torch.zeros(1 << 27, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    ctx.timings_reset()
    for _ in range(args.steps):
        flush.add_(1)
        step()
    torch.cuda.synchronize()
    ms0c, n0c = ctx.timings()["probe0"]
    avg_probe0_ms = ms0c / max(n0c, 1)
    del flush
    # per-phase times: a further pass of warm steps with every kernel class
    # between events (the events cost a little; the step time above has none)
    ctx.set_timing(1)
    ctx.timings_reset()
    for _ in range(args.steps):
        step()
    phase_tim = ctx.timings()
    ctx.set_timing(2)
    # algorithmic bytes of one node-0 probe launch, which also writes the
    # result rows: the four int32 fact columns streamed once (16 B per fact
    # row), and per result row its 8 int32 values written and, per
    # dimension, the tail offset and attribute gathered (4 x 8 B)
    alg_bytes = 16 * n_fact + written * (8 * 4 + 4 * 8)
    achieved = alg_bytes / (avg_probe0_ms * 1e-3) / 1e9
    achieved_warm = alg_bytes / (warm_probe0_ms * 1e-3) / 1e9
    phases = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
              for k, v in phase_tim.items() if v[1]}
    hbm_copy = practical_hbm()
    tr = measured_traffic()
    traffic_bytes, traffic_note = None, "no counter summary for the current kernel source"
    if tr:
        traffic_bytes = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]
        traffic_note = (f"rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by a 1 GiB copy "
                        f"(factors {tr['copy_factor_fetch']:.3f}, {tr['copy_factor_write']:.3f})")

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
            if r["count"] != count:
                raise SystemExit(f"count mismatch: GPU {count} vs CPU oracle {r['count']}")
        tmed = statistics.median(times)
        one = {"value": n_fact / tmed, "unit": "probe tuples/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload ({n_fact} fact rows, selections, builds, join, "
                         f"materialization), median of {args.cpu_reps} runs, single-threaded C oracle",
               "s_per_run": tmed}
        procs = host_cores()
        import tempfile
        with tempfile.TemporaryDirectory(dir="/dev/shm" if os.path.isdir("/dev/shm") else None) as td:
            tot, wall = oracle_all_cores(dq, oplan, ("slice", 0), procs, td)
        if tot != count:
            raise SystemExit(f"count mismatch: GPU {count} vs all-cores CPU oracle {tot}")
        cpu = {"value": n_fact / wall, "unit": "probe tuples/s", "cores": procs, "kind": "oracle",
               "sample": f"the full workload, count only: the fact table cut into {procs} row ranges, one "
                         f"process each running the C oracle on its range against the whole dimensions "
                         f"(each process filters and builds all four), one run, wall time from the moment "
                         f"every process holds its inputs",
               "s_per_run": wall, "host_cpus": os.cpu_count(), "single_core": one}

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes,
                     "traffic_note": traffic_note,
                     "kernel": ("k_scan_filter + k_scan_rounds (node 0 in two launches: the first lookup's "
                                "key filter in LDS, then the later lookups over the rows that pass it)" if filtered
                                else "k_scan_probe (node 0)"),
                     "first_lookup_filtered": filtered, "node0_lookups": probe0_lookups,
                     "avg_launch_ms": avg_probe0_ms,
                     "launches": "cold: a 512 MiB buffer rewritten before each step",
                     "alg_bytes_per_launch": alg_bytes,
                     "warm": {"avg_launch_ms": warm_probe0_ms, "achieved": achieved_warm,
                              "frac": achieved_warm / HBM_PEAK_GBS},
                     "practical_hbm_copy_GBs": hbm_copy,
                     "frac_of_practical": achieved / hbm_copy if hbm_copy else None,
                     "useful_byte_efficiency": alg_bytes / traffic_bytes if traffic_bytes else None,
                     "l2_hit_rate": tr["tcc_hit_rate"] if tr else None},
        "phases": phases,
        "phases_note": "a separate pass of warm steps with hipEvents around every kernel class",
        "cpu_baseline": cpu,
    }
    for c in colts:
        c.free()
    if not args.no_extras:
        res["one_filter_variant"] = star_one_filter(ctx, args)
    if args.chooser_queries > 0 and not args.no_extras:
        res["learned_vs_plain"] = chooser_leg(ctx, args.chooser_queries)
    ctx.close()
    print(json.dumps(res), flush=True)


def star_one_filter(ctx, args):
    """The star with the selection on D1 only: about 1M result rows, all
    materialized, so row emission runs at size.  Output tuples/s over whole
    steps (its parity with the oracle is a GPU test)."""
    import torch

    import datagen
    from paper_2301_10841_amd import runner
    dq = datagen.star_schema(datagen.seed_for(2, args.seed_rep), filter_dims=(0,))
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary([0, 1, 2, 3, 4], True)
    colts = d.build(plan)
    want, _, _ = ctx.execute(d.q, plan, colts)
    d.rebuild(colts)
    out = torch.empty((max(want, 1), dq.nvars), dtype=torch.int32, device="cuda:0")

    def step():
        d.apply_filters()
        d.rebuild(colts)
        return ctx.execute(d.q, plan, colts, out=out)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    steps = max(5, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        cnt, written, _ = step()
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / steps
    for c in colts:
        c.free()
    if cnt != want or written != cnt:
        raise SystemExit(f"one-filter star: count {cnt}, written {written}, count-only run {want}")
    return {"count": cnt, "materialized_rows": written, "ms_per_step": per * 1e3,
            "output_tuples_per_s": cnt / per, "probe_tuples_per_s": dq.relations[0].nrows / per}


def chooser_leg(ctx, n):
    """Learned vs plain plan time on n held-out queries of the batched
    generator (a seed disjoint from the chooser's training and held-out
    sets): every candidate timed (root builds + join, median of 5) and both
    choices' overheads timed live; end-to-end = choice + chosen plan."""
    import datagen
    from paper_2301_10841_amd import learn
    t0 = time.time()
    m, info = learn.load(ctx)
    rows = learn.evaluate(ctx, m, learn.QuerySupply(0), datagen.seed_for(5, 3), n, reps=5,
                          margin=float(info.get("margin", 0.0)), gate_rows=int(info.get("gate_rows", 0)))
    s = learn.summarize(rows)
    m.free()
    log(f"chooser leg: {n} queries in {time.time() - t0:.1f}s")
    return {"queries": n, "learned_over_plain_total": s["learned_over_plain_total"],
            "learned_over_plain_geomean": s["learned_over_plain_geomean"],
            "learned_mean_regret": s["learned_mean_regret_vs_best"],
            "plain_mean_regret": s["plain_mean_regret_vs_best"],
            "choose_learned_ms": s["choose_learned_ms_mean"], "choose_plain_ms": s["choose_plain_ms_mean"],
            "gate_rows": int(info.get("gate_rows", 0)), "margin": float(info.get("margin", 0.0)),
            "weights": "paper_2301_10841_amd/weights/chooser.npz"}


def host_cores():
    """Host threads the oracle may use: the CPUs this process may run on,
    at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _slice_rel(rel, lo, hi):
    from datagen import synth
    return synth.Relation(rel.name, [c[lo:hi] for c in rel.cols])


def _part_query(spec, rels, part, nparts):
    """Part `part` of `nparts` of a query whose result splits over disjoint
    inputs: ("slice", r) cuts relation r into contiguous row ranges (every
    result row uses one row of r); ("xmod", (a_r, a_s, a_t)) takes the
    triangle atoms R(x, y), S(y, z), T(z, x) and keeps the R and T rows
    whose x is congruent to part and the S rows such an R row reaches (a
    triangle counts in the part of its x)."""
    import numpy as np
    from datagen import synth
    kind, arg = spec["split"]
    if kind == "slice":
        rels = list(rels)
        n = rels[arg].nrows
        lo, hi = n * part // nparts, n * (part + 1) // nparts
        rels[arg] = _slice_rel(rels[arg], lo, hi)
        return synth.make_query(spec["var_names"], rels, spec["atoms"], spec["filters"], spec["head"])
    atoms = spec["atoms"]
    (r_src, r_dst), (s_src, s_dst), (t_src, t_dst) = (rels[atoms[a][0]].cols for a in arg)
    kr = (r_src % nparts) == part
    nv = int(max(r_dst.max(initial=0), s_src.max(initial=0))) + 1
    reach = np.zeros(nv, bool)
    reach[r_dst[kr]] = True
    ks = reach[s_src]
    kt = (t_dst % nparts) == part
    out = [synth.Relation("R", [r_src[kr], r_dst[kr]]), synth.Relation("S", [s_src[ks], s_dst[ks]]),
           synth.Relation("T", [t_src[kt], t_dst[kt]])]
    return synth.make_query(spec["var_names"], out, [(i, atoms[a][1]) for i, a in enumerate(arg)],
                            None, spec["head"])


def _oracle_worker(spec, paths, parts, nparts, barrier, results):
    """One host process of the all-cores oracle leg: load the columns, cut
    its parts, wait for every process, then run the oracle on each part."""
    try:
        import numpy as np
        from datagen import synth
        from oracle import cfj
        rels = [synth.Relation(name, [np.load(f, mmap_mode="r") for f in files]) for name, files in paths]
        queries = [_part_query(spec, rels, p, nparts) for p in parts]
        barrier.wait()
        total = 0
        for q in queries:
            total += cfj.run(q, spec["plan"], materialize=False, counters=False)["count"]
        results.put(total)
    except BaseException:
        barrier.abort()
        results.put(None)
        raise


def oracle_all_cores(dq, plan, split, procs, tmpdir):
    """The C oracle over `procs` host processes, one part each (count
    only); returns (count, wall seconds from the moment every process has
    its inputs to the last one's end)."""
    import multiprocessing as mp

    import numpy as np
    paths = []
    for i, rel in enumerate(dq.relations):
        files = []
        for j, c in enumerate(rel.cols):
            f = os.path.join(tmpdir, f"r{i}_c{j}.npy")
            np.save(f, np.ascontiguousarray(c))
            files.append(f)
        paths.append((rel.name, files))
    spec = {"var_names": dq.var_names, "atoms": dq.atoms, "filters": dq.filters, "head": dq.head,
            "plan": plan, "split": split}
    mpc = mp.get_context("spawn")   # the parent holds a GPU context: no fork
    barrier = mpc.Barrier(procs + 1)
    results = mpc.Queue()
    ps = [mpc.Process(target=_oracle_worker, args=(spec, paths, [w], procs, barrier, results)) for w in range(procs)]
    for p in ps:
        p.start()
    barrier.wait(timeout=300)
    t0 = time.monotonic()
    got = [results.get(timeout=600) for _ in ps]
    wall = time.monotonic() - t0
    if any(g is None for g in got):
        raise SystemExit("an all-cores oracle process failed")
    total = sum(got)
    for p in ps:
        p.join()
    return total, wall


def trace_power4(src, dst):
    """trace(A^4) of a 0/1 adjacency matrix: the number of closed walks of
    length 4, sum over (u, v) of (A^2)[u, v] (A^2)[v, u]."""
    import numpy as np
    import scipy.sparse as sp
    n = int(max(src.max(), dst.max())) + 1
    a = sp.csr_matrix((np.ones(src.size, np.int64), (src.astype(np.int64), dst.astype(np.int64))), shape=(n, n))
    a2 = a @ a
    return int(a2.multiply(a2.T).sum())


def sampled_triangles(src, dst, xs):
    """Exact number of triangles E(x,y), E(y,z), E(z,x) whose x is in xs,
    by intersecting adjacency lists with numpy (edges are distinct)."""
    import numpy as np
    order = np.argsort(src, kind="stable")
    s_sorted, d_by_src = src[order], dst[order]
    out_ptr = np.searchsorted(s_sorted, np.arange(int(max(src.max(), dst.max())) + 2))
    order_in = np.argsort(dst, kind="stable")
    d_sorted, s_by_dst = dst[order_in], src[order_in]
    in_ptr = np.searchsorted(d_sorted, np.arange(int(max(src.max(), dst.max())) + 2))
    total = 0
    for x in xs:
        ys = d_by_src[out_ptr[x]:out_ptr[x + 1]]
        ins = s_by_dst[in_ptr[x]:in_ptr[x + 1]]
        if ys.size == 0 or ins.size == 0:
            continue
        zs = np.concatenate([d_by_src[out_ptr[y]:out_ptr[y + 1]] for y in ys])
        total += int(np.isin(zs, ins).sum())
    return total


def bench_ablation(args):
    """The paper's ablation (Section 5) on synthetic inputs: the same plans
    over the three tries (simple trie: every level built ahead; simple lazy
    trie: every root built ahead, inner levels lazily; COLT), then the COLT
    with frontier tiles of 2^10 .. 2^24 tuples (the GPU's vectorization
    batch).  A run is a rebuild of every COLT plus the join, count only;
    each figure is the median of up to 5 runs, or the first run when that
    took over 2 s."""
    import torch

    import datagen
    from datagen import synth
    from paper_2301_10841_amd import fj, runner
    cases = []
    e = datagen.rmat_edges(datagen.seed_for(3, 1), 18, 3_000_000)
    tri = synth.triangle_query(e)
    cases.append(("R-MAT 2^18 / 3M edges, triangle, Generic Join plan", tri,
                  [[(0, (0,)), (2, (0,))], [(0, (1,)), (1, (1,))], [(1, (2,)), (2, (2,))]]))
    cases.append(("R-MAT 2^18 / 3M edges, triangle, converted plan [R, S, T]", tri, [0, 1, 2]))
    cases.append(("star, 10M facts x 4 dims, converted plan", datagen.star_schema(datagen.seed_for(2, 0)),
                  [0, 1, 2, 3, 4]))
    qi = 0
    while True:
        dq, _ = datagen.batch_query(datagen.seed_for(6, 0), qi, min_rows=1_000_000, max_rows=1_000_000,
                                    frac_chain=1.0, frac_star=0.0)
        if len(dq.atoms) == 4:
            break
        qi += 1
    cases.append(("4-chain, 1M rows each, converted plan", dq, [0, 1, 2, 3]))

    def run_case(ctx, dq, spec):
        d = runner.DeviceQuery(ctx, dq)
        plan = d.plan_nodes(spec) if isinstance(spec[0], list) else d.plan_binary(spec, True)
        colts = d.build(plan)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            count = ctx.execute(d.q, plan, colts)[0]
            torch.cuda.synchronize()
            first = time.perf_counter() - t0
            if first > 2.0:          # a slow configuration: its first run is the figure
                return count, first
            ts = []
            for _ in range(max(min(args.steps, 5), 1)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                d.rebuild(colts)
                c = ctx.execute(d.q, plan, colts)[0]
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                if c != count:
                    raise SystemExit(f"count changed between runs: {c} vs {count}")
            return count, statistics.median(ts)
        finally:
            for t in colts:
                t.free()

    modes = [("simple trie", 2), ("simple lazy trie", 1), ("COLT", 0)]
    tiles = [1 << 12, 1 << 16, 1 << 20, 1 << 24]
    rows = []
    for name, dq, spec in cases:
        row = {"case": name, "trie_ms": {}, "tile_ms": {}}
        counts = set()
        for mname, trie in modes:
            log(f"{name} | {mname} ...")
            ctx = fj.Context(0, trie=trie)
            c, t = run_case(ctx, dq, spec)
            ctx.close()
            counts.add(c)
            row["trie_ms"][mname] = t * 1e3
            log(f"{name} | {mname}: {t * 1e3:.2f} ms")
        for tile in tiles:
            log(f"{name} | tile {tile} ...")
            ctx = fj.Context(0, tile=tile)
            c, t = run_case(ctx, dq, spec)
            ctx.close()
            counts.add(c)
            row["tile_ms"][str(tile)] = t * 1e3
            log(f"{name} | tile {tile}: {t * 1e3:.2f} ms")
        if len(counts) != 1:
            raise SystemExit(f"{name}: counts differ across tries and tiles: {counts}")
        row["count"] = counts.pop()
        rows.append(row)

    def geo(xs):
        return float(statistics.geometric_mean(xs))

    sp_slt = geo([r["trie_ms"]["simple lazy trie"] / r["trie_ms"]["COLT"] for r in rows])
    sp_simple = geo([r["trie_ms"]["simple trie"] / r["trie_ms"]["COLT"] for r in rows])
    sp_tile = geo([r["tile_ms"][str(tiles[0])] / r["tile_ms"][str(tiles[-1])] for r in rows])
    res = {
        "metric": "COLT speedup over the simple lazy trie and the simple trie (geometric mean over the cases)",
        "value": sp_slt, "unit": "x", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic (seeded R-MAT, Zipf star schema, Zipf PK-FK chain)",
        "config": {"workload": "ablation: tries and frontier tile sizes", "cases": [r["case"] for r in rows],
                   "tiles": tiles},
        "colt_over_slt_geomean": sp_slt, "colt_over_simple_trie_geomean": sp_simple,
        "tile_2p24_over_2p12_geomean": sp_tile, "cases": rows,
    }
    print(json.dumps(res), flush=True)


def bench_factorized(args):
    """Factorized against full results on a fan-out chain R(x, y) join S(y, z)
    (1M R rows, 100K keys, 20 S rows per key: 20M result rows from 1M final
    bindings).  A step runs the plan keeping the final bindings (Section 4.4's
    factorized view, kept as the result as in Section 5.2); the full path
    writes every row.  Expansion of all rows in 1M-row pages is timed apart."""
    import torch

    import datagen
    from paper_2301_10841_amd import fj, runner
    dq = datagen.fanout_chain(datagen.seed_for(10, args.seed_rep))
    ctx = fj.Context(0)
    d = runner.DeviceQuery(ctx, dq)
    plan = d.plan_binary([0, 1], True)
    colts = d.build(plan)
    count = ctx.execute(d.q, plan, colts)[0]
    d.rebuild(colts)
    out = torch.empty((count, d.q.nhead), dtype=torch.int32, device="cuda:0")

    def timed(fn):
        for _ in range(args.warmup):
            r = fn()
            if isinstance(r, fj.Result):
                r.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
            if isinstance(r, fj.Result):
                r.free()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    def full_step():
        c, w, _ = ctx.execute(d.q, plan, colts, out=out)
        if c != count or w != count:
            raise SystemExit(f"full run wrote {w} of {c} rows, expected {count}")

    def fact_step():
        return ctx.execute_factorized(d.q, plan, colts)

    log("factorized: full materialization")
    t_full = timed(full_step)
    sums_full = out.to(torch.int64).sum(dim=0).cpu().tolist()
    log("factorized: bindings kept")
    t_fact = timed(fact_step)
    res = ctx.execute_factorized(d.q, plan, colts)
    if res.count != count:
        raise SystemExit(f"factorized count {res.count} != {count}")
    page = 1 << 20
    pbuf = out[:page]
    log("factorized: expansion")
    # checked pass (also computes the row counts' scan, once per result)
    sums = torch.zeros(d.q.nhead, dtype=torch.int64, device="cuda:0")
    first = 0
    while first < count:
        w = res.expand(first, pbuf)
        sums += pbuf[:w].to(torch.int64).sum(dim=0)
        first += w
    if sums.cpu().tolist() != sums_full:
        raise SystemExit("expanded rows differ from the fully materialized rows")
    # timed pass: every page, nothing else
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first = 0
    while first < count:
        first += res.expand(first, pbuf)
    torch.cuda.synchronize()
    t_exp = time.perf_counter() - t0
    bindings = res.bindings
    res.free()
    # bytes the result holds: x, y values, one handle into S's level and a
    # multiplicity per binding, against nhead int32 per row
    fact_bytes = bindings * (2 * 4 + 4 + 8)
    full_bytes = count * d.q.nhead * 4
    cpu = None
    if not args.no_cpu:
        from oracle import cfj
        from oracle import plans as P
        t0 = time.perf_counter()
        want = cfj.run(dq, P.factor(P.binary2fj(dq, [0, 1])), batch=1000, materialize=False, counters=False)
        tc = time.perf_counter() - t0
        if want["count"] != count:
            raise SystemExit(f"count mismatch: GPU {count} vs CPU oracle {want['count']}")
        cpu = {"value": count / tc, "unit": "output tuples/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload counted (no rows written), one run, single-threaded C oracle",
               "s_per_run": tc}
    for t in colts:
        t.free()
    res = {
        "metric": "output tuples/s with the result kept factorized",
        "value": count / t_fact, "unit": "output tuples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_fact * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic (seeded uniform fan-out chain)",
        "config": {"workload": "R(x,y) 1M rows join S(y,z) 2M rows, 100K keys, 20 S rows per key; "
                               "20M result rows"},
        "full_ms": t_full * 1e3, "expand_all_ms": t_exp * 1e3, "rows": count, "bindings": bindings,
        "factorized_bytes": fact_bytes, "full_bytes": full_bytes,
        "full_over_factorized_time": t_full / t_fact,
        "roofline": None, "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def bench_bushy(args):
    """A bushy plan against the left-deep one on a 4-chain of 1M-row
    relations (primary-key/foreign-key joins with Zipf skew, the batched
    generator's chain recipe): ((R0 R1) (R2 R3)) runs [R2, R3] first, its
    result materialized on the device as a relation, then [R0, R1, P1]
    (Section 2.2).  Count only; a step includes every plan's COLT builds."""
    import torch

    import datagen
    from paper_2301_10841_amd import fj, runner
    seed = datagen.seed_for(6, args.seed_rep)
    qi = 0
    while True:
        dq, _ = datagen.batch_query(seed, qi, min_rows=1_000_000, max_rows=1_000_000,
                                    frac_chain=1.0, frac_star=0.0)
        if len(dq.atoms) == 4:
            break
        qi += 1
    tree = ((0, 1), (2, 3))
    ctx = fj.Context(0)
    d = runner.DeviceQuery(ctx, dq)

    def bushy_step():
        return d.run_bushy(tree, materialize=False)["count"]

    plan = d.plan_binary([0, 1, 2, 3], True)

    def left_deep_step():
        colts = d.build(plan)
        c = ctx.execute(d.q, plan, colts)[0]
        for t in colts:
            t.free()
        return c

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            c = fn()
        torch.cuda.synchronize()
        return c, (time.perf_counter() - t0) / args.steps

    count, t_bushy = timed(bushy_step)
    count_ld, t_ld = timed(left_deep_step)
    if count_ld != count:
        raise SystemExit(f"bushy count {count} != left-deep count {count_ld}")
    # the materialized intermediate's size: the first plan of the decomposition
    sub = fj.bushy_decompose(tree)
    inter = runner.DeviceQuery(ctx, datagen.synth.make_query(
        [dq.var_names[v] for v in (2, 3, 4)], [dq.relations[dq.atoms[2][0]], dq.relations[dq.atoms[3][0]]],
        [(0, (0, 1)), (1, (1, 2))]))
    p1 = inter.plan_binary([0, 1], True)
    c1 = inter.build(p1)
    inter_rows = ctx.execute(inter.q, p1, c1)[0]
    for t in c1:
        t.free()
    cpu = None
    if not args.no_cpu:
        from oracle import bushy as B
        t0 = time.perf_counter()
        want = B.evaluate(dq, tree)
        tc = time.perf_counter() - t0
        if want["count"] != count:
            raise SystemExit(f"count mismatch: GPU {count} vs CPU oracle {want['count']}")
        cpu = {"value": want["count"] / tc, "unit": "output tuples/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload (both plans of the decomposition, intermediate materialized, "
                         "final rows materialized), one run, single-threaded C oracle",
               "s_per_run": tc}
    res = {
        "metric": "output tuples/s of a bushy plan (intermediate materialized on the device), count only",
        "value": count / t_bushy, "unit": "output tuples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_bushy * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic (seeded Zipf PK-FK chain)",
        "config": {"workload": "4-chain R0(x0,x1)..R3(x3,x4), 1M rows each, PK-FK with Zipf skew; "
                               "bushy ((R0 R1) (R2 R3)) vs left-deep [R0, R1, R2, R3]",
                   "rows": [int(dq.relations[r].nrows) for r, _ in dq.atoms]},
        "count": count, "decomposition": sub, "intermediate_rows": inter_rows,
        "left_deep_ms_per_step": t_ld * 1e3, "bushy_over_left_deep": t_bushy / t_ld,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(res), flush=True)


def rmat_cached(args, seed, scale, n_edges):
    """datagen.rmat_edges, kept in --rmat-cache (when given) so that runs of
    one session (profiler passes) draw the graph once."""
    import numpy as np

    import datagen
    if not args.rmat_cache:
        return datagen.rmat_edges(seed, scale, n_edges)
    os.makedirs(args.rmat_cache, exist_ok=True)
    f = os.path.join(args.rmat_cache, f"rmat_{seed:x}_{scale}_{n_edges}.npz")
    if os.path.exists(f):
        z = np.load(f)
        return z["src"], z["dst"]
    src, dst = datagen.rmat_edges(seed, scale, n_edges)
    np.savez(f + ".tmp.npz", src=src, dst=dst)
    os.replace(f + ".tmp.npz", f)
    return src, dst


def bench_rmat(args):
    """Cyclic joins on an R-MAT graph (2^scale vertices, the first n distinct
    edges, self-loops dropped).  Triangle count with the Generic Join plan
    [[R(x),T(x)],[R(y),S(y)],[S(z),T(z)]]; one step = COLT root builds + the
    join (inner tries forced lazily).  Checks: the converted plan gives the
    same count, and the triangles through 64 sampled x vertices equal an
    independent numpy count.  Then the 4-cycle at a reduced scale, counted
    with its Generic Join plan and checked against trace(A^4)."""
    import numpy as np
    import torch

    import datagen
    from datagen import synth
    from paper_2301_10841_amd import fj, runner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    src, dst = rmat_cached(args, datagen.seed_for(3, 1 + args.seed_rep), args.rmat_scale, args.rmat_edges)
    log(f"generated {src.size} R-MAT edges (scale {args.rmat_scale}) in {time.time() - t0:.1f}s")
    ctx = fj.Context(0, timing=True)
    dq = synth.triangle_query((src, dst))
    d = runner.DeviceQuery(ctx, dq)
    gj = d.plan_nodes([[(0, (0,)), (2, (0,))], [(0, (1,)), (1, (1,))], [(1, (2,)), (2, (2,))]])
    colts = d.build(gj)

    def step():
        d.rebuild(colts)
        return ctx.execute(d.q, gj, colts)[0]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timings_reset()
    ts = time.perf_counter()
    counts = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    tim = ctx.timings()
    assert len(set(counts)) == 1, counts
    tri = counts[0]
    log(f"triangles: {tri}, {elapsed / args.steps * 1e3:.1f} ms per step")
    d.rebuild(colts)
    _, _, st = ctx.execute(d.q, gj, colts, stats=True)
    nodes = st.per_node()
    probe_tuples = sum(n["cover"] for n in nodes)
    probes = sum(n["probe"] for n in nodes)
    # algorithmic bytes of the probe kernels per step: each cover tuple's
    # key (4 B, stored beside its offset), each get()'s map slot (16 B) and
    # each binding passed to the next node, written once and read once
    # (two values, two handles, an 8-byte multiplicity: 24 B each way)
    probe_alg_bytes = sum(4 * n["cover"] + 16 * n["probe"] for n in nodes) + \
        48 * sum(n["survivors"] for n in nodes[:-1])
    pr_ms, pr_n = tim["probe"]
    pr_ms += tim["probe0"][0]
    pr_n += tim["probe0"][1]
    probe_s = pr_ms * 1e-3 / args.steps
    probe_roof = {"bound": "hbm", "kernel": "k_probe (nodes 0-2)", "achieved": probe_alg_bytes / probe_s / 1e9,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": probe_alg_bytes / probe_s / 1e9 / HBM_PEAK_GBS,
                  "alg_bytes_per_step": probe_alg_bytes, "probe_ms_per_step": pr_ms / args.steps,
                  "launches_per_step": pr_n / args.steps, "traffic": None}
    per = elapsed / args.steps
    if args.no_extras:
        for c in colts:
            c.free()
        ctx.close()
        print(json.dumps({"workload": "rmat triangle", "triangles": tri, "ms_per_step": per * 1e3,
                          "probe_tuples_per_s": probe_tuples / per, "probes_per_s": probes / per,
                          "phases": {k: v[0] / args.steps for k, v in tim.items() if v[1]},
                          "launches": {k: v[1] / args.steps for k, v in tim.items() if v[1]},
                          "roofline": probe_roof, "per_node": nodes}), flush=True)
        return
    # plan invariance: the converted, factored plan of [R, S, T]
    conv = d.plan_binary([0, 1, 2], True)
    t1 = time.perf_counter()
    r = d.run(conv, materialize=False)
    conv_s = time.perf_counter() - t1
    for c in r["colts"]:
        c.free()
    assert r["count"] == tri, (r["count"], tri)
    log(f"converted plan: same count in {conv_s:.2f} s")
    # sampled parity: the triangles through 2048 random x vertices.  The
    # sampled query keeps the R rows with x in the sample, the S rows whose
    # y such an R row reaches and the T rows that close back to the sample:
    # exactly the rows those triangles use.
    rng = np.random.default_rng(12345)
    xs = np.sort(rng.choice(np.unique(src), size=2048, replace=False))
    want = sampled_triangles(src, dst, xs)
    keep = np.isin(src, xs)
    keep_s = np.isin(src, np.unique(dst[keep]))
    keep_t = np.isin(dst, xs)
    es = synth.Relation("Rs", [src[keep], dst[keep]])
    ss = synth.Relation("Ss", [src[keep_s], dst[keep_s]])
    ts = synth.Relation("Ts", [src[keep_t], dst[keep_t]])
    sq = synth.make_query(["x", "y", "z"], [es, ss, ts], [(0, (0, 1)), (1, (1, 2)), (2, (2, 0))])
    ds = runner.DeviceQuery(ctx, sq)
    rs = ds.run(ds.plan_binary([0, 1, 2], True), materialize=False, stats=True)
    rs_probe = sum(n_["cover"] for n_ in rs["stats"].per_node())
    for c in rs["colts"]:
        c.free()
    assert rs["count"] == want, (rs["count"], want)
    for c in colts:
        c.free()
    del d, ds
    # CPU baseline: the C oracle on the sampled query
    cpu = None
    if not args.no_cpu:
        from oracle import cfj
        from oracle import plans as P
        tc = time.perf_counter()
        r_cpu = cfj.run(sq, P.factor(P.binary2fj(sq, [0, 1, 2])), materialize=False, counters=False)
        t_cpu = time.perf_counter() - tc
        if r_cpu["count"] != rs["count"]:
            raise SystemExit(f"sampled triangles: GPU {rs['count']} vs CPU oracle {r_cpu['count']}")
        one = {"value": rs_probe / t_cpu if rs_probe else None, "unit": "probe tuples/s", "cores": 1,
               "kind": "oracle", "s_per_run": t_cpu}
        procs = host_cores()
        import tempfile
        with tempfile.TemporaryDirectory(dir="/dev/shm" if os.path.isdir("/dev/shm") else None) as td:
            tot, wall = oracle_all_cores(sq, P.factor(P.binary2fj(sq, [0, 1, 2])), ("xmod", (0, 1, 2)), procs, td)
        if tot != rs["count"]:
            raise SystemExit(f"sampled triangles: GPU {rs['count']} vs all-cores CPU oracle {tot}")
        cpu = {"value": rs_probe / wall if rs_probe else None, "unit": "probe tuples/s", "cores": procs,
               "kind": "oracle",
               "sample": f"the triangle query restricted to {xs.size} sampled x vertices ({int(keep.sum())} R, "
                         f"{int(keep_s.sum())} S and {int(keep_t.sum())} T rows), converted plan, count only, "
                         f"one run including its COLT builds; all cores: the sample split over {procs} "
                         f"processes by x mod {procs}, wall time once every process holds its part",
               "s_per_run": wall, "host_cpus": os.cpu_count(), "single_core": one}
    log("sampled triangles and CPU oracle legs done")
    # 4-cycle at a reduced scale against trace(A^4)
    s4, d4 = datagen.rmat_edges(datagen.seed_for(3, 1 + args.seed_rep), args.cycle4_scale,
                                int(round(11.92 * (1 << args.cycle4_scale))))
    # Counted in parts by ranges of w (every cycle has one w): part i keeps
    # the E(w,x) and E(z,w) rows whose w falls in its range and all of
    # E(x,y) and E(y,z); the parts' counts add up to the count, and each part
    # reports when it is done.  Each part's COLT builds are in its time.
    nv = int(max(s4.max(), d4.max())) + 1
    parts = args.cycle4_parts
    cyc, cyc_s, probes4 = 0, 0.0, 0
    e_all = synth.Relation("E", [s4, d4])
    for i in range(parts):
        lo, hi = nv * i // parts, nv * (i + 1) // parts
        k0 = (s4 >= lo) & (s4 < hi)
        k3 = (d4 >= lo) & (d4 < hi)
        q4 = synth.make_query(["w", "x", "y", "z"],
                              [synth.Relation("E0", [s4[k0], d4[k0]]), e_all,
                               synth.Relation("E3", [s4[k3], d4[k3]])],
                              [(0, (0, 1)), (1, (1, 2)), (1, (2, 3)), (2, (3, 0))])
        dc = runner.DeviceQuery(ctx, q4)
        gj4 = dc.plan_nodes([[(0, (0,)), (3, (0,))], [(0, (1,)), (1, (1,))], [(1, (2,)), (2, (2,))],
                             [(2, (3,)), (3, (3,))]])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        c4 = dc.build(gj4)
        n4, _, st4 = ctx.execute(dc.q, gj4, c4, stats=True)
        torch.cuda.synchronize()
        cyc_s += time.perf_counter() - t2
        cyc += n4
        probes4 += sum(n["probe"] for n in st4.per_node())
        for c in c4:
            c.free()
        del dc
        log(f"4-cycles at 2^{args.cycle4_scale}, part {i + 1}/{parts}: {n4} ({cyc_s:.1f} s so far)")
    # the check: trace(A^4), stored for the scales whose closed form takes
    # the CPU minutes (tests/golden/make_rmat_cycle4.py), else computed here
    want4, check4 = None, "trace(A^4)"
    if args.seed_rep == 0:
        gold = os.path.join(ROOT, "tests", "golden", "rmat_cycle4_counts.txt")
        for ln in open(gold):
            f = ln.split()
            if f and not ln.startswith("#") and int(f[0]) == args.cycle4_scale and int(f[1]) == s4.size:
                want4, check4 = int(f[2]), "trace(A^4), stored by tests/golden/make_rmat_cycle4.py"
    if want4 is None:
        want4 = trace_power4(s4, d4)
    assert cyc == want4, (cyc, want4)
    res = {
        "metric": "probe tuples/sec + output tuples/sec, achieved HBM GB/s; learned vs plain plan time",
        "value": probe_tuples / per,
        "unit": "probe tuples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": per * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded R-MAT a=.57 b=.19 c=.19 d=.05)",
        "config": {"workload": f"R-MAT triangle count: 2^{args.rmat_scale} vertices, {src.size} distinct edges, "
                               f"Generic Join plan; 4-cycle count at 2^{args.cycle4_scale}",
                   "edges": int(src.size)},
        "triangles": tri,
        "probes_per_s": probes / per,
        "output_tuples_per_s": tri / per,
        "probe_kernel_ms_per_step": pr_ms / args.steps,
        "probe_launches_per_step": pr_n / args.steps,
        "roofline": probe_roof,
        "phases": {k: v[0] / args.steps for k, v in tim.items() if v[1]},
        "converted_plan_s": conv_s,
        "sampled_x": int(xs.size), "sampled_triangles": want,
        "cycle4": {"scale": args.cycle4_scale, "edges": int(s4.size), "count": cyc, "seconds": cyc_s,
                   "parts": parts,
                   "probes": probes4, "probes_per_s": probes4 / cyc_s, "check": check4},
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(res), flush=True)


def practical_hbm():
    """Read plus write bytes per second of a plain 1 GiB device copy (best
    of five): the bandwidth a streaming kernel reaches on this GPU."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    best = None
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * 4 * n / (best * 1e-3) / 1e9


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, five times: the profiler's
    FETCH_SIZE / WRITE_SIZE for this kernel divided by 1 GiB is the factor
    that turns the counters into bytes."""
    import torch
    n = 1 << 28
    src = torch.arange(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    assert bool((dst[-4:] == src[-4:]).all())
    print(json.dumps({"copy_bytes": 4 * n, "launches": 5}), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "star_10M_scan_probe_pmc.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2301_10841_amd", "csrc", "fj_kernels.hip")


def measured_traffic():
    """HBM bytes per node-0 probe launch from the committed counter summary,
    or None when the kernel source has changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_FILE):
        return None
    m = re.search(r"^traffic_json: (\{.*\})$", open(TRAFFIC_FILE).read(), flags=re.M)
    if not m:
        return None
    t = json.loads(m.group(1))
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if t.get("source_sha256") != src:
        return None
    return t


def bench_batch(args):
    """Batched workload: independent chain / star / triangle queries with
    log-uniform relation sizes (1K..2M rows) and per-query Zipf skew, counted
    together.  One step = one replay of the captured graph: every COLT
    rebuilt, then one persistent kernel for all queries.  Reports aggregate
    first-node (probe) tuples per second and queries per second, beside the
    same queries run one by one through fj_execute."""
    import torch

    import datagen
    from paper_2301_10841_amd import autotune, fj, runner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ctx = fj.Context(0)

    def load(seed, n):
        t0 = time.time()
        qs, redraws = datagen.batch_mix(seed, n_queries=n)
        items, rows, kinds, devs = [], [], [], []
        for dq in qs:
            d = runner.DeviceQuery(ctx, dq)
            plan = d.plan_binary(list(range(len(dq.atoms))), True)
            colts = d.build(plan)
            items.append((d.q, plan, colts))
            rows.append(dq.relations[dq.atoms[0][0]].nrows)
            kinds.append(dq.kind)
            devs.append(d)
        log(f"loaded {n} queries ({sum(r.nrows for q in qs for r in q.relations)} rows, {redraws} redraws) "
            f"in {time.time() - t0:.1f}s")
        return items, rows, kinds, devs

    # tune on a calibration batch drawn with another seed
    cal_items, cal_rows, _, _ = load(datagen.seed_for(4, 99), args.tune_queries)
    setting = autotune.tune(ctx, cal_items, cal_rows, reps=3, log=log)
    log(f"tuned: {setting}")
    for _, _, cs in cal_items:
        for c in cs:
            c.free()
    del cal_items

    items, rows, kinds, devs = load(datagen.seed_for(4, args.seed_rep), args.queries)
    # one by one: rebuild + execute per query
    for _ in range(max(1, args.warmup)):
        seq_counts = []
        for d, (q, plan, colts) in zip(devs, items):
            d.rebuild(colts)
            seq_counts.append(ctx.execute(q, plan, colts)[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, (q, plan, colts) in zip(devs, items):
        d.rebuild(colts)
        ctx.execute(q, plan, colts)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0

    b = fj.Batch(ctx, items, block=setting["block"], query_chunk=autotune.chunks_for(setting, rows))
    for _ in range(args.warmup):
        got = b.run()
    assert got == seq_counts, "batched counts differ from single-query counts"
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    per = elapsed / args.steps
    n0 = sum(rows)
    res = {
        "metric": "probe tuples/sec + output tuples/sec, achieved HBM GB/s; learned vs plain plan time",
        "value": n0 / per,
        "unit": "probe tuples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": per * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded batched mix)",
        "config": {"workload": f"batched: {args.queries} queries (30% chains, 30% stars of 3-6 relations, "
                               f"40% triangles), rows log-uniform 1K-2M, Zipf s in [0,1.5], count only",
                   "queries": args.queries, "first_node_rows": n0},
        "queries_per_s": args.queries / per,
        "output_tuples_per_s": sum(got) / per,
        "sequential_ms": seq_s * 1e3,
        "speedup_vs_sequential": seq_s / per,
        "tuned": setting,
        "cpu_baseline": None,
    }
    b.free()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
