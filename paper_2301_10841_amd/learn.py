"""Training and evaluation of the learned plan chooser on the executor's own
timings.

For every generated query the candidates of ``fj_plan_candidates`` are timed
through the library (COLT root builds into allocated COLTs, then the join;
median of ``reps`` runs after one warm-up), giving one (feature row, log time)
sample per candidate.  The perceptron (3 layers of width 128, FP32) is fitted
on the GPU by the library's own kernels (``fj_mlp_train_step``) to the
standardized natural log of the time in microseconds.

Evaluation on held-out queries compares, per query and live on the same GPU,
the end-to-end time of
  * plain:   greedy left-deep order + conversion and factoring (Section 4.1)
             + root builds + join, and
  * learned: ``fj_choose_plan`` (candidates, features, GPU inference, the
             plain plan as fallback) + root builds + join,
with the relations' sketches (per-relation statistics, like a catalog's)
computed once beforehand and excluded from both.  It also reports the regret
against the best candidate measured for that query.

Relation contents come from ``datagen.batch_query``; a pool of worker
processes, started before this process touches the GPU, draws them.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "chooser.npz")
HIDDEN = 128


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ query supply

def _draw(args):
    import datagen
    seed, qi, max_rows = args
    q, _ = datagen.batch_query(seed, qi, max_rows=max_rows)
    return qi, q


class QuerySupply:
    """Queries drawn by worker processes, handed out in index order with a
    bounded number in flight.  Create it before any GPU work (the workers
    are forked)."""

    def __init__(self, workers: int):
        import multiprocessing as mp
        self.workers = workers
        self.pool = mp.get_context("fork").Pool(workers) if workers > 0 else None

    def queries(self, seed: int, n: int, max_rows: int = 2_000_000, window: int = 48):
        if self.pool is None:
            for qi in range(n):
                yield _draw((seed, qi, max_rows))[1]
            return
        pending = {}
        nxt = 0
        for qi in range(n):
            while nxt < n and nxt < qi + window:
                pending[nxt] = self.pool.apply_async(_draw, ((seed, nxt, max_rows),))
                nxt += 1
            _, q = pending.pop(qi).get()
            yield q

    def close(self):
        if self.pool is not None:
            self.pool.terminate()
            self.pool.join()
            self.pool = None


# ------------------------------------------------------------------ timing

def sync():
    import torch
    torch.cuda.synchronize()


def time_plan(ctx, d, plan, reps: int, slow_s: float = 0.25):
    """(median seconds of rebuild + execute, count).  Slow plans get one run."""
    colts = d.build(plan)
    try:
        sync()
        t0 = time.perf_counter()
        cnt = ctx.execute(d.q, plan, colts)[0]
        first = time.perf_counter() - t0
        ts = []
        for _ in range(reps if first < slow_s else 1):
            t0 = time.perf_counter()
            d.rebuild(colts)
            c = ctx.execute(d.q, plan, colts)[0]
            ts.append(time.perf_counter() - t0)
            assert c == cnt
        return statistics.median(ts), cnt
    finally:
        for c in colts:
            c.free()


def collect(ctx, supply: QuerySupply, seed: int, n: int, reps: int = 5, max_rows: int = 2_000_000,
            tag: str = "train", checkpoint: Optional[str] = None):
    """Per candidate: features, seconds; per query: kind, candidate range,
    count.  Candidates the library refuses (outside its documented limits)
    are skipped and counted.  With ``checkpoint`` the samples so far are
    saved every 512 queries."""
    from . import fj, runner
    feats, secs, qidx, cidx = [], [], [], []
    qinfo = []
    skipped = 0
    t_start = time.time()
    for qi, dq in enumerate(supply.queries(seed, n, max_rows)):
        d = runner.DeviceQuery(ctx, dq)
        sks = d.sketches()
        cands, f = d.candidates(sks)
        counts = set()
        for ci, c in enumerate(cands):
            plan = d.candidate_plan(c)
            try:
                s, cnt = time_plan(ctx, d, plan, reps)
            except fj.FJError as e:
                if e.status not in (-1, -6) or ci == 0:
                    raise
                skipped += 1
                continue
            counts.add(cnt)
            feats.append(f[ci])
            secs.append(s)
            qidx.append(qi)
            cidx.append(ci)
        if len(counts) != 1:
            raise RuntimeError(f"{tag} query {qi}: candidate plans disagree on the count: {counts}")
        qinfo.append({"kind": dq.kind, "ncand": len(cands), "count": counts.pop(),
                      "rows": [r.nrows for r in dq.relations],
                      "atom_rows": int(sum(dq.atom_rows(a) for a in range(len(dq.atoms))))})
        del d
        if (qi + 1) % 64 == 0 or qi + 1 == n:
            log(f"[{tag}] {qi + 1}/{n} queries, {len(secs)} timed plans, {skipped} skipped, "
                f"{time.time() - t_start:.0f}s")
        if checkpoint and ((qi + 1) % 512 == 0 or qi + 1 == n):
            np.savez(checkpoint, x=np.array(feats, np.float32), sec=np.array(secs, np.float64),
                     q=np.array(qidx, np.int32), c=np.array(cidx, np.int32),
                     kind=np.array([qi_["kind"] for qi_ in qinfo]), count=np.array([qi_["count"] for qi_ in qinfo]))
    return {"x": np.array(feats, np.float32), "sec": np.array(secs, np.float64),
            "q": np.array(qidx, np.int32), "c": np.array(cidx, np.int32), "queries": qinfo, "skipped": skipped}


# ---------------------------------------------------------------- training

def targets(sec: np.ndarray) -> np.ndarray:
    return np.log(np.maximum(sec, 1e-7) * 1e6)


def train(ctx, data: Dict, epochs: int = 60, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          val_frac: float = 0.1):
    """Fit the perceptron on the GPU; returns (Mlp, info)."""
    import torch
    from . import fj
    from . import mlp_init
    rng = np.random.default_rng(seed)
    y = targets(data["sec"])
    mu, sd = float(y.mean()), float(y.std() + 1e-9)
    t = ((y - mu) / sd).astype(np.float32)
    nq = int(data["q"].max()) + 1
    val_q = set(rng.choice(nq, size=max(1, int(nq * val_frac)), replace=False).tolist())
    is_val = np.array([q in val_q for q in data["q"]])
    tr = np.flatnonzero(~is_val)
    dev = f"cuda:{ctx.device}"
    x_all = torch.from_numpy(data["x"]).to(dev)
    t_all = torch.from_numpy(t).to(dev)
    x_tr, t_tr = x_all[tr].contiguous(), t_all[tr].contiguous()
    m = fj.Mlp(ctx, fj.FEATURES, HIDDEN)
    m.set_params(mlp_init.he_init(rng, fj.FEATURES, HIDDEN))
    n = len(tr)
    hist = []
    t0 = time.time()
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    for ep in range(epochs):
        step_lr = lr * (0.1 if ep >= int(0.8 * epochs) else (0.3 if ep >= int(0.6 * epochs) else 1.0))
        perm = torch.randperm(n, generator=g).to(dev)
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            m.train_step(x_tr[idx].contiguous(), t_tr[idx].contiguous(), step_lr)
        if ep % 10 == 9 or ep == epochs - 1:
            _, ltr = m.gradient(x_tr, t_tr)
            pred = m.forward(x_all).cpu().numpy()
            vr = selection_quality(data, pred, is_val)
            hist.append({"epoch": ep + 1, "train_mse": ltr, **vr})
            log(f"epoch {ep + 1}: train mse {ltr:.4f}, val regret {vr['val_mean_regret']:.3f}, "
                f"val time ratio {vr['val_time_ratio']:.3f}")
    info = {"mu": mu, "sd": sd, "epochs": epochs, "batch": batch, "lr": lr, "train_rows": int(n),
            "val_queries": len(val_q), "history": hist, "train_seconds": time.time() - t0}
    info["val_mask_queries"] = sorted(int(q) for q in val_q)
    info["_pred"] = m.forward(x_all).cpu().numpy()
    return m, info


def fit_gate(data: Dict, pred: np.ndarray, val_queries, oh_plain: float, oh_learn: float) -> Dict:
    """The row gate and the score margin of fj_choose_plan fitted on the
    validation queries: with the choice overheads measured live (oh_plain:
    the plain plan alone; oh_learn: enumeration, features and inference), a
    query with fewer than G rows takes the plain plan at oh_plain; any other
    takes the predicted best at oh_learn when its predicted score is at least
    M below the plain plan's, else the plain plan.  (G, M) minimizes the
    validation queries' total end-to-end time."""
    q = data["q"]
    per = []
    for qi in val_queries:
        rows = np.flatnonzero(q == qi)
        if rows.size == 0:
            continue
        s = data["sec"][rows]
        pr = pred[rows]
        k = int(np.argmin(pr))
        per.append((data["queries"][qi]["atom_rows"], s[0], s[k], float(pr[0] - pr[k])))
    if not per:
        return {"gate_rows": 0, "margin": 0.0}
    per.sort()
    best = None
    for margin in [0.0, 0.05, 0.1, 0.15, 0.2, 0.3, 0.4, 0.6, 0.8]:
        learned = [(r, p + oh_plain, (l if d >= margin else p) + oh_learn) for r, p, l, d in per]
        for g in [0] + [r + 1 for r, _, _ in learned]:
            t = sum(p if r < g else l for r, p, l in learned)
            if best is None or t < best[0]:
                best = (t, g, margin)
    t0 = sum(l + oh_learn for _, _, l, _ in per)
    return {"gate_rows": int(best[1]), "margin": float(best[2]), "val_total_gated_s": best[0],
            "val_total_ungated_s": t0, "oh_plain_s": oh_plain, "oh_learn_s": oh_learn, "val_queries": len(per)}


# Choice overheads are a few to a few tens of microseconds of host time, so
# each is timed over many alternating repetitions after one untimed call of
# each (first calls pay for cold caches), and the median is taken.
CHOICE_REPS = 15


def choice_times(fj, d, m, sks, margin: float, gate_rows: int, reps: int):
    """Seconds of each repetition of the plain choice (greedy order,
    converted and factored) and of the learned one, alternating."""
    fj.plan_from_binary(d.q, fj.greedy_order(d.q, sks), True)
    d.choose(m, sks, margin, gate_rows)
    tp, tl = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        p = fj.plan_from_binary(d.q, fj.greedy_order(d.q, sks), True)
        del p
        tp.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        r = d.choose(m, sks, margin, gate_rows)
        del r
        tl.append(time.perf_counter() - t0)
    return tp, tl


def choice_overheads(ctx, m, supply, seed: int, n: int, reps: int, max_rows: int):
    """Median seconds of the plain choice and of the ungated learned choice
    over n queries (sketches computed beforehand, as a catalog's)."""
    from . import fj, runner
    tp, tl = [], []
    for dq in supply.queries(seed, n, max_rows):
        d = runner.DeviceQuery(ctx, dq)
        sks = d.sketches()
        a, b = choice_times(fj, d, m, sks, 0.0, 0, max(reps, CHOICE_REPS))
        tp += a
        tl += b
        del d
    return statistics.median(tp), statistics.median(tl)


def selection_quality(data: Dict, pred: np.ndarray, mask: np.ndarray) -> Dict:
    """On the queries selected by mask: chosen / plain time ratio (sums) and
    mean regret (chosen / best - 1) when choosing the argmin prediction."""
    tot_plain = tot_chosen = 0.0
    regrets = []
    q = data["q"]
    for qi in np.unique(q[mask]):
        rows = np.flatnonzero(q == qi)
        s = data["sec"][rows]
        k = int(np.argmin(pred[rows]))
        tot_plain += s[0]
        tot_chosen += s[k]
        regrets.append(s[k] / s.min() - 1.0)
    return {"val_time_ratio": tot_chosen / max(tot_plain, 1e-30), "val_mean_regret": float(np.mean(regrets))}


def save(m, info: Dict, path: str):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=m.get_params(), in_dim=m.in_dim, hidden=m.hidden,
             info=json.dumps(info))
    os.replace(tmp, path)


def load(ctx, path: str = DEFAULT_WEIGHTS):
    """(Mlp, info) from a weights file written by ``save``."""
    from . import fj
    z = np.load(path, allow_pickle=False)
    m = fj.Mlp(ctx, int(z["in_dim"]), int(z["hidden"]))
    m.set_params(z["params"])
    return m, json.loads(str(z["info"]))


# -------------------------------------------------------------- evaluation

def evaluate(ctx, m, supply: QuerySupply, seed: int, n: int, reps: int = 5, margin: float = 0.0,
             max_rows: int = 2_000_000, tag: str = "heldout", out_npz: Optional[str] = None,
             gate_rows: int = 0):
    """Per held-out query: every candidate timed (root builds + join, median
    of reps), the choice overheads of the plain and the learned choosers
    timed live (median of reps), and the learned chooser's pick.  End-to-end
    time = choice + the chosen plan's time."""
    from . import fj, runner
    rows = []
    feats, secs, qidx = [], [], []
    t_start = time.time()
    for qi, dq in enumerate(supply.queries(seed, n, max_rows)):
        d = runner.DeviceQuery(ctx, dq)
        sks = d.sketches()
        cands, f = d.candidates(sks)
        times = []
        counts = set()
        for c in cands:
            try:
                s, cnt = time_plan(ctx, d, d.candidate_plan(c), reps)
            except fj.FJError as e:
                if e.status not in (-1, -6) or not times:
                    raise
                s, cnt = float("inf"), None
            times.append(s)
            if cnt is not None:
                counts.add(cnt)
        assert len(counts) == 1, (qi, counts)
        tc_plain, tc_learn = choice_times(fj, d, m, sks, margin, gate_rows, CHOICE_REPS)
        _, k, _ = d.choose(m, sks, margin, gate_rows)
        rows.append({"kind": dq.kind, "chosen": k, "ncand": len(cands), "count": counts.pop(),
                     "atom_rows": int(sum(dq.atom_rows(a) for a in range(len(dq.atoms)))),
                     "choose_plain_s": statistics.median(tc_plain), "choose_learned_s": statistics.median(tc_learn),
                     "run_plain_s": times[0], "run_learned_s": times[k], "best_s": min(times)})
        for ci in range(len(cands)):
            if math.isfinite(times[ci]):
                feats.append(f[ci]); secs.append(times[ci]); qidx.append(qi)
        del d
        if (qi + 1) % 64 == 0 or qi + 1 == n:
            log(f"[{tag}] {qi + 1}/{n} queries, {time.time() - t_start:.0f}s")
            if out_npz:
                np.savez(out_npz, x=np.array(feats, np.float32), sec=np.array(secs), q=np.array(qidx, np.int32))
    return rows


def summarize(rows: List[Dict]) -> Dict:
    e_plain = np.array([r["choose_plain_s"] + r["run_plain_s"] for r in rows])
    e_learn = np.array([r["choose_learned_s"] + r["run_learned_s"] for r in rows])
    best = np.array([r["best_s"] for r in rows])
    ratio = e_learn / e_plain
    out = {
        "queries": len(rows),
        "plain_total_s": float(e_plain.sum()),
        "learned_total_s": float(e_learn.sum()),
        "learned_over_plain_total": float(e_learn.sum() / e_plain.sum()),
        "learned_over_plain_geomean": float(np.exp(np.mean(np.log(ratio)))),
        "learned_mean_regret_vs_best": float(np.mean(np.array([r["run_learned_s"] for r in rows]) / best - 1)),
        "plain_mean_regret_vs_best": float(np.mean(np.array([r["run_plain_s"] for r in rows]) / best - 1)),
        "chose_other_than_plain": int(sum(r["chosen"] != 0 for r in rows)),
        "wins_gt_5pct": int(np.sum(ratio < 0.95)),
        "losses_gt_5pct": int(np.sum(ratio > 1.05)),
        "ties_within_5pct": int(np.sum((ratio >= 0.95) & (ratio <= 1.05))),
        "choose_learned_ms_mean": float(np.mean([r["choose_learned_s"] for r in rows]) * 1e3),
        "choose_plain_ms_mean": float(np.mean([r["choose_plain_s"] for r in rows]) * 1e3),
    }
    kinds = sorted(set(r["kind"].rstrip("0123456789") for r in rows))
    out["by_kind"] = {}
    for k in kinds:
        sel = [i for i, r in enumerate(rows) if r["kind"].rstrip("0123456789") == k]
        out["by_kind"][k] = {"queries": len(sel), "learned_over_plain_total": float(e_learn[sel].sum() / e_plain[sel].sum())}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--heldout", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--max-rows", type=int, default=2_000_000)
    ap.add_argument("--margin", type=float, default=None, help="score margin (default: the fitted one)")
    ap.add_argument("--train-seed", type=int, default=None)
    ap.add_argument("--heldout-seed", type=int, default=None)
    ap.add_argument("--out", default="chooser_report")
    ap.add_argument("--weights", default=None, help="skip training: evaluate these weights")
    args = ap.parse_args(argv)
    supply = QuerySupply(args.workers)     # fork before the GPU is touched
    import datagen
    import torch
    from . import fj
    torch.cuda.set_device(0)
    ctx = fj.Context(0)
    os.makedirs(args.out, exist_ok=True)
    train_seed = datagen.seed_for(5, 0) if args.train_seed is None else args.train_seed
    held_seed = datagen.seed_for(5, 1) if args.heldout_seed is None else args.heldout_seed
    report = {"train_seed": train_seed, "heldout_seed": held_seed, "reps": args.reps,
              "max_rows": args.max_rows}
    try:
        if args.weights:
            m, info = load(ctx, args.weights)
        else:
            data = collect(ctx, supply, train_seed, args.train, args.reps, args.max_rows,
                           checkpoint=os.path.join(args.out, "train_data.npz"))
            m, info = train(ctx, data, epochs=args.epochs)
            pred = info.pop("_pred")
            val_queries = info.pop("val_mask_queries")
            oh_p, oh_l = choice_overheads(ctx, m, supply, datagen.seed_for(5, 4), 32, args.reps, args.max_rows)
            info["gate"] = fit_gate(data, pred, val_queries, oh_p, oh_l)
            info.update({"train_queries": args.train, "train_seed": train_seed, "features": fj.FEATURES,
                         "hidden": HIDDEN, "target": "standardized ln(microseconds)",
                         "gate_rows": info["gate"]["gate_rows"], "margin": info["gate"]["margin"]})
            log(f"gate: {info['gate']}")
            save(m, info, os.path.join(args.out, "chooser.npz"))
        report["train"] = {k: v for k, v in info.items() if k != "history"}
        report["train_history"] = info.get("history")
        margin = args.margin if args.margin is not None else float(info.get("margin", 0.0))
        rows = evaluate(ctx, m, supply, held_seed, args.heldout, args.reps, margin, args.max_rows,
                        out_npz=os.path.join(args.out, "heldout_data.npz"),
                        gate_rows=int(info.get("gate_rows", 0)))
        report["heldout"] = summarize(rows)
        with open(os.path.join(args.out, "heldout_rows.json"), "w") as f:
            json.dump(rows, f)
        with open(os.path.join(args.out, "report.json"), "w") as f:
            json.dump(report, f, indent=1)
        print(json.dumps(report["heldout"]), flush=True)
    finally:
        supply.close()
        ctx.close()


if __name__ == "__main__":
    main()
