"""Autotuner for the batched executor.

The batched kernel's two knobs are the vector batch of a work item (first-node
rows per item: how many cover tuples one workgroup takes before moving on, the
GPU counterpart of the paper's vectorized batch size, Section 4.3) and the
workgroup size.  No single batch size wins everywhere (the paper's batch-size
ablation finds small batches better for short queries and large ones for long
queries), so the tuner picks a chunk per size bucket of first-node rows, by
coordinate descent on the executor's own measured run time.

Tuned settings can be kept in a JSON cache keyed by the workload signature.
"""

from __future__ import annotations

import json
import math
import os
import statistics
import time
from typing import Dict, List, Optional, Sequence, Tuple

from . import fj

CHUNKS = (64, 128, 256, 512, 1024, 2048, 4096)
BLOCKS = (64, 128, 256, 512)


def size_bucket(rows: int) -> int:
    """Buckets of first-node rows: < 4K, < 32K, < 256K, < 2M, larger."""
    if rows <= 0:
        return 0
    return min(4, max(0, int(math.log(rows, 8)) - 3))


def time_batch(ctx, items, chunks: Sequence[int], block: int, reps: int = 3) -> float:
    b = fj.Batch(ctx, items, block=block, query_chunk=list(chunks))
    try:
        b.run()                                   # warm-up
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            b.run()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)
    finally:
        b.free()


def tune(ctx, items, first_rows: Sequence[int], reps: int = 3, log=None,
         chunks=CHUNKS, blocks=BLOCKS) -> Dict:
    """Returns {"block": B, "chunk_by_bucket": {bucket: chunk}, "seconds": t}."""
    buckets = [size_bucket(r) for r in first_rows]
    present = sorted(set(buckets))
    choice = {bk: 1024 for bk in present}

    def per_query():
        return [choice[bk] for bk in buckets]

    best_block, best_t = None, float("inf")
    for blk in blocks:
        t = time_batch(ctx, items, per_query(), blk, reps)
        if log:
            log(f"block {blk}: {t * 1e3:.2f} ms")
        if t < best_t:
            best_block, best_t = blk, t
    for bk in present:
        for ch in chunks:
            if ch == choice[bk]:
                continue
            old = choice[bk]
            choice[bk] = ch
            t = time_batch(ctx, items, per_query(), best_block, reps)
            if log:
                log(f"bucket {bk} chunk {ch}: {t * 1e3:.2f} ms")
            if t < best_t:
                best_t = t
            else:
                choice[bk] = old
    return {"block": best_block, "chunk_by_bucket": {str(k): v for k, v in choice.items()}, "seconds": best_t}


def chunks_for(setting: Dict, first_rows: Sequence[int]) -> List[int]:
    cb = setting["chunk_by_bucket"]
    return [int(cb.get(str(size_bucket(r)), 1024)) for r in first_rows]


class TuneCache:
    """JSON cache of tuned settings keyed by a workload signature."""

    def __init__(self, path: Optional[str]):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    @staticmethod
    def signature(kinds: Sequence[str], first_rows: Sequence[int]) -> str:
        hist = {}
        for k, r in zip(kinds, first_rows):
            key = f"{k.rstrip('0123456789')}:{size_bucket(r)}"
            hist[key] = hist.get(key, 0) + 1
        return ";".join(f"{k}={hist[k]}" for k in sorted(hist))

    def get(self, sig: str):
        return self.data.get(sig)

    def put(self, sig: str, setting: Dict):
        self.data[sig] = setting
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
