"""Autotuner of the batched matrix pipeline's launch shape.

Candidates: workgroup output tile (64 or 128) x sketch work items per pass
(target_blocks) x bytes of gathered operands per pass (gather_budget: the
larger budget means fewer, larger passes and fewer merges of the level
state), and the single-launch form at either tile (batches it is not built
for plan the launch-per-pass form for it).  Each candidate runs the batch's whole ladder with a quarter of every
level's realisations on the GPU (warm-up, then timed with HIP events via
torch on the current stream); the fastest is cached in a JSON file keyed by
a signature of the batch (precision, ladder head, per-product shapes bucketed
to powers of two), so later runs with a similar batch reuse it without
timing."""
from __future__ import annotations

import hashlib
import json
import os
from typing import Sequence

import torch

from .mlmc import BatchedEstimate, BatchProblem

CANDIDATES = [{"tile": t, "target_blocks": b, "gather_budget": g, "single_launch": 0}
              for t in (64, 128) for b in (1024, 4096) for g in (192 << 20, 768 << 20)] + \
             [{"tile": t, "target_blocks": 0, "gather_budget": 768 << 20, "single_launch": 1} for t in (64, 128)]


def cache_path() -> str:
    return os.environ.get("MLMC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mlmc_autotune.json"))


def signature(problems: Sequence[BatchProblem], c: Sequence[int], prec: str) -> str:
    def bucket(x):
        return 1 << max(0, (int(x) - 1).bit_length())
    shapes = sorted((bucket(p.m), bucket(p.p)) for p in problems)
    key = json.dumps({"prec": prec, "c": list(c)[:2], "levels": len(c), "shapes": shapes})
    return hashlib.sha256(key.encode()).hexdigest()[:24]


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(table: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1)
    os.replace(tmp, path)


def tune(problems: Sequence[BatchProblem], c: Sequence[int], n_samples: Sequence[int], prec: str = "fp32",
         device=None, repeats: int = 2, use_cache: bool = True) -> dict:
    """Return the fastest {"tile", "target_blocks", "gather_budget"} for this batch."""
    sig = signature(problems, c, prec)
    table = _load() if use_cache else {}
    if sig in table:
        return table[sig]["best"]
    # time the whole ladder with a quarter of every level's realisations (at
    # least 2), so that every level's pass shape weighs in
    probe_c, probe_n = list(c), [max(2, int(x) // 4) for x in n_samples]
    timings = []
    for cand in CANDIDATES:
        est = BatchedEstimate(problems, probe_c, probe_n, seed=0, prec=prec, tuning=cand, device=device)
        est.run()
        torch.cuda.synchronize(est.device)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(repeats):
            est.run()
        stop.record()
        stop.synchronize()
        timings.append((start.elapsed_time(stop) / repeats, cand))
        del est
    best = min(timings, key=lambda t: t[0])[1]
    table[sig] = {"best": best, "timings_ms": [[t, cd] for t, cd in timings]}
    if use_cache:
        _store(table)
    return best
