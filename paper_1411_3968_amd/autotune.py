"""Autotuner of the pipeline's launch parameters.

The knobs (``trig_tune``): the ordering kernel and its LDS capacity per time
segment (256 or 512 hits: one wave per segment; 2048, 4096 or 8192 hits: one
workgroup per segment, compiled variants), the expected hits per segment (which sets the
segment width 2^s ns of a slice from its density), the number of persistent
workgroups per compute unit, and the fold stage's tiles per workgroup and the
window seeds it stages in LDS (the paper sizes its sub-slices per GPU thread,
Sec. 4.1).  Each
PMT-count class is tuned on representative slices (a held-out sample, not the
timed workload) by timing the whole pipeline (``trig_batch`` with marshalling
done once): first the ordering knobs, then the fold knobs with the best
ordering.  The choice is kept in a JSON cache keyed by the class.  Correctness
never depends on the choice: every setting gives byte-identical results.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import trig as T

WAVE_CAP = 512
WAVE_CAP_SMALL = 256

DEFAULT_CANDIDATES = (
    [(WAVE_CAP, tgt, g) for tgt in (192, 256, 320, 384) for g in (2, 3, 4)] +
    [(WAVE_CAP_SMALL, tgt, g) for tgt in (128, 160, 192) for g in (4, 5)] +
    [(cap, tgt, g) for cap in (2048, 4096) for tgt in (cap // 4, cap // 2) for g in (1, 2, 4)]
)


def _time_batch(ctx, slices, params, reps: int, stream=None) -> float:
    first = T.trig_batch(ctx, slices, params, stream=stream)     # sizes the result lists
    caps = [(max(1, r["n_fires"]), max(1, r["n_events"])) for r in first]
    run = T.BatchRunner(ctx, slices, params, stream=stream, caps=caps)
    run()                                                        # graph capture
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


COUNT_CANDIDATES = [(g, h) for g in (1, 2, 4) for h in (512, 2048)]
KNOBS = ("seg_cap", "seg_target", "grid_per_cu", "tile_group", "window_cap")


def tune_class(ctx, n_pmt_max: int, slices, params, candidates=None, reps: int = 9, stream=None, log=None,
               time_budget_s: float | None = None, count_candidates=None) -> dict:
    """Try the candidates on ``slices`` (list of (geom_id, pmt, t, q)); keep the
    fastest.  First the ordering knobs ``candidates`` (cap, target, grid per CU)
    with the class's fold knobs, then the fold knobs ``count_candidates``
    (tiles per workgroup, window seeds in LDS) with the best ordering.  With
    ``time_budget_s`` each stage stops once that much time is spent (the
    candidates tried so far decide)."""
    cur = T.trig_tune_get(ctx, n_pmt_max)
    best = None
    trials = []
    t_start = time.perf_counter()

    def trial(k):
        T.trig_tune_set(ctx, n_pmt_max, k["seg_target"], k["seg_cap"], k["grid_per_cu"], k["tile_group"],
                        k["window_cap"])
        dt = _time_batch(ctx, slices, params, reps, stream)
        trials.append(dict(k, s=dt))
        if log:
            log(f"n_pmt<={n_pmt_max} " + " ".join(f"{x}={k[x]}" for x in KNOBS) + f": {dt * 1e3:.3f} ms")
        return trials[-1]

    for (cap, tgt, g) in candidates or DEFAULT_CANDIDATES:
        if time_budget_s is not None and trials and time.perf_counter() - t_start > time_budget_s:
            break
        r = trial(dict(seg_cap=cap, seg_target=tgt, grid_per_cu=g, tile_group=cur["tile_group"],
                       window_cap=cur["window_cap"]))
        if best is None or r["s"] < best["s"]:
            best = r
    t_mid = time.perf_counter()
    for (tg, h) in count_candidates or COUNT_CANDIDATES:
        if time_budget_s is not None and time.perf_counter() - t_mid > time_budget_s:
            break
        if (tg, h) == (best["tile_group"], best["window_cap"]):
            continue
        r = trial(dict({k: best[k] for k in ("seg_cap", "seg_target", "grid_per_cu")}, tile_group=tg, window_cap=h))
        if r["s"] < best["s"]:
            best = r
    T.trig_tune_set(ctx, n_pmt_max, *(best[k] for k in ("seg_target", "seg_cap", "grid_per_cu", "tile_group",
                                                        "window_cap")))
    return dict(n_pmt_max=n_pmt_max, best=best, trials=trials, seconds=time.perf_counter() - t_start)


def save(path: str, results: list, device: str = "") -> None:
    doc = dict(device=device, classes=[dict(n_pmt_max=r["n_pmt_max"], **{k: r["best"][k] for k in KNOBS})
                                       for r in results])
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)


def apply_one(ctx, c: dict) -> None:
    """Set one class record of a cache (n_pmt_max and the knobs) on the context."""
    T.trig_tune_set(ctx, int(c["n_pmt_max"]), int(c["seg_target"]), int(c["seg_cap"]), int(c["grid_per_cu"]),
                    c.get("tile_group"), c.get("window_cap"))


def apply(ctx, path: str) -> list:
    """Load a JSON cache written by :func:`save` and set it on the context."""
    with open(path) as f:
        doc = json.load(f)
    for c in doc["classes"]:
        apply_one(ctx, c)
    return doc["classes"]
