"""Autotuner of the ordering stage's launch parameters.

The knobs (``trig_tune``): the ordering kernel and its LDS capacity per time
segment (256 or 512 hits: one wave per segment; 2048, 4096 or 8192 hits: one
workgroup per segment, compiled variants), the expected hits per segment (which sets the
segment width 2^s ns of a slice from its density), and the number of persistent
workgroups per compute unit.  Each PMT-count class is tuned on representative
slices by timing the whole pipeline (``trig_batch`` with marshalling done once),
and the choice is kept in a JSON cache keyed by the class.  Correctness never
depends on the choice: every setting gives byte-identical results.
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


def tune_class(ctx, n_pmt_max: int, slices, params, candidates=None, reps: int = 5, stream=None, log=None,
               time_budget_s: float | None = None) -> dict:
    """Try the candidates on ``slices`` (list of (geom_id, pmt, t, q)); keep the
    fastest.  With ``time_budget_s`` the search stops once that much time is spent
    (the candidates tried so far decide)."""
    best = None
    trials = []
    t_start = time.perf_counter()
    for (cap, tgt, g) in candidates or DEFAULT_CANDIDATES:
        if time_budget_s is not None and trials and time.perf_counter() - t_start > time_budget_s:
            break
        T.trig_tune_set(ctx, n_pmt_max, tgt, cap, g)
        dt = _time_batch(ctx, slices, params, reps, stream)
        trials.append(dict(seg_cap=cap, seg_target=tgt, grid_per_cu=g, s=dt))
        if log:
            log(f"n_pmt<={n_pmt_max} cap={cap} target={tgt} grid/CU={g}: {dt * 1e3:.3f} ms")
        if best is None or dt < best["s"]:
            best = trials[-1]
    T.trig_tune_set(ctx, n_pmt_max, best["seg_target"], best["seg_cap"], best["grid_per_cu"])
    return dict(n_pmt_max=n_pmt_max, best=best, trials=trials, seconds=time.perf_counter() - t_start)


def save(path: str, results: list, device: str = "") -> None:
    doc = dict(device=device, classes=[dict(n_pmt_max=r["n_pmt_max"], **{k: r["best"][k] for k in
                                                                        ("seg_cap", "seg_target", "grid_per_cu")})
                                       for r in results])
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)


def apply(ctx, path: str) -> list:
    """Load a JSON cache written by :func:`save` and set it on the context."""
    with open(path) as f:
        doc = json.load(f)
    for c in doc["classes"]:
        T.trig_tune_set(ctx, int(c["n_pmt_max"]), int(c["seg_target"]), int(c["seg_cap"]), int(c["grid_per_cu"]))
    return doc["classes"]
