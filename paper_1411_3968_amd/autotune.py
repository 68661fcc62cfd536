"""Autotuner of the ordering stage's launch parameters.

The knobs (``trig_tune``): the LDS capacity of one time segment (2048, 4096 or
8192 hits, a compiled kernel variant), the expected hits per segment (which
sets the segment width 2^s ns of a slice from its density), and the number of
persistent workgroups per compute unit.  Each PMT-count class is tuned on
representative slices by timing the whole pipeline (``trig_batch``), and the
choice is kept in a JSON cache keyed by the class.  Correctness never depends
on the choice: every setting gives byte-identical results.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import trig as T

DEFAULT_CANDIDATES = [
    (cap, tgt, g)
    for cap in (2048, 4096, 8192)
    for tgt in (cap // 8, cap // 4, cap // 2)
    for g in (1, 2, 4)
    if not (cap == 8192 and g > 1)          # one 8192-hit segment fills most of a CU's LDS
]


def _time_batch(ctx, slices, params, reps: int, stream=None) -> float:
    T.trig_batch(ctx, slices, params, stream=stream)      # warm-up (workspace, graph capture)
    T.trig_batch(ctx, slices, params, stream=stream)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        T.trig_batch(ctx, slices, params, stream=stream)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune_class(ctx, n_pmt_max: int, slices, params, candidates=None, reps: int = 5, stream=None, log=None) -> dict:
    """Try every candidate on ``slices`` (list of (geom_id, pmt, t, q)); keep the fastest."""
    best = None
    trials = []
    for (cap, tgt, g) in candidates or DEFAULT_CANDIDATES:
        T.trig_tune_set(ctx, n_pmt_max, tgt, cap, g)
        dt = _time_batch(ctx, slices, params, reps, stream)
        trials.append(dict(seg_cap=cap, seg_target=tgt, grid_per_cu=g, s=dt))
        if log:
            log(f"n_pmt<={n_pmt_max} cap={cap} target={tgt} grid/CU={g}: {dt * 1e3:.3f} ms")
        if best is None or dt < best["s"]:
            best = trials[-1]
    T.trig_tune_set(ctx, n_pmt_max, best["seg_target"], best["seg_cap"], best["grid_per_cu"])
    return dict(n_pmt_max=n_pmt_max, best=best, trials=trials)


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
