"""The five synthetic workloads (inputs only), plus scaled-down variants for tests.

* ``nemo``: NEMO Phase II-like tower, 32 PMTs on 8 floors x 4, floors 40 m
  apart, 6 m arms; one 200 ms slice at 55 kHz per PMT (about 352k hits) with 5
  injected muon tracks.  Shape from Sec. 2 and Sec. 5 (first simulation).
* ``km3``: KM3Net-It-like tower, 84 PMTs on 14 floors x 6, floors 20 m apart,
  8 m arms; one 200 ms slice at 55 kHz (about 924k hits), 20 tracks.  Shape
  from Sec. 5 (second simulation).
* ``batch``: 256 uneven slices mixing both towers; lengths U[50, 200] ms,
  rates U[50, 150] kHz per PMT; 10 % of slices carry a 1 MHz burst on one PMT
  for 20 ms (bioluminescence, Sec. 4.1).
* ``block``: 32 towers x 84 PMTs (2688 PMTs) on a 4 x 8 grid of 90 m pitch,
  one 200 ms slice at 55 kHz (about 30M hits), 1 % of PMTs bursting at 1 MHz
  for 20 ms, 200 tracks.  The dense 2688^2 threshold table is part of the input.
* ``serving``: a pool of 84-PMT slices at U[50, 150] kHz with 2 % of slices at
  5x rate (the 5x design margin of Sec. 4.1), replayed by the serving loop.

Default trigger parameters (the paper gives the rule shapes, these numbers
follow the workload definition): charge seed at 3 pe (300 in 0.01 pe),
same-floor coincidence within 20 ns, causal window capped at 3000 ns (Sec. 3:
muon light arrives within 3 us), 4-fold trigger, +-3 us event window
(Sec. 2: a 6 us window centred on the trigger seed).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import geometry as G
from .slices import T0_EPOCH_NS, Slice, make_slice

SLICE_NS = 200_000_000
RATE_HZ = 55_000.0

DEFAULT_PARAMS = dict(q_seed=300, t_floor_ns=20, w_ns=3000, min_fold=4, half_event_ns=3000)


@dataclass
class Workload:
    name: str
    geoms: dict          # key -> (Geometry, thr uint32 [P,P])
    slices: list         # list of (geom_key, Slice)
    params: dict


_GEOM_CACHE: dict = {}


def _draw_all(jobs, workers=None):
    """Run ``make_slice`` jobs (tuples of args and kwargs) on a thread pool; every
    slice has its own random streams, so the result does not depend on the pool."""
    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda j: make_slice(*j[0], **j[1]), jobs))


def geometry(key: str):
    """``(Geometry, thr)`` for ``nemo``, ``km3`` or ``block``; cached."""
    if key not in _GEOM_CACHE:
        g = {"nemo": G.nemo_tower, "km3": G.km3net_it_tower, "block": G.block}[key]()
        _GEOM_CACHE[key] = (g, G.thr_table(g))
    return _GEOM_CACHE[key]


def nemo(seed: int = 0, length_ns: int = SLICE_NS, n_tracks: int = 5, order: str = "runs") -> Workload:
    g, thr = geometry("nemo")
    s = make_slice(g, length_ns, RATE_HZ, seed, n_tracks=n_tracks, order=order)
    return Workload("nemo-32pmt-200ms", {"nemo": (g, thr)}, [("nemo", s)], dict(DEFAULT_PARAMS))


def km3(seed: int = 1, length_ns: int = SLICE_NS, n_tracks: int = 20, order: str = "runs") -> Workload:
    g, thr = geometry("km3")
    s = make_slice(g, length_ns, RATE_HZ, seed, n_tracks=n_tracks, order=order)
    return Workload("km3net-it-84pmt-200ms", {"km3": (g, thr)}, [("km3", s)], dict(DEFAULT_PARAMS))


def batch_specs(seed: int = 2, n_slices: int = 256, len_ms=(50.0, 200.0), rate_khz=(50.0, 150.0),
                burst_frac: float = 0.10):
    """Per-slice recipe of the batched workload (tower, length, rate, burst, tracks, seed)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    specs = []
    for i in range(n_slices):
        key = "nemo" if rng.random() < 0.5 else "km3"
        P = 32 if key == "nemo" else 84
        L = int(round(rng.uniform(*len_ms) * 1e6))
        R = float(rng.uniform(*rate_khz) * 1e3)
        bursts = []
        if rng.random() < burst_frac:
            bp = int(rng.integers(0, P))
            dur = min(20_000_000, L)
            start = int(rng.integers(0, max(1, L - dur + 1)))
            bursts.append((bp, 1.0e6, start, dur))
        dens = 25.0 if key == "nemo" else 100.0      # tracks per second, as nemo / km3
        n_tr = int(round(dens * L * 1e-9))
        specs.append(dict(key=key, length_ns=L, rate_hz=R, bursts=bursts, n_tracks=n_tr,
                          seed=[seed, i], t0=T0_EPOCH_NS + i * SLICE_NS))
    return specs


def batch(seed: int = 2, n_slices: int = 256, scale: float = 1.0, order: str = "runs") -> Workload:
    """Batched workload; ``scale`` < 1 shortens every slice (tests)."""
    geoms = {k: geometry(k) for k in ("nemo", "km3")}
    jobs, keys = [], []
    for sp in batch_specs(seed, n_slices):
        L = max(1000, int(sp["length_ns"] * scale))
        bursts = [(bp, br, int(bs * scale), max(1, int(bd * scale))) for (bp, br, bs, bd) in sp["bursts"]]
        g, _ = geoms[sp["key"]]
        jobs.append(((g, L, sp["rate_hz"], sp["seed"]),
                     dict(t0=sp["t0"], n_tracks=sp["n_tracks"] if scale >= 0.05 else 0, bursts=bursts, order=order)))
        keys.append(sp["key"])
    out = list(zip(keys, _draw_all(jobs)))
    return Workload("batch-256-mixed", geoms, out, dict(DEFAULT_PARAMS))


def block_workload(seed: int = 3, length_ns: int = SLICE_NS, n_tracks: int = 200,
                   burst_frac: float = 0.01) -> Workload:
    g, thr = geometry("block")
    P = g.n_pmt
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    nb = int(round(burst_frac * P))
    bps = rng.choice(P, size=nb, replace=False)
    dur = min(20_000_000, length_ns)
    bursts = [(int(p), 1.0e6, int(rng.integers(0, max(1, length_ns - dur + 1))), dur) for p in bps]
    s = make_slice(g, length_ns, RATE_HZ, seed, n_tracks=n_tracks, bursts=bursts)
    return Workload("block-32x84pmt-200ms", {"block": (g, thr)}, [("block", s)], dict(DEFAULT_PARAMS))


def serving_pool(seed: int = 4, n_pool: int = 256, length_ns: int = SLICE_NS, burst_frac: float = 0.02):
    """Pool of 84-PMT slices for the serving loop: rate U[50,150] kHz, 2 % at 5x."""
    g, thr = geometry("km3")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 13])))
    jobs = []
    for i in range(n_pool):
        R = float(rng.uniform(50e3, 150e3))
        if rng.random() < burst_frac:
            R *= 5.0
        jobs.append(((g, length_ns, R, [seed, i]),
                     dict(t0=T0_EPOCH_NS + i * length_ns, n_tracks=max(0, int(round(20 * length_ns / SLICE_NS))))))
    out = [("km3", s) for s in _draw_all(jobs)]
    return Workload("serving-16x84pmt", {"km3": (g, thr)}, out, dict(DEFAULT_PARAMS))
