"""Seeded synthetic time slices shaped like the paper's tower data.

Inputs only: this module draws hits and never evaluates the trigger rule.

What the paper fixes (Sec. 2 and Sec. 3): PMT background rates of 50-55 kHz,
about 1.7 Mhits/s per 32-PMT tower and 4.6 Mhits/s per 84-PMT tower, 200 ms
time slices, hit streams that arrive time-ordered per PMT (Sec. 4.2: the data
within a GPU thread is time-ordered per PMT), bioluminescence bursts of 1 MHz
on single PMTs (Sec. 4.1), and Cherenkov light of a muon correlated in time
and space (Sec. 3).  Everything else (charge spectrum, track sampling) is a
stated proposal; see the recipe in ``make_slice``.

Hits are structure-of-arrays: ``pmt`` uint16, ``t`` int64 ns, ``q`` uint16 in
0.01 pe units.  Random streams: ``numpy.random.Generator(PCG64)`` from a
``SeedSequence``, with one child stream per PMT plus one for the tracks, so a
slice is a pure function of its seed and recipe.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .geometry import C_M_PER_NS, N_WATER, Geometry

T0_EPOCH_NS = 1_400_000_000_000_000_000
TAN_CHERENKOV = float(np.sqrt(N_WATER ** 2 - 1.0))   # tan(theta_C) with cos(theta_C) = 1/n


@dataclass
class Track:
    """Ground truth of one injected muon: detected PMTs, jittered times, final positions."""

    pmt: np.ndarray          # int64 [k]
    t: np.ndarray            # int64 [k] (as stored in the slice)
    q: np.ndarray            # int64 [k]
    hit_index: np.ndarray    # int64 [k] position in the slice arrays
    t_axis: int              # time the muon passes its reference point


@dataclass
class Slice:
    pmt: np.ndarray            # uint16 [n]
    t: np.ndarray              # int64 [n]
    q: np.ndarray              # uint16 [n]
    n_pmt: int
    t0: int
    length_ns: int
    tracks: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


def quantise_charge(pe: np.ndarray) -> np.ndarray:
    """0.01 pe units, ``rint(x*100)`` clamped to [0, 65535]."""
    return np.clip(np.rint(pe * 100.0), 0, 65535).astype(np.uint16)


def background_charge(rng: np.random.Generator, k: int) -> np.ndarray:
    """N(1.0, 0.3) pe, with 5 % of hits multiplied by U[2, 5] (in pe, float64)."""
    x = rng.normal(1.0, 0.3, size=k)
    big = rng.random(k) < 0.05
    x[big] *= rng.uniform(2.0, 5.0, size=int(big.sum()))
    return x


def _track_arrivals(geom: Geometry, rng: np.random.Generator, centre_xy, t_axis: int,
                    radius_m: float = 30.0, att_m: float = 30.0, jitter_ns: float = 3.0,
                    min_hits: int = 6, max_tries: int = 1000):
    """One straight muon passing within ``radius_m`` of a tower axis.

    Arrival time at a PMT at longitudinal coordinate ``l`` and distance ``rho``
    from the track is ``t_axis + (l + rho * tan(theta_C)) / c`` (direct
    Cherenkov light, cos(theta_C) = 1/n).  A PMT detects the track with
    probability ``exp(-rho / att_m)``; resampled until >= ``min_hits`` PMTs fire.
    """
    for _ in range(max_tries):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        # reference point: on the axis at a uniform height, offset in the plane normal to u
        z = rng.uniform(0.0, geom.height)
        w = rng.normal(size=3)
        w -= w.dot(u) * u
        w /= np.linalg.norm(w)
        r0 = np.array([centre_xy[0], centre_xy[1], z]) + w * radius_m * np.sqrt(rng.random())
        v = geom.pos - r0
        lon = v @ u
        rho = np.sqrt(np.maximum((v * v).sum(1) - lon * lon, 0.0))
        det = rng.random(len(rho)) < np.exp(-rho / att_m)
        if det.sum() < min_hits:
            continue
        idx = np.nonzero(det)[0]
        # offsets in float64 relative to t_axis (an absolute 1.4e18 ns epoch would lose precision)
        dt_true = (lon[idx] + rho[idx] * TAN_CHERENKOV) / C_M_PER_NS
        t_hit = t_axis + np.rint(dt_true + rng.normal(0.0, jitter_ns, size=len(idx))).astype(np.int64)
        q = quantise_charge(np.maximum(rng.normal(4.0, 1.5, size=len(idx)), 0.1))
        return idx.astype(np.int64), t_hit, q.astype(np.int64)
    raise RuntimeError("could not sample a detected track")


def make_slice(geom: Geometry, length_ns: int, rate_hz, seed, *, t0: int = T0_EPOCH_NS,
               n_tracks: int = 0, bursts=(), order: str = "runs",
               track_towers=None) -> Slice:
    """Draw one slice.

    * background: per PMT, ``Poisson(R * T)`` hits at integer times uniform in
      ``[t0, t0 + T)``; ``rate_hz`` is a scalar or a per-PMT array.
    * bursts: ``(pmt, rate_hz, start_ns, dur_ns)`` adds a Poisson stream on one
      PMT over ``[t0 + start, t0 + start + dur)``.
    * tracks: reference time uniform in ``[t0 + 1 ms, t0 + T - 1 ms]`` (or the
      middle of short slices); each passes a random tower of ``track_towers``
      (default: all towers).
    * order: ``runs`` = concatenated per-PMT time-ordered runs (the DAQ
      stream layout), ``shuffled`` = random permutation, ``sorted`` = by time.
    """
    P = geom.n_pmt
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(P + 2)
    rates = np.broadcast_to(np.asarray(rate_hz, dtype=np.float64), (P,))
    T = int(length_ns)
    per_t, per_q, per_src = [], [], []
    for p in range(P):
        rng = np.random.Generator(np.random.PCG64(kids[p]))
        k = int(rng.poisson(rates[p] * T * 1e-9))
        tp = t0 + rng.integers(0, T, size=k, dtype=np.int64)
        qp = quantise_charge(background_charge(rng, k)).astype(np.int64)
        per_t.append([tp])
        per_q.append([qp])
        per_src.append([np.full(k, -1, np.int64)])
    brng = np.random.Generator(np.random.PCG64(kids[P]))
    for (bp, brate, bstart, bdur) in bursts:
        k = int(brng.poisson(brate * bdur * 1e-9))
        tp = t0 + int(bstart) + brng.integers(0, int(bdur), size=k, dtype=np.int64)
        per_t[bp].append(tp)
        per_q[bp].append(quantise_charge(background_charge(brng, k)).astype(np.int64))
        per_src[bp].append(np.full(k, -1, np.int64))
    trng = np.random.Generator(np.random.PCG64(kids[P + 1]))
    towers = np.arange(len(geom.tower_xy)) if track_towers is None else np.asarray(track_towers)
    track_axis_times = []
    for j in range(n_tracks):
        lo, hi = 1_000_000, T - 1_000_000
        if hi <= lo:
            lo, hi = T // 4, max(T // 4 + 1, 3 * T // 4)
        t_axis = t0 + int(trng.integers(lo, hi))
        tw = int(trng.choice(towers))
        idx, th, qh = _track_arrivals(geom, trng, geom.tower_xy[tw], t_axis)
        track_axis_times.append(t_axis)
        for p, tt, qq in zip(idx, th, qh):
            per_t[p].append(np.array([tt], np.int64))
            per_q[p].append(np.array([qq], np.int64))
            per_src[p].append(np.array([j], np.int64))
    # per-PMT time-ordered streams (stable, so equal times keep draw order)
    pm, tm, qm, sm = [], [], [], []
    for p in range(P):
        tp = np.concatenate(per_t[p])
        qp = np.concatenate(per_q[p])
        sp = np.concatenate(per_src[p])
        o = np.argsort(tp, kind="stable")
        pm.append(np.full(len(tp), p, np.uint16))
        tm.append(tp[o])
        qm.append(qp[o])
        sm.append(sp[o])
    pmt = np.concatenate(pm) if pm else np.zeros(0, np.uint16)
    t = np.concatenate(tm) if tm else np.zeros(0, np.int64)
    q = np.concatenate(qm).astype(np.uint16) if qm else np.zeros(0, np.uint16)
    src = np.concatenate(sm) if sm else np.zeros(0, np.int64)
    if order == "shuffled":
        perm = np.random.Generator(np.random.PCG64(ss.spawn(1)[0])).permutation(len(t))
    elif order == "sorted":
        perm = np.lexsort((np.arange(len(t)), pmt, t))
    elif order == "runs":
        perm = None
    else:
        raise ValueError(order)
    if perm is not None:
        pmt, t, q, src = pmt[perm], t[perm], q[perm], src[perm]
    tracks = []
    # positions of each track's hits, ascending (one pass over the slice)
    tpos = np.nonzero(src >= 0)[0]
    tpos = tpos[np.argsort(src[tpos], kind="stable")]
    bounds = np.searchsorted(src[tpos], np.arange(n_tracks + 1))
    for j in range(n_tracks):
        pos = tpos[bounds[j]:bounds[j + 1]]
        tracks.append(Track(pmt=pmt[pos].astype(np.int64), t=t[pos], q=q[pos].astype(np.int64),
                            hit_index=pos, t_axis=track_axis_times[j]))
    return Slice(pmt=np.ascontiguousarray(pmt), t=np.ascontiguousarray(t),
                 q=np.ascontiguousarray(q), n_pmt=P, t0=t0, length_ns=T, tracks=tracks)


def concat_runs_order(s: Slice) -> bool:
    """True if the slice is a concatenation of per-PMT time-ordered runs."""
    if s.n == 0:
        return True
    same = s.pmt[1:] == s.pmt[:-1]
    return bool(np.all(s.t[1:][same] >= s.t[:-1][same]))
