"""Tower geometry and the pair-threshold table (seeded input generation only).

This module builds *inputs*: PMT positions, the floor index of every PMT and
the integer causality table ``thr``.  It holds none of the trigger's
arithmetic; both the oracle and the HIP library receive ``floor_id`` and
``thr`` as plain arrays.

Geometry facts from the paper (Sec. 2, DAQ system of NEMO Phase II): a NEMO
Phase II tower has 8 floors of 4 detection units, floors 40 m apart, 6 m
floors.  Sec. 5 (Results) gives the KM3Net-It tower: 14 floors, floors 20 m
apart, 84 PMTs.  The paper prints no PMT coordinates (its tower figure is
not available), so the layout within a floor is a proposal: the PMTs sit at
the two ends of the floor bar (+-L/2), split evenly between the ends, with
1 m vertical offsets within one end, and alternate floors are rotated by 90
degrees.

``thr[i][j] = ceil(n * d_ij / c) + tol`` (ns), computed in float64, with
``n = 1.35`` and ``c = 0.299792458 m/ns``: the largest arrival-time
difference a single Cherenkov front can produce between PMTs ``i`` and ``j``
(Sec. 3, Muon trigger strategy: arrival times are correlated in time and
space), plus a tolerance for time jitter.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C_M_PER_NS = 0.299792458
N_WATER = 1.35


@dataclass
class Geometry:
    """PMT positions (metres), global floor index per PMT, tower index per PMT."""

    pos: np.ndarray        # float64 [P, 3]
    floor_id: np.ndarray   # int32 [P]
    tower_id: np.ndarray   # int32 [P]
    tower_xy: np.ndarray   # float64 [n_towers, 2]
    height: float          # metres spanned by one tower's floors

    @property
    def n_pmt(self) -> int:
        return int(self.pos.shape[0])


def _tower_positions(n_floors: int, per_floor: int, dz: float, arm: float):
    """Positions of one tower's PMTs around the origin, and their floor index."""
    if per_floor % 2:
        raise ValueError("per_floor must be even (PMTs split between both bar ends)")
    half = per_floor // 2
    # vertical offsets within one end of the bar: 1 m apart, centred on the floor
    offs = (np.arange(half, dtype=np.float64) - (half - 1) / 2.0) * 1.0
    pos = []
    floor = []
    for f in range(n_floors):
        z = f * dz
        # alternate floors rotated by 90 degrees
        ax = np.array([1.0, 0.0]) if f % 2 == 0 else np.array([0.0, 1.0])
        for end in (-1.0, 1.0):
            xy = end * (arm / 2.0) * ax
            for o in offs:
                pos.append((xy[0], xy[1], z + o))
                floor.append(f)
    return np.asarray(pos, dtype=np.float64), np.asarray(floor, dtype=np.int32)


def tower(n_floors: int = 8, per_floor: int = 4, dz: float = 40.0, arm: float = 6.0) -> Geometry:
    """A single tower centred on x = y = 0 (NEMO-like defaults)."""
    pos, floor = _tower_positions(n_floors, per_floor, dz, arm)
    return Geometry(pos=pos, floor_id=floor, tower_id=np.zeros(len(floor), np.int32),
                    tower_xy=np.zeros((1, 2)), height=(n_floors - 1) * dz)


def nemo_tower() -> Geometry:
    """NEMO Phase II-like tower: 8 floors x 4 PMTs, 40 m apart, 6 m arms."""
    return tower(8, 4, 40.0, 6.0)


def km3net_it_tower() -> Geometry:
    """KM3Net-It-like tower: 14 floors x 6 PMTs, 20 m apart, 8 m arms."""
    return tower(14, 6, 20.0, 8.0)


def block(nx: int = 4, ny: int = 8, pitch: float = 90.0, n_floors: int = 14,
          per_floor: int = 6, dz: float = 20.0, arm: float = 8.0) -> Geometry:
    """``nx * ny`` KM3Net-It-like towers on a square grid; floors numbered globally,
    with a gap of two ids between towers so that only floors of one tower are
    consecutive (the AFC rule pairs PMTs on consecutive floors of a tower)."""
    one_pos, one_floor = _tower_positions(n_floors, per_floor, dz, arm)
    pos, floor, tid, txy = [], [], [], []
    k = 0
    for ix in range(nx):
        for iy in range(ny):
            x0, y0 = ix * pitch, iy * pitch
            p = one_pos.copy()
            p[:, 0] += x0
            p[:, 1] += y0
            pos.append(p)
            floor.append(one_floor + k * (n_floors + 2))   # a gap: no two towers have consecutive floors
            tid.append(np.full(len(one_floor), k, np.int32))
            txy.append((x0, y0))
            k += 1
    return Geometry(pos=np.concatenate(pos), floor_id=np.concatenate(floor).astype(np.int32),
                    tower_id=np.concatenate(tid), tower_xy=np.asarray(txy, np.float64),
                    height=(n_floors - 1) * dz)


def bar_end_groups(geom: Geometry) -> np.ndarray:
    """Group index per PMT: the PMTs at one end of one floor's bar (same floor,
    same horizontal position) share a group; numbered in order of appearance."""
    key = {}
    out = np.empty(geom.n_pmt, np.int32)
    for i in range(geom.n_pmt):
        k = (int(geom.floor_id[i]), round(float(geom.pos[i, 0]), 3), round(float(geom.pos[i, 1]), 3))
        out[i] = key.setdefault(k, len(key))
    return out


def thr_table(geom: Geometry, n: float = N_WATER, c: float = C_M_PER_NS, tol_ns: int = 20) -> np.ndarray:
    """Dense row-major ``uint32 [P, P]`` table ``ceil(n*d/c) + tol_ns`` (float64)."""
    d = np.sqrt(((geom.pos[:, None, :] - geom.pos[None, :, :]) ** 2).sum(-1))
    t = np.ceil(n * d / c) + tol_ns
    return t.astype(np.uint32)


def max_causal_ns(d_m: float, n: float = N_WATER, c: float = C_M_PER_NS) -> float:
    return n * d_m / c


__all__ = ["Geometry", "tower", "nemo_tower", "km3net_it_tower", "block", "thr_table",
           "C_M_PER_NS", "N_WATER", "max_causal_ns"]
