"""Seeded synthetic inputs (geometry, threshold tables, hit slices).

Shared by the tests, the benchmark and the oracle's checks.  Holds no part of
the trigger's arithmetic: it only draws inputs.
"""
from .geometry import Geometry, block, km3net_it_tower, nemo_tower, thr_table, tower  # noqa: F401
from .slices import Slice, Track, make_slice, T0_EPOCH_NS  # noqa: F401
