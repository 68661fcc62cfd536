"""ctypes front end of the C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product library never imports it.

``build()`` compiles ``oracle.c`` with gcc (OpenMP) into ``liboracle.so``
next to this file.  ``run()`` evaluates the whole rule on one slice and
returns numpy arrays; ``point()`` evaluates the seed flag and fold of a few
sampled hits at any slice size; ``tag()`` lists the hits within the event
windows of a fire list.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FIRE_DTYPE = np.dtype([("t_ns", "<i8"), ("hit_index", "<u4"), ("fold", "<u4"),
                       ("pmt_id", "<u2"), ("pad", "<u2", (3,))])
EVENT_DTYPE = np.dtype([("t_trig", "<i8"), ("t_begin", "<i8"), ("t_end", "<i8"),
                        ("n_fire", "<u4"), ("max_fold", "<u4")])
assert FIRE_DTYPE.itemsize == 24 and EVENT_DTYPE.itemsize == 32


class Params(C.Structure):
    _fields_ = [("q_seed", C.c_uint32), ("t_floor_ns", C.c_int32), ("w_ns", C.c_uint32),
                ("min_fold", C.c_uint32), ("half_event_ns", C.c_uint32),
                ("l0_n", C.c_uint32), ("l0_tw_ns", C.c_uint32), ("l0_distinct", C.c_uint32),
                ("t_adj_ns", C.c_int32), ("t_afloor_ns", C.c_int32), ("seed_mode", C.c_uint32)]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                        "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.orc_run.argtypes = [C.c_int, C.c_uint64, P, P, P, C.c_uint32, P, P, P, C.POINTER(Params),
                                P, P, P, C.POINTER(C.c_uint64), P, C.POINTER(C.c_uint64), C.c_int]
        lib.orc_run.restype = C.c_int
        lib.orc_point.argtypes = [C.c_uint64, P, P, P, C.c_uint32, P, P, C.POINTER(Params),
                                  P, C.c_uint64, P, P, C.c_int]
        lib.orc_point.restype = C.c_int
        lib.orc_tag.argtypes = [C.c_uint64, P, P, P, C.c_uint64, C.c_uint32, P]
        lib.orc_tag.restype = C.c_uint64
        _lib = lib
    return _lib


def _params(p: dict) -> Params:
    return Params(int(p.get("q_seed", 300)), int(p.get("t_floor_ns", 20)), int(p.get("w_ns", 3000)),
                  int(p.get("min_fold", 4)), int(p.get("half_event_ns", 3000)),
                  int(p.get("l0_n", 0)), int(p.get("l0_tw_ns", 1000)), int(bool(p.get("l0_distinct", 0))),
                  int(p.get("t_adj_ns", -1)), int(p.get("t_afloor_ns", -1)), int(p.get("seed_mode", 0)))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _inputs(pmt, t, q, floor_id, thr):
    pmt = np.ascontiguousarray(pmt, dtype=np.uint16)
    t = np.ascontiguousarray(t, dtype=np.int64)
    q = np.ascontiguousarray(q, dtype=np.uint16)
    floor_id = np.ascontiguousarray(floor_id, dtype=np.int32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32).reshape(-1)
    return pmt, t, q, floor_id, thr


def run(pmt, t, q, floor_id, thr, params: dict | None = None, form: str = "blocked",
        threads: int = 0, adj_id=None) -> dict:
    """Whole rule on one slice.  ``form`` is ``strict`` (all pairs) or ``blocked``;
    ``adj_id`` (per PMT) groups the adjacent PMTs of a floor for the SC rule."""
    pmt, t, q, floor_id, thr = _inputs(pmt, t, q, floor_id, thr)
    adj = None if adj_id is None else np.ascontiguousarray(adj_id, dtype=np.int32)
    n = t.shape[0]
    seed = np.zeros(max(n, 1), np.uint8)
    fold = np.zeros(max(n, 1), np.uint32)
    fires = np.zeros(max(n, 1), FIRE_DTYPE)
    events = np.zeros(max(n, 1), EVENT_DTYPE)
    nf, ne = C.c_uint64(0), C.c_uint64(0)
    prm = _params(params or {})
    rc = _load().orc_run(0 if form == "strict" else 1, n, _ptr(pmt), _ptr(t), _ptr(q), len(floor_id),
                         _ptr(floor_id), _ptr(adj), _ptr(thr), C.byref(prm), seed.ctypes.data_as(C.c_void_p),
                         fold.ctypes.data_as(C.c_void_p), fires.ctypes.data_as(C.c_void_p), C.byref(nf),
                         events.ctypes.data_as(C.c_void_p), C.byref(ne), int(threads))
    return dict(status=int(rc), seed=seed[:n] if rc == 0 else seed[:0], fold=fold[:n] if rc == 0 else fold[:0],
                fires=fires[:nf.value].copy(), events=events[:ne.value].copy())


def tag(pmt, t, fires, half_event_ns: int = 3000):
    """Input indices of the hits within +-half_event_ns of some fire, ordered by
    (t, pmt, input index).  ``fires`` as returned by :func:`run` (time order)."""
    pmt = np.ascontiguousarray(pmt, dtype=np.uint16)
    t = np.ascontiguousarray(t, dtype=np.int64)
    fires = np.ascontiguousarray(fires, dtype=FIRE_DTYPE)
    n = t.shape[0]
    out = np.zeros(max(n, 1), np.uint32)
    lib = _load()
    c = lib.orc_tag(n, _ptr(pmt), _ptr(t), _ptr(fires), len(fires), int(half_event_ns),
                    out.ctypes.data_as(C.c_void_p))
    if c == (1 << 64) - 1:
        raise MemoryError("orc_tag")
    return out[:c].copy()


def point(pmt, t, q, floor_id, thr, ks, params: dict | None = None, threads: int = 0):
    """Seed flag and fold (0 for non-seeds) of the hits at input positions ``ks``."""
    pmt, t, q, floor_id, thr = _inputs(pmt, t, q, floor_id, thr)
    ks = np.ascontiguousarray(ks, dtype=np.uint64)
    seed = np.zeros(max(len(ks), 1), np.uint8)
    fold = np.zeros(max(len(ks), 1), np.uint32)
    prm = _params(params or {})
    rc = _load().orc_point(t.shape[0], _ptr(pmt), _ptr(t), _ptr(q), len(floor_id), _ptr(floor_id), _ptr(thr),
                           C.byref(prm), _ptr(ks), len(ks), seed.ctypes.data_as(C.c_void_p),
                           fold.ctypes.data_as(C.c_void_p), int(threads))
    if rc != 0:
        raise RuntimeError(f"orc_point failed: {rc}")
    return seed[:len(ks)], fold[:len(ks)]
