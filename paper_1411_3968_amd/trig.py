"""Thin ctypes binding of libtrig.so (argument marshalling only).

The functions carry the C ABI's names (``trig_create``, ``trig_geom_load``,
``trig_slice``, ``trig_batch``, ``trig_stream_submit``, ``trig_stream_poll``,
...).  Inputs are numpy arrays (host memory) or torch tensors on the GPU
(device memory, passed by ``data_ptr()``); torch is only used for device memory
and streams.  Every step of the trigger runs in the HIP library: if
``libtrig.so`` is missing or fails to load, the import raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrig.so")

TRIG_OK, TRIG_PENDING = 0, 1
TRIG_EINVAL, TRIG_ERANGE, TRIG_ENOMEM, TRIG_EAGAIN, TRIG_EOVERFLOW, TRIG_EHIP, TRIG_ECANCELED = -1, -2, -3, -4, -5, -6, -7
TRIG_MEM_HOST, TRIG_MEM_DEVICE = 0, 1
STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ERANGE", -3: "ENOMEM", -4: "EAGAIN",
                -5: "EOVERFLOW", -6: "EHIP", -7: "ECANCELED"}

FIRE_DTYPE = np.dtype([("t_ns", "<i8"), ("hit_index", "<u4"), ("fold", "<u4"),
                       ("pmt_id", "<u2"), ("pad", "<u2", (3,))])
EVENT_DTYPE = np.dtype([("t_trig", "<i8"), ("t_begin", "<i8"), ("t_end", "<i8"),
                        ("n_fire", "<u4"), ("max_fold", "<u4")])


class TrigError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GeomDesc(C.Structure):
    _fields_ = [("n_pmt", C.c_uint32), ("floor_id", C.c_void_p), ("thr_ns", C.c_void_p), ("adj_id", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("q_seed", C.c_uint32), ("t_floor_ns", C.c_int32), ("w_ns", C.c_uint32),
                ("min_fold", C.c_uint32), ("half_event_ns", C.c_uint32),
                ("l0_n", C.c_uint32), ("l0_tw_ns", C.c_uint32), ("l0_distinct", C.c_uint32),
                ("t_adj_ns", C.c_int32), ("t_afloor_ns", C.c_int32), ("seed_mode", C.c_uint32)]


class SliceDesc(C.Structure):
    _fields_ = [("geom_id", C.c_uint32), ("mem", C.c_uint32), ("n_hits", C.c_uint64),
                ("pmt_id", C.c_void_p), ("t_ns", C.c_void_p), ("charge", C.c_void_p), ("tag", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("fires", C.c_void_p), ("fire_cap", C.c_uint64), ("n_fires", C.c_uint64),
                ("events", C.c_void_p), ("event_cap", C.c_uint64), ("n_events", C.c_uint64),
                ("seed_flags", C.c_void_p), ("n_hits", C.c_uint64), ("n_seeds", C.c_uint64),
                ("tag", C.c_uint64), ("status", C.c_int32), ("path", C.c_uint32),
                ("tagged", C.c_void_p), ("tagged_cap", C.c_uint64), ("n_tagged", C.c_uint64)]


class Tune(C.Structure):
    _fields_ = [("seg_target", C.c_uint32), ("seg_cap", C.c_uint32), ("grid_per_cu", C.c_uint32),
                ("tile_group", C.c_uint32), ("window_cap", C.c_uint32), ("reserved", C.c_uint32)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("total_ms", C.c_double)]


class StreamStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected_again", C.c_uint64),
                ("in_flight", C.c_uint64), ("device_bytes_in_use", C.c_uint64),
                ("device_bytes_peak", C.c_uint64), ("rounds", C.c_uint64)]


assert C.sizeof(Result) == 112 and C.sizeof(SliceDesc) == 48 and C.sizeof(Params) == 44

EXPORTS = ["trig_create", "trig_destroy", "trig_last_error", "trig_version", "trig_geom_load", "trig_slice",
           "trig_slice_noalloc", "trig_batch", "trig_stream_submit", "trig_stream_poll", "trig_stream_next_done", "trig_stream_pause",
           "trig_stream_stats_get",
           "trig_tune_get",
           "trig_tune_set", "trig_profile_enable", "trig_profile_read"]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libtrig.so not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    P, V = C.c_void_p, C.c_void_p
    lib.trig_create.argtypes = [C.POINTER(P), C.c_int, C.c_uint64]
    lib.trig_destroy.argtypes = [P]
    lib.trig_destroy.restype = None
    lib.trig_last_error.argtypes = [P]
    lib.trig_last_error.restype = C.c_char_p
    lib.trig_version.argtypes = []
    lib.trig_version.restype = C.c_char_p
    lib.trig_geom_load.argtypes = [P, C.POINTER(GeomDesc), C.POINTER(C.c_uint32)]
    lib.trig_slice.argtypes = [P, C.POINTER(SliceDesc), C.POINTER(Params), C.POINTER(Result), V]
    lib.trig_slice_noalloc.argtypes = [P, C.POINTER(SliceDesc), C.POINTER(Params), C.POINTER(Result), V]
    lib.trig_batch.argtypes = [P, C.c_uint32, C.POINTER(SliceDesc), C.POINTER(Params), C.POINTER(Result), V]
    lib.trig_stream_submit.argtypes = [P, C.POINTER(SliceDesc), C.POINTER(Params), C.POINTER(C.c_uint64)]
    lib.trig_stream_poll.argtypes = [P, C.c_uint64, C.POINTER(Result), C.c_int32]
    lib.trig_stream_next_done.argtypes = [P, C.POINTER(C.c_uint64), C.c_int32]
    lib.trig_stream_stats_get.argtypes = [P, C.POINTER(StreamStats)]
    lib.trig_stream_pause.argtypes = [P, C.c_int]
    lib.trig_tune_get.argtypes = [P, C.c_uint32, C.POINTER(Tune)]
    lib.trig_tune_set.argtypes = [P, C.c_uint32, C.POINTER(Tune)]
    lib.trig_profile_enable.argtypes = [P, C.c_int]
    lib.trig_profile_read.argtypes = [P, C.POINTER(KernelTime), C.c_uint32, C.POINTER(C.c_uint32)]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if fn.restype is C.c_int or name in ("trig_create", "trig_geom_load", "trig_slice", "trig_slice_noalloc",
                                               "trig_batch",
                                               "trig_stream_submit", "trig_stream_poll", "trig_stream_next_done",
                                               "trig_stream_stats_get",
                                               "trig_stream_pause",
                                               "trig_tune_get", "trig_tune_set", "trig_profile_enable",
                                               "trig_profile_read"):
            fn.restype = C.c_int
    return lib


_LIB = load_library()


def lib() -> C.CDLL:
    return _LIB


def params_struct(p: dict | None) -> Params:
    p = p or {}
    return Params(int(p.get("q_seed", 300)), int(p.get("t_floor_ns", 20)), int(p.get("w_ns", 3000)),
                  int(p.get("min_fold", 4)), int(p.get("half_event_ns", 3000)),
                  int(p.get("l0_n", 0)), int(p.get("l0_tw_ns", 1000)), int(bool(p.get("l0_distinct", 0))),
                  int(p.get("t_adj_ns", -1)), int(p.get("t_afloor_ns", -1)), int(p.get("seed_mode", 0)))


def _err(ctx) -> str:
    m = _LIB.trig_last_error(ctx)
    return m.decode() if m else ""


# ------------------------------------------------------------ C-ABI mirrors

def trig_version() -> str:
    return _LIB.trig_version().decode()


def trig_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = C.c_void_p()
    rc = _LIB.trig_create(C.byref(h), int(device), int(hbm_budget_bytes))
    if rc != TRIG_OK:
        raise TrigError(rc, "trig_create failed")
    return h


def trig_destroy(ctx) -> None:
    _LIB.trig_destroy(ctx)


def trig_last_error(ctx) -> str:
    return _err(ctx)


def trig_geom_load(ctx, floor_id, thr, adj_id=None) -> int:
    floor_id = np.ascontiguousarray(floor_id, dtype=np.int32)
    thr = np.ascontiguousarray(thr, dtype=np.uint32).reshape(-1)
    P = floor_id.shape[0]
    if thr.shape[0] != P * P:
        raise ValueError("thr must be n_pmt x n_pmt")
    adj = None if adj_id is None else np.ascontiguousarray(adj_id, dtype=np.int32)
    if adj is not None and adj.shape[0] != P:
        raise ValueError("adj_id must have n_pmt entries")
    g = GeomDesc(P, floor_id.ctypes.data, thr.ctypes.data, adj.ctypes.data if adj is not None else None)
    gid = C.c_uint32()
    rc = _LIB.trig_geom_load(ctx, C.byref(g), C.byref(gid))
    if rc != TRIG_OK:
        raise TrigError(rc, _err(ctx))
    return int(gid.value)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def slice_desc(geom_id: int, pmt, t, q, tag: int = 0):
    """Descriptor plus the objects that must stay alive while it is used."""
    if _is_torch(t):
        for a in (pmt, t, q):
            if not a.is_cuda or not a.is_contiguous():
                raise ValueError("device inputs must be contiguous GPU tensors")
        n = int(t.numel())
        d = SliceDesc(geom_id, TRIG_MEM_DEVICE, n, pmt.data_ptr(), t.data_ptr(), q.data_ptr(), tag)
        return d, (pmt, t, q)
    pmt = np.ascontiguousarray(pmt, dtype=np.uint16)
    t = np.ascontiguousarray(t, dtype=np.int64)
    q = np.ascontiguousarray(q, dtype=np.uint16)
    if not (pmt.shape == t.shape == q.shape):
        raise ValueError("pmt, t and q must have one length")
    n = int(t.shape[0])
    d = SliceDesc(geom_id, TRIG_MEM_HOST, n, pmt.ctypes.data if n else None, t.ctypes.data if n else None,
                  q.ctypes.data if n else None, tag)
    return d, (pmt, t, q)


def _host_array(count: int, dtype, pinned: bool):
    """A zeroed host array; ``pinned`` places it in pinned (page-locked) memory,
    which the library's kernels write large result lists into directly."""
    dtype = np.dtype(dtype)
    if not pinned:
        return np.zeros(count, dtype), None
    import torch
    buf = torch.zeros(count * dtype.itemsize, dtype=torch.uint8, pin_memory=True)
    return buf.numpy().view(dtype), buf


class ResultBuffers:
    """Host buffers of one result record (``pinned``: fire, event and tagged
    lists in pinned memory)."""

    def __init__(self, fire_cap: int, event_cap: int, n_hits: int, seed_flags: bool, tagged_cap: int | None = None,
                 pinned: bool = False):
        self.fires, self._pf = _host_array(max(fire_cap, 1), FIRE_DTYPE, pinned)
        self.events, self._pe = _host_array(max(event_cap, 1), EVENT_DTYPE, pinned)
        self.flags = np.zeros(max(n_hits, 1), np.uint8) if seed_flags else None
        self.tagged, self._pt = _host_array(max(tagged_cap, 1), np.uint32, pinned) if tagged_cap is not None \
            else (None, None)
        self.rec = Result()
        self.reset()

    def reset(self):
        r = self.rec
        r.fires = self.fires.ctypes.data
        r.fire_cap = len(self.fires)
        r.events = self.events.ctypes.data
        r.event_cap = len(self.events)
        r.seed_flags = self.flags.ctypes.data if self.flags is not None else None
        r.tagged = self.tagged.ctypes.data if self.tagged is not None else None
        r.tagged_cap = len(self.tagged) if self.tagged is not None else 0

    def as_dict(self, copy: bool = True) -> dict:
        """Counts and lists of the record; ``copy=False`` returns views into the
        buffers (valid until they are reused)."""
        r = self.rec
        ok = r.status == TRIG_OK
        cp = (lambda a: a.copy()) if copy else (lambda a: a)
        out = dict(status=int(r.status), n_hits=int(r.n_hits), n_seeds=int(r.n_seeds), tag=int(r.tag),
                   path=int(r.path), n_fires=int(r.n_fires), n_events=int(r.n_events),
                   fires=cp(self.fires[:r.n_fires] if ok else self.fires[:0]),
                   events=cp(self.events[:r.n_events] if ok else self.events[:0]))
        if self.flags is not None:
            out["seed_flags"] = cp(self.flags[:r.n_hits] if ok else self.flags[:0])
        if self.tagged is not None:
            out["n_tagged"] = int(r.n_tagged)
            out["tagged"] = cp(self.tagged[:r.n_tagged] if ok else self.tagged[:0])
        return out


def _default_caps(n: int):
    return max(4096, n // 8), max(4096, n // 8)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def trig_slice(ctx, geom_id: int, pmt, t, q, params: dict | None = None, *, seed_flags: bool = False,
               fire_cap: int | None = None, event_cap: int | None = None, stream=None, tag: int = 0,
               raise_on_error: bool = True, tagged: bool = False, tagged_cap: int | None = None) -> dict:
    """Trigger one slice; retries once with exact capacities on TRIG_EOVERFLOW.
    ``tagged=True`` also returns the input indices of the hits inside the event
    windows (``tagged``, ordered by time, PMT, input index)."""
    return _one_slice(_LIB.trig_slice, ctx, geom_id, pmt, t, q, params, seed_flags, fire_cap, event_cap, stream,
                      tag, raise_on_error, tagged, tagged_cap)


def trig_slice_noalloc(ctx, geom_id: int, pmt, t, q, params: dict | None = None, *, seed_flags: bool = False,
                       fire_cap: int | None = None, event_cap: int | None = None, stream=None, tag: int = 0,
                       raise_on_error: bool = True, tagged: bool = False, tagged_cap: int | None = None) -> dict:
    """``trig_slice`` through the allocation-free entry point: device inputs only,
    the workspace in the library's fixed per-GPU scratch (TRIG_ENOMEM beyond it)."""
    return _one_slice(_LIB.trig_slice_noalloc, ctx, geom_id, pmt, t, q, params, seed_flags, fire_cap, event_cap,
                      stream, tag, raise_on_error, tagged, tagged_cap)


def _one_slice(fn, ctx, geom_id, pmt, t, q, params, seed_flags, fire_cap, event_cap, stream, tag, raise_on_error,
               tagged, tagged_cap) -> dict:
    d, keep = slice_desc(geom_id, pmt, t, q, tag)
    n = int(d.n_hits)
    fc, ec = _default_caps(n)
    fc = fire_cap if fire_cap is not None else fc
    ec = event_cap if event_cap is not None else ec
    prm = params_struct(params)
    if stream is None and _is_torch(t):
        import torch
        stream = torch.cuda.current_stream()
    sp = _stream_ptr(stream)
    tc = (tagged_cap if tagged_cap is not None else max(4096, n // 8)) if tagged else None
    for attempt in range(2):
        rb = ResultBuffers(fc, ec, n, seed_flags, tc)
        rc = fn(ctx, C.byref(d), C.byref(prm), C.byref(rb.rec), sp)
        if rc == TRIG_EOVERFLOW and attempt == 0 and fire_cap is None and event_cap is None \
                and (not tagged or tagged_cap is None):
            fc, ec = int(rb.rec.n_fires), int(rb.rec.n_events)
            tc = int(rb.rec.n_tagged) if tagged else None
            continue
        break
    del keep
    if rc != TRIG_OK and raise_on_error and rc not in (TRIG_ERANGE, TRIG_EOVERFLOW):
        raise TrigError(rc, _err(ctx))
    return rb.as_dict()


def trig_batch(ctx, slices, params: dict | None = None, *, seed_flags: bool = False, stream=None,
               caps=None, tagged: bool = False) -> list:
    """``slices``: list of ``(geom_id, pmt, t, q)``.  Returns one dict per slice
    (with ``tagged``, the hits inside the event windows, when asked for)."""
    n = len(slices)
    descs = (SliceDesc * max(n, 1))()
    keep = []
    ns = []
    for i, (gid, pmt, t, q) in enumerate(slices):
        d, k = slice_desc(gid, pmt, t, q, tag=i)
        descs[i] = d
        keep.append(k)
        ns.append(int(d.n_hits))
    if stream is None and n and _is_torch(slices[0][2]):
        import torch
        stream = torch.cuda.current_stream()
    sp = _stream_ptr(stream)
    prm = params_struct(params)
    caps = caps or [_default_caps(x) for x in ns]
    tcaps = [max(4096, x // 8) for x in ns] if tagged else None
    for attempt in range(2):
        bufs = [ResultBuffers(caps[i][0], caps[i][1], ns[i], seed_flags, tcaps[i] if tagged else None)
                for i in range(n)]
        recs = (Result * max(n, 1))()
        for i in range(n):
            recs[i] = bufs[i].rec
        rc = _LIB.trig_batch(ctx, n, descs, C.byref(prm), recs, sp)
        over = [i for i in range(n) if recs[i].status == TRIG_EOVERFLOW]
        if over and attempt == 0:
            caps = [(max(int(recs[i].n_fires), caps[i][0]), max(int(recs[i].n_events), caps[i][1]))
                    for i in range(n)]
            if tagged:
                tcaps = [max(int(recs[i].n_tagged), tcaps[i]) for i in range(n)]
            continue
        break
    out = []
    for i in range(n):
        ctypes_rec = recs[i]
        bufs[i].rec = ctypes_rec
        out.append(bufs[i].as_dict())
    del keep
    if rc not in (TRIG_OK, TRIG_ERANGE, TRIG_EINVAL, TRIG_EOVERFLOW):
        raise TrigError(rc, _err(ctx))
    return out


def trig_stream_submit(ctx, geom_id: int, pmt, t, q, params: dict | None = None, tag: int = 0):
    """Returns ``(status, ticket)``; status is TRIG_OK, TRIG_EAGAIN or an error."""
    d, keep = slice_desc(geom_id, pmt, t, q, tag)
    prm = params_struct(params)
    tk = C.c_uint64()
    rc = _LIB.trig_stream_submit(ctx, C.byref(d), C.byref(prm), C.byref(tk))
    del keep
    return rc, int(tk.value)


class StreamSubmitter:
    """``trig_stream_submit`` over a fixed set of slices with marshalling done
    once: the descriptors (``slices``: list of ``(geom_id, pmt, t, q)``) and the
    parameters are built at construction; a call sets the tag of slice ``i`` and
    invokes the C ABI (which copies the descriptor into its ticket).  Returns
    ``(status, ticket)`` like ``trig_stream_submit``."""

    def __init__(self, ctx, slices, params: dict | None = None):
        self.ctx = ctx
        self._d, self._keep = [], []
        for geom_id, pmt, t, q in slices:
            d, keep = slice_desc(geom_id, pmt, t, q)
            self._d.append(d)
            self._keep.append(keep)
        self.prm = params_struct(params)
        self._pp = C.byref(self.prm)
        self._tk = C.c_uint64()
        self._ptk = C.byref(self._tk)

    def __call__(self, i: int, tag: int = 0):
        d = self._d[i]
        d.tag = tag
        rc = _LIB.trig_stream_submit(self.ctx, C.byref(d), self._pp, self._ptk)
        return rc, int(self._tk.value)


def trig_stream_poll(ctx, ticket: int, timeout_us: int = -1, fire_cap: int = 1 << 16, event_cap: int = 1 << 16,
                     n_hits: int = 0, seed_flags: bool = False, buffers: ResultBuffers | None = None,
                     copy: bool = True):
    """Returns ``(status, result dict or None)``.  ``buffers``: reuse these host
    buffers (their capacities apply) instead of allocating new ones; with
    ``copy=False`` the lists are views into them."""
    if buffers is not None:
        rb = buffers
        rb.reset()
    else:
        rb = ResultBuffers(fire_cap, event_cap, n_hits, seed_flags)
    rc = _LIB.trig_stream_poll(ctx, int(ticket), C.byref(rb.rec), int(timeout_us))
    if rc == TRIG_PENDING:
        return rc, None
    return rc, rb.as_dict(copy)


def trig_stream_next_done(ctx, timeout_us: int = -1):
    """Returns ``(status, ticket)``: TRIG_OK with the next finished ticket, or
    TRIG_PENDING (ticket 0) when none finished within ``timeout_us``."""
    tk = C.c_uint64()
    rc = _LIB.trig_stream_next_done(ctx, C.byref(tk), int(timeout_us))
    if rc not in (TRIG_OK, TRIG_PENDING):
        raise TrigError(rc, _err(ctx))
    return rc, int(tk.value) if rc == TRIG_OK else 0


def trig_stream_pause(ctx, paused: bool = True) -> None:
    rc = _LIB.trig_stream_pause(ctx, 1 if paused else 0)
    if rc != TRIG_OK:
        raise TrigError(rc, _err(ctx))


def trig_stream_stats_get(ctx) -> dict:
    s = StreamStats()
    rc = _LIB.trig_stream_stats_get(ctx, C.byref(s))
    if rc != TRIG_OK:
        raise TrigError(rc, _err(ctx))
    return {k: int(getattr(s, k)) for k, _ in StreamStats._fields_}


def trig_tune_get(ctx, n_pmt: int) -> dict:
    t = Tune()
    rc = _LIB.trig_tune_get(ctx, int(n_pmt), C.byref(t))
    if rc != TRIG_OK:
        raise TrigError(rc, _err(ctx))
    return dict(seg_target=t.seg_target, seg_cap=t.seg_cap, grid_per_cu=t.grid_per_cu, tile_group=t.tile_group,
                window_cap=t.window_cap)


def trig_tune_set(ctx, n_pmt_max: int, seg_target: int, seg_cap: int, grid_per_cu: int,
                  tile_group: int | None = None, window_cap: int | None = None) -> None:
    """Set the knobs of one PMT-count class; a knob left at None keeps the value
    the class has now."""
    if tile_group is None or window_cap is None:
        cur = trig_tune_get(ctx, n_pmt_max)
        tile_group = cur["tile_group"] if tile_group is None else tile_group
        window_cap = cur["window_cap"] if window_cap is None else window_cap
    t = Tune(int(seg_target), int(seg_cap), int(grid_per_cu), int(tile_group), int(window_cap), 0)
    rc = _LIB.trig_tune_set(ctx, int(n_pmt_max), C.byref(t))
    if rc != TRIG_OK:
        raise TrigError(rc, _err(ctx))


def trig_profile_enable(ctx, enable: bool = True) -> None:
    _LIB.trig_profile_enable(ctx, 1 if enable else 0)


def trig_profile_read(ctx) -> list:
    n = C.c_uint32()
    _LIB.trig_profile_read(ctx, None, 0, C.byref(n))
    arr = (KernelTime * max(n.value, 1))()
    _LIB.trig_profile_read(ctx, arr, n.value, C.byref(n))
    return [dict(name=arr[i].name.decode(), launches=int(arr[i].launches), total_ms=float(arr[i].total_ms))
            for i in range(n.value)]


class SliceRunner:
    """Repeated ``trig_slice`` on one slice with marshalling done once.

    Descriptor, parameters and result buffers are built at construction; each
    call only invokes the C ABI.  Returned arrays are views into buffers that
    the next call overwrites.
    """

    def __init__(self, ctx, geom_id, pmt, t, q, params=None, *, stream=None, fire_cap=None, event_cap=None,
                 seed_flags=False, tagged=False, tagged_cap=None, pinned=False):
        self.ctx = ctx
        self.desc, self._keep = slice_desc(geom_id, pmt, t, q)
        n = int(self.desc.n_hits)
        fc, ec = _default_caps(n)
        tc = (tagged_cap or max(4096, n // 8)) if tagged else None
        self.buf = ResultBuffers(fire_cap or fc, event_cap or ec, n, seed_flags, tc, pinned)
        self.prm = params_struct(params)
        if stream is None and _is_torch(t):
            import torch
            stream = torch.cuda.current_stream()
        self.sp = _stream_ptr(stream)
        self._pd, self._pp, self._pr = C.byref(self.desc), C.byref(self.prm), C.byref(self.buf.rec)

    def launch(self) -> int:
        """One ``trig_slice`` call: the results are in the buffers on return
        (read them with :meth:`results`)."""
        rc = _LIB.trig_slice(self.ctx, self._pd, self._pp, self._pr, self.sp)
        if rc != TRIG_OK:
            raise TrigError(rc, _err(self.ctx))
        return rc

    def __call__(self) -> dict:
        self.launch()
        return self.results()

    def results(self) -> dict:
        """The last call's results (views into the buffers)."""
        r = self.buf.rec
        rc = TRIG_OK
        out = dict(status=rc, n_seeds=int(r.n_seeds), n_fires=int(r.n_fires), n_events=int(r.n_events),
                   path=int(r.path), fires=self.buf.fires[:r.n_fires], events=self.buf.events[:r.n_events])
        if self.buf.flags is not None:
            out["seed_flags"] = self.buf.flags[:r.n_hits]
        if self.buf.tagged is not None:
            out["n_tagged"] = int(r.n_tagged)
            out["tagged"] = self.buf.tagged[:r.n_tagged]
        return out


class BatchRunner:
    """Repeated ``trig_batch`` over one list of slices with marshalling done once.

    ``slices``: list of ``(geom_id, pmt, t, q)``.  ``caps``: per slice
    ``(fire_cap, event_cap)`` (default: an eighth of the hits, at least 4096).
    Each call returns one dict per slice whose arrays are views into buffers
    that the next call overwrites; a slice whose lists exceed its capacity
    reports TRIG_EOVERFLOW in its ``status``.
    """

    def __init__(self, ctx, slices, params=None, *, stream=None, caps=None):
        self.ctx = ctx
        n = len(slices)
        self.n = n
        self.descs = (SliceDesc * max(n, 1))()
        self._keep = []
        ns = []
        for i, (gid, pmt, t, q) in enumerate(slices):
            d, k = slice_desc(gid, pmt, t, q, tag=i)
            self.descs[i] = d
            self._keep.append(k)
            ns.append(int(d.n_hits))
        caps = caps or [_default_caps(x) for x in ns]
        self.bufs = [ResultBuffers(caps[i][0], caps[i][1], ns[i], False) for i in range(n)]
        self.recs = (Result * max(n, 1))()
        self.prm = params_struct(params)
        if stream is None and n and _is_torch(slices[0][2]):
            import torch
            stream = torch.cuda.current_stream()
        self.sp = _stream_ptr(stream)

    def launch(self) -> int:
        """One ``trig_batch`` call: the results are in the buffers on return
        (read them with :meth:`results`); returns its status."""
        for i in range(self.n):
            self.recs[i] = self.bufs[i].rec
        rc = _LIB.trig_batch(self.ctx, self.n, self.descs, C.byref(self.prm), self.recs, self.sp)
        if rc not in (TRIG_OK, TRIG_ERANGE, TRIG_EINVAL, TRIG_EOVERFLOW):
            raise TrigError(rc, _err(self.ctx))
        return rc

    def __call__(self) -> list:
        self.launch()
        return self.results()

    def results(self) -> list:
        """The last call's results, one dict per slice (views into the buffers)."""
        out = []
        for i in range(self.n):
            r, b = self.recs[i], self.bufs[i]
            out.append(dict(status=int(r.status), n_hits=int(r.n_hits), n_seeds=int(r.n_seeds), path=int(r.path),
                            n_fires=int(r.n_fires), n_events=int(r.n_events),
                            fires=b.fires[:r.n_fires] if r.status == TRIG_OK else b.fires[:0],
                            events=b.events[:r.n_events] if r.status == TRIG_OK else b.events[:0]))
        return out


class Trigger:
    """Convenience owner of one context (``with Trigger() as tr: ...``)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.ctx = trig_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx is not None:
            trig_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load_geometry(self, floor_id, thr, adj_id=None) -> int:
        return trig_geom_load(self.ctx, floor_id, thr, adj_id)

    def slice(self, geom_id, pmt, t, q, params=None, **kw) -> dict:
        return trig_slice(self.ctx, geom_id, pmt, t, q, params, **kw)

    def batch(self, slices, params=None, **kw) -> list:
        return trig_batch(self.ctx, slices, params, **kw)
