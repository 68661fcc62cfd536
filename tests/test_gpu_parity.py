"""GPU parity: the HIP library against the CPU oracle, byte for byte.

Every output of the trigger is an integer, so the bar is exact equality of the
fire list (t, input index, fold, PMT), the event list, the seed count and the
per-hit seed flags.
"""
import numpy as np
import pytest

from conftest import load_hand_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1411_3968_amd import trig
    return trig


@pytest.fixture(scope="module")
def tr(T):
    t = T.Trigger(0)
    yield t
    t.close()


@pytest.fixture(scope="module")
def orc():
    from oracle import cpu
    return cpu


_GEOM = {}


def gid_for(tr, floor_id, thr):
    key = (floor_id.tobytes(), thr.tobytes())
    if key not in _GEOM:
        _GEOM[key] = tr.load_geometry(floor_id, thr)
    return _GEOM[key]


def check(got, ref, flags=True):
    assert got["status"] == 0, got["status"]
    assert got["n_seeds"] == int(ref["seed"].sum())
    assert got["n_fires"] == len(ref["fires"])
    assert np.array_equal(got["fires"], ref["fires"])
    assert np.array_equal(got["events"], ref["events"])
    if flags and "seed_flags" in got:
        assert np.array_equal(got["seed_flags"], ref["seed"])


def to_dev(s):
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(s.pmt).view(np.int16)).to(dev),
            torch.from_numpy(np.ascontiguousarray(s.t)).to(dev),
            torch.from_numpy(np.ascontiguousarray(s.q).view(np.int16)).to(dev))


HAND = load_hand_cases()


@pytest.mark.parametrize("case", HAND, ids=[c["name"] for c in HAND])
def test_hand_cases(tr, case):
    gid = gid_for(tr, case["floor_id"], case["thr"])
    got = tr.slice(gid, case["pmt"], case["t"], case["q"], case["params"], seed_flags=True)
    assert got["status"] == case["status"], case["cite"]
    if case["status"] != 0:
        return
    assert got["seed_flags"].tolist() == case["seed"]
    assert [[int(f["t_ns"]), int(f["hit_index"]), int(f["fold"]), int(f["pmt_id"])] for f in got["fires"]] == case["fires"]
    assert [[int(e["t_trig"]), int(e["t_begin"]), int(e["t_end"]), int(e["n_fire"]), int(e["max_fold"])]
            for e in got["events"]] == case["events"]


def _random_case(rng, n, n_pmt, n_floor, span, dense_frac=0.0, tie_frac=0.0):
    floor_id = rng.integers(0, n_floor, size=n_pmt).astype(np.int32)
    thr = rng.integers(0, 4000, size=(n_pmt, n_pmt)).astype(np.uint32)
    pmt = rng.integers(0, n_pmt, size=n).astype(np.uint16)
    t = rng.integers(0, span, size=n).astype(np.int64) + int(rng.integers(-10**17, 10**17))
    k = int(dense_frac * n)
    if k:
        t[:k] = t[0] + rng.integers(0, 200, size=k)
    k = int(tie_frac * n)
    if k:
        t[-k:] = t[-1] + rng.integers(0, 3, size=k)
    q = rng.integers(0, 600, size=n).astype(np.uint16)
    params = dict(q_seed=int(rng.integers(200, 700)), t_floor_ns=int(rng.integers(-1, 60)),
                  w_ns=int(rng.integers(0, 5000)), min_fold=int(rng.integers(0, 7)),
                  half_event_ns=int(rng.integers(0, 5000)))
    return pmt, t, q, floor_id, thr, params


@pytest.mark.parametrize("seed", range(16))
def test_random_slices(tr, orc, seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(1, 30000)) if seed % 4 else int(rng.integers(1, 300))
    pmt, t, q, floor_id, thr, params = _random_case(rng, n, int(rng.integers(1, 40)), int(rng.integers(1, 6)),
                                                     int(rng.integers(10, 5_000_000)),
                                                     dense_frac=0.05 * (seed % 3 == 1), tie_frac=0.1 * (seed % 3 == 2))
    if seed % 2:                       # runs per PMT, like DAQ streams
        o = np.lexsort((t, pmt))
        pmt, t, q = pmt[o], t[o], q[o]
    gid = gid_for(tr, floor_id, thr)
    got = tr.slice(gid, pmt, t, q, params, seed_flags=True)
    ref = orc.run(pmt, t, q, floor_id, thr, params, "strict" if n < 5000 else "blocked")
    check(got, ref)


@pytest.mark.parametrize("order", ["runs", "sorted", "shuffled"])
@pytest.mark.parametrize("key", ["nemo", "km3"])
def test_tower_slices(tr, orc, key, order):
    from gen import configs as C
    w = (C.nemo if key == "nemo" else C.km3)(seed=21, length_ns=30_000_000, n_tracks=5, order=order)
    g, thr = w.geoms[key]
    s = w.slices[0][1]
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, s.pmt, s.t, s.q, w.params, seed_flags=True)
    ref = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    assert got["path"] == (1 if order == "shuffled" else 0)


@pytest.mark.parametrize("key", ["nemo", "km3"])
def test_full_size_tower_device_inputs(tr, orc, key):
    from gen import configs as C
    w = C.nemo() if key == "nemo" else C.km3()
    g, thr = w.geoms[key]
    s = w.slices[0][1]
    gid = gid_for(tr, g.floor_id, thr)
    dp, dt, dq = to_dev(s)
    got = tr.slice(gid, dp, dt, dq, w.params, seed_flags=True)
    ref = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    assert got["path"] == 0 and got["n_fires"] > 0


# (seg_cap, seg_target, grid_per_cu): both wave-per-segment variants and the
# workgroup-per-segment kernel, small and large segments
TUNINGS = [(512, 384, 3), (512, 192, 2), (256, 192, 5), (256, 128, 4), (2048, 1024, 2), (4096, 2048, 1)]


@pytest.mark.parametrize("key", ["nemo", "km3"])
def test_every_tuning_gives_the_oracle_result(T, orc, key):
    """The ordering stage's launch choices (kernel variant, segment size, grid)
    never change a byte of the result; each setting is run twice so the second
    call replays the captured launch sequence."""
    from gen import configs as C
    w = (C.nemo if key == "nemo" else C.km3)(seed=23, length_ns=40_000_000, n_tracks=6)
    g, thr = w.geoms[key]
    s = w.slices[0][1]
    ref = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    with T.Trigger(0) as t2:
        gid = t2.load_geometry(g.floor_id, thr)
        dp, dt, dq = to_dev(s)
        for cap, tgt, grid in TUNINGS:
            T.trig_tune_set(t2.ctx, g.n_pmt, tgt, cap, grid)
            for _ in range(2):
                got = t2.slice(gid, dp, dt, dq, w.params, seed_flags=True)
                check(got, ref)
                assert got["path"] == 0, (cap, tgt, grid)


def test_repeat_is_bit_identical(tr):
    from gen import configs as C
    w = C.km3(seed=8, length_ns=50_000_000)
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    gid = gid_for(tr, g.floor_id, thr)
    dp, dt, dq = to_dev(s)
    first = tr.slice(gid, dp, dt, dq, w.params, seed_flags=True)
    for _ in range(9):
        again = tr.slice(gid, dp, dt, dq, w.params, seed_flags=True)
        assert np.array_equal(first["fires"], again["fires"])
        assert np.array_equal(first["events"], again["events"])
        assert np.array_equal(first["seed_flags"], again["seed_flags"])


def test_graph_replays_match_eager_with_work_between(tr, orc):
    """The launch sequence is captured into a HIP graph on its second use; every
    replay, with other slices (eager or captured) run in between, equals the
    first (eager) result and the oracle."""
    from gen import configs as C
    wa = C.km3(seed=31, length_ns=15_000_000)
    wb = C.nemo(seed=32, length_ns=25_000_000)
    ga, thra = wa.geoms["km3"]
    gb, thrb = wb.geoms["nemo"]
    sa, sb = wa.slices[0][1], wb.slices[0][1]
    ida, idb = gid_for(tr, ga.floor_id, thra), gid_for(tr, gb.floor_id, thrb)
    da, db = to_dev(sa), to_dev(sb)
    ra0 = tr.slice(ida, *da, wa.params, seed_flags=True)
    rb0 = tr.slice(idb, *db, wb.params, seed_flags=True)
    check(ra0, orc.run(sa.pmt, sa.t, sa.q, ga.floor_id, thra, wa.params))
    check(rb0, orc.run(sb.pmt, sb.t, sb.q, gb.floor_id, thrb, wb.params))
    seq = "aaabababbbaaab"
    for x in seq:
        if x == "a":
            r = tr.slice(ida, *da, wa.params, seed_flags=True)
            ref = ra0
        else:
            r = tr.slice(idb, *db, wb.params, seed_flags=True)
            ref = rb0
        assert np.array_equal(r["fires"], ref["fires"])
        assert np.array_equal(r["events"], ref["events"])
        assert np.array_equal(r["seed_flags"], ref["seed_flags"])


def test_dense_segment_takes_general_path(tr, orc):
    """A burst far denser than a segment's LDS capacity: the run-merge ordering hands
    the slice to the general radix path; results are unchanged."""
    from gen import configs as C
    w = C.km3(seed=9, length_ns=20_000_000, n_tracks=0)
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    rng = np.random.default_rng(3)
    k = 20000
    bt = s.t.min() + 5_000_000 + np.sort(rng.integers(0, 500, size=k))
    bp = np.full(k, 17, np.uint16)
    bq = rng.integers(0, 500, size=k).astype(np.uint16)
    pmt = np.concatenate([s.pmt, bp])
    t = np.concatenate([s.t, bt])
    q = np.concatenate([s.q, bq])
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, pmt, t, q, w.params, seed_flags=True)
    ref = orc.run(pmt, t, q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    # general ordering; the burst outruns the seed kernel's staged neighbours and
    # the fold kernel's staged window, which read past them in device memory
    assert got["path"] == 1


def test_dense_window_on_run_merge(tr, orc):
    """A short burst on one floor, far denser than the slice's mean but small
    enough for the run-merge ordering, straddling a tile boundary: the causal
    windows of its seeds span several tiles' seed lists; no rerun."""
    from gen import configs as C
    w = C.nemo(seed=11, length_ns=20_000_000, n_tracks=2)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    rng = np.random.default_rng(5)
    k = 240
    floor0 = np.flatnonzero(g.floor_id == g.floor_id[0])[:4].astype(np.uint16)
    # the burst straddles the boundary of trigger tiles 9 and 10 (ordered position 10240)
    t0 = np.sort(s.t)[10240 - k // 2] + 1
    bt = t0 + np.sort(rng.integers(0, 400, size=k))
    bp = rng.choice(floor0, size=k).astype(np.uint16)
    bq = rng.integers(50, 400, size=k).astype(np.uint16)
    # appended as one more time-ordered run per PMT
    order = np.lexsort((bt, bp))
    pmt = np.concatenate([s.pmt, bp[order]])
    t = np.concatenate([s.t, bt[order]])
    q = np.concatenate([s.q, bq[order]])
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, pmt, t, q, w.params, seed_flags=True)
    ref = orc.run(pmt, t, q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    assert got["path"] == 0 and got["n_fires"] > 0


def test_fold_window_past_staged_tiles(tr, orc):
    """80 000 hits on one PMT within 2 us, a few of them over the charge threshold:
    the causal windows of the burst's seeds span more than 64 tiles, so the fold
    kernel reads the seed lists tile by tile from device memory, and the seed
    kernel's staged neighbours do not span t_floor_ns inside the burst."""
    from gen import configs as C
    w = C.nemo(seed=12, length_ns=20_000_000, n_tracks=2)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    rng = np.random.default_rng(7)
    k = 80_000
    bt = s.t.min() + 7_000_000 + np.sort(rng.integers(0, 2000, size=k))
    bp = np.full(k, 5, np.uint16)
    bq = rng.integers(0, 300, size=k).astype(np.uint16)
    bq[rng.random(k) < 0.002] = 400
    pmt = np.concatenate([s.pmt, bp])
    t = np.concatenate([s.t, bt])
    q = np.concatenate([s.q, bq])
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, pmt, t, q, w.params, seed_flags=True)
    ref = orc.run(pmt, t, q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    assert got["n_fires"] > 0


@pytest.mark.parametrize("window_cap", [512, 2048])
def test_floor_burst_denser_than_staged_neighbours(T, tr, orc, window_cap):
    """1500 hits on the four PMTs of one floor within 30 ns, none over the charge
    threshold (every hit a floor-coincidence seed): the seed kernel searches
    partners past its staged neighbours, and the fold windows hold 1500 seeds (in
    device memory with a 512-seed LDS window, staged with 2048)."""
    from gen import configs as C
    w = C.nemo(seed=13, length_ns=20_000_000, n_tracks=2)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    rng = np.random.default_rng(11)
    k = 1500
    floor0 = np.flatnonzero(g.floor_id == g.floor_id[0])[:4].astype(np.uint16)
    bt = np.sort(s.t)[30000] + 1 + np.sort(rng.integers(0, 30, size=k))
    bp = rng.choice(floor0, size=k).astype(np.uint16)
    bq = rng.integers(0, 200, size=k).astype(np.uint16)
    order = np.lexsort((bt, bp))
    pmt = np.concatenate([s.pmt, bp[order]])
    t = np.concatenate([s.t, bt[order]])
    q = np.concatenate([s.q, bq[order]])
    gid = gid_for(tr, g.floor_id, thr)
    cur = T.trig_tune_get(tr.ctx, 32)
    T.trig_tune_set(tr.ctx, 128, cur["seg_target"], cur["seg_cap"], cur["grid_per_cu"], window_cap=window_cap)
    try:
        got = tr.slice(gid, pmt, t, q, w.params, seed_flags=True)
    finally:
        T.trig_tune_set(tr.ctx, 128, cur["seg_target"], cur["seg_cap"], cur["grid_per_cu"],
                        window_cap=cur["window_cap"])
    ref = orc.run(pmt, t, q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    assert got["n_seeds"] >= k

def test_errors(T, tr):
    from gen import configs as C
    w = C.nemo(seed=4, length_ns=5_000_000)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    gid = gid_for(tr, g.floor_id, thr)
    bad = s.pmt.copy()
    bad[17] = 32
    r = tr.slice(gid, bad, s.t, s.q, w.params)
    assert r["status"] == T.TRIG_ERANGE
    t2 = s.t.copy()
    t2[3] = t2.min() + (1 << 31)
    r = tr.slice(gid, s.pmt, t2, s.q, w.params)
    assert r["status"] == T.TRIG_ERANGE
    ok = tr.slice(gid, s.pmt, s.t, s.q, dict(w.params, min_fold=1))
    assert ok["n_fires"] > 2
    small = tr.slice(gid, s.pmt, s.t, s.q, dict(w.params, min_fold=1), fire_cap=1, event_cap=1)
    assert small["status"] == T.TRIG_EOVERFLOW
    assert small["n_fires"] == ok["n_fires"] and small["n_events"] == ok["n_events"]
    with pytest.raises(T.TrigError):
        T.trig_slice(tr.ctx, 12345, s.pmt, s.t, s.q, w.params)


def test_batch_matches_alone_and_oracle(tr, orc):
    from gen import configs as C
    w = C.batch(seed=2, n_slices=24, scale=0.08)
    gids = {k: gid_for(tr, g.floor_id, thr) for k, (g, thr) in w.geoms.items()}
    sl = [(gids[k], s.pmt, s.t, s.q) for k, s in w.slices]
    bad = w.slices[5][1].pmt.copy()
    bad[0] = 500
    sl[5] = (sl[5][0], bad, sl[5][2], sl[5][3])
    res = tr.batch(sl, w.params, seed_flags=True)
    assert res[5]["status"] == -2
    for i, (k, s) in enumerate(w.slices):
        if i == 5:
            continue
        g, thr = w.geoms[k]
        ref = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
        check(res[i], ref)
        alone = tr.slice(gids[k], s.pmt, s.t, s.q, w.params, seed_flags=True)
        assert np.array_equal(alone["fires"], res[i]["fires"])
        assert np.array_equal(alone["events"], res[i]["events"])


def test_block_slice_reduced(tr, orc):
    """2688-PMT block (dense 2688^2 table, row groups on the 8 XCDs), 20 ms."""
    from gen import configs as C
    w = C.block_workload(seed=3, length_ns=20_000_000, n_tracks=20)
    g, thr = w.geoms["block"]
    s = w.slices[0][1]
    gid = gid_for(tr, g.floor_id, thr)
    dp, dt, dq = to_dev(s)
    got = tr.slice(gid, dp, dt, dq, w.params, seed_flags=True)
    ref = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    check(got, ref)
    assert got["path"] == 0   # (the two-level run merge)


def test_batch_many_slices_with_empty_ones(tr, orc):
    """150 slices (the slice lookup of a work item takes two levels of its 64-way
    search), among them empty and one-hit slices whose item ranges are empty and
    share a base with the next slice; every slice equals the oracle."""
    rng = np.random.default_rng(77)
    P = 12
    floor_id = (np.arange(P) // 3).astype(np.int32)
    thr = rng.integers(0, 2500, size=(P, P)).astype(np.uint32)
    gid = gid_for(tr, floor_id, thr)
    params = dict(q_seed=400, t_floor_ns=30, w_ns=2500, min_fold=2, half_event_ns=1500)
    items, raw = [], []
    for i in range(150):
        kind = i % 7
        n = 0 if kind in (0, 3) else 1 if kind == 5 else int(rng.integers(2, 6000))
        pmt = rng.integers(0, P, size=n).astype(np.uint16)
        t = np.sort(rng.integers(0, 3_000_000, size=n)).astype(np.int64) + int(rng.integers(0, 10**12))
        q = rng.integers(0, 600, size=n).astype(np.uint16)
        items.append((gid, pmt, t, q))
        raw.append((pmt, t, q))
    res = tr.batch(items, params, seed_flags=True)
    assert len(res) == 150
    for (pmt, t, q), r in zip(raw, res):
        ref = orc.run(pmt, t, q, floor_id, thr, params, "blocked")
        check(r, ref)


def test_one_pmt_burst_keeps_the_fast_ordering(tr, orc):
    """A 32-PMT slice at 40 kHz per PMT with one PMT at 3 MHz for 20 of its 60 ms.
    Sized for the mean density alone (2.3 MHz: 131 us segments) a segment in the
    burst would hold about 560 hits, past the 512 of a wave; sized for the mean
    plus the densest chunk the segments are half as wide, so the slice stays on
    the run-merge ordering (path 0) and equals the oracle."""
    from gen import configs as C
    from gen.slices import make_slice
    g, thr = C.geometry("nemo")
    s = make_slice(g, 60_000_000, 40e3, 91, n_tracks=3, bursts=[(5, 3.0e6, 20_000_000, 20_000_000)])
    span = int(s.t.max() - s.t.min()) + 1
    x_mean = 384 * span / s.n                    # the width rule at the mean density
    width = 1 << (int(x_mean).bit_length() - 1)
    burst_rate = (32 * 40e3 + 3.0e6) * 1e-9      # hits per ns inside the burst
    assert burst_rate * width > 512              # (so the case does test the rule)
    params = dict(C.DEFAULT_PARAMS)
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, s.pmt, s.t, s.q, params, seed_flags=True)
    check(got, orc.run(s.pmt, s.t, s.q, g.floor_id, thr, params, "blocked"))
    assert got["path"] == 0


@pytest.mark.parametrize("case", ["span_all_ones", "gap_and_burst"])
def test_two_level_merge_edges(tr, orc, case):
    """2688 per-PMT runs (more than a wave merges: two ordering levels, the second
    over the groups' ordered outputs, whose boundary table level 1 writes).
    span_all_ones: t_max - t_min = 2^24 - 1, so the last level-1 segment also
    owns the table's final row; gap_and_burst: 4 ms without hits (empty segments
    at both levels) and one PMT at 2 MHz.  Both stay on the run merge (path 0)
    and equal the oracle."""
    from gen import configs as C
    from gen.slices import make_slice
    g, thr = C.geometry("block")
    if case == "span_all_ones":
        T = 1 << 24
        s = make_slice(g, T, 20e3, 93, n_tracks=4)
        t = s.t.copy()
        t[np.flatnonzero(s.pmt == 0)[0]] = t.min()           # (the runs stay ordered)
        t[np.flatnonzero(s.pmt == 1)[-1]] = t.min() + T - 1
        pmt, q = s.pmt, s.q
        assert int(t.max() - t.min()) == T - 1
    else:
        s = make_slice(g, 30_000_000, 20e3, 94, n_tracks=4, bursts=[(7, 2.0e6, 2_000_000, 2_000_000)])
        rel = s.t - s.t.min()
        keep = (rel < 10_000_000) | (rel >= 14_000_000)
        t, pmt, q = s.t[keep], s.pmt[keep], s.q[keep]
    params = dict(C.DEFAULT_PARAMS)
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, pmt, t, q, params, seed_flags=True)
    check(got, orc.run(pmt, t, q, g.floor_id, thr, params, "blocked"))
    assert got["path"] == 0


def test_unaligned_device_inputs(tr, orc):
    """Device arrays that start one element into their allocations (times 8 bytes
    and PMT ids and charges 2 bytes past an aligned address): the ingest takes
    its scalar loads; the result equals the oracle and the aligned call."""
    import torch
    from gen import configs as C
    w = C.km3(seed=5, length_ns=20_000_000, n_tracks=3)
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    dev = torch.device("cuda:0")

    def shifted(a, dtype):
        x = torch.empty(len(a) + 1, dtype=dtype, device=dev)
        x[1:] = torch.from_numpy(np.ascontiguousarray(a).view(np.int16 if dtype == torch.int16 else np.int64)).to(dev)
        return x[1:]

    dp, dt, dq = shifted(s.pmt, torch.int16), shifted(s.t, torch.int64), shifted(s.q, torch.int16)
    assert dt.data_ptr() % 16 == 8 and dp.data_ptr() % 8 == 2
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, dp, dt, dq, w.params, seed_flags=True)
    check(got, orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked"))
    base = tr.slice(gid, *to_dev(s), w.params, seed_flags=True)
    assert np.array_equal(got["fires"], base["fires"]) and np.array_equal(got["seed_flags"], base["seed_flags"])


@pytest.mark.parametrize("tau", [65533, 65534, 70000])
def test_long_floor_window(tr, orc, tau):
    """Same-floor windows near and past 2^16 ns: the seed kernel's staged pair test
    holds up to 65533 ns and hands longer windows to its search over device
    memory; both equal the oracle."""
    from gen import configs as C
    w = C.nemo(seed=9, length_ns=4_000_000, n_tracks=2)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    params = dict(C.DEFAULT_PARAMS, t_floor_ns=tau)
    gid = gid_for(tr, g.floor_id, thr)
    got = tr.slice(gid, s.pmt, s.t, s.q, params, seed_flags=True)
    check(got, orc.run(s.pmt, s.t, s.q, g.floor_id, thr, params, "blocked"))


@pytest.mark.parametrize("seed", range(6))
def test_block_bounds_random_tables(tr, orc, seed):
    """Detectors of 256 PMTs or more: the fold kernel decides most pairs from
    lower and upper bounds of the table per pair of PMT blocks and reads the
    table only in between.  Random asymmetric tables with block structure at
    another granularity, entries of 0, exact multiples of 16 ns, beyond the
    bounds' 4064 ns range and beyond 65535, and windows below, at and past those
    limits (W > 65535 turns the bounds off): equal to the oracle."""
    rng = np.random.default_rng(7100 + seed)
    P = int(rng.integers(256, 900))
    gsz = int(rng.choice([8, 32, 50]))
    nb = (P + gsz - 1) // gsz
    base = rng.integers(0, 4200, size=(nb, nb))
    spread = int(rng.choice([1, 16, 300]))
    blk = np.arange(P) // gsz
    thr = (base[blk][:, blk] + rng.integers(0, spread, size=(P, P))).astype(np.uint32)
    u = rng.random((P, P))
    thr[u < 0.02] = 0
    thr[(u >= 0.02) & (u < 0.04)] = (thr[(u >= 0.02) & (u < 0.04)] // 16) * 16
    thr[(u >= 0.04) & (u < 0.05)] = rng.integers(4064, 70000, size=int(((u >= 0.04) & (u < 0.05)).sum()))
    floor_id = (np.arange(P) // 6).astype(np.int32)
    n = int(rng.integers(5000, 25000))
    pmt = rng.integers(0, P, size=n).astype(np.uint16)
    t = rng.integers(0, n * 40, size=n).astype(np.int64) + 10**15
    q = rng.integers(0, 600, size=n).astype(np.uint16)
    o = np.lexsort((t, pmt))   # runs per PMT
    pmt, t, q = pmt[o], t[o], q[o]
    w_ns = int(rng.choice([int(rng.integers(50, 5000)), 4064, 4080, 65535, 70000]))
    params = dict(q_seed=int(rng.integers(250, 500)), t_floor_ns=int(rng.integers(-1, 30)), w_ns=w_ns,
                  min_fold=int(rng.integers(2, 12)), half_event_ns=int(rng.integers(0, 3000)))
    gid = gid_for(tr, floor_id, thr)
    got = tr.slice(gid, pmt, t, q, params, seed_flags=True)
    check(got, orc.run(pmt, t, q, floor_id, thr, params, "blocked"))
    assert got["n_fires"] > 0
