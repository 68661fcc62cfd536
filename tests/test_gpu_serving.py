"""Serving loop on the GPU: each ticket's result equals the slice triggered alone,
while other slices overlap on the device; admission by HBM budget; cancellation."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1411_3968_amd import trig
    return trig


@pytest.fixture(scope="module")
def pool():
    from gen import configs as C
    return C.serving_pool(seed=4, n_pool=12, length_ns=20_000_000)


def _alone(T, pool):
    out = []
    with T.Trigger(0) as tr:
        g, thr = pool.geoms["km3"]
        gid = tr.load_geometry(g.floor_id, thr)
        for _, s in pool.slices:
            out.append(tr.slice(gid, s.pmt, s.t, s.q, pool.params))
    return out


def test_stream_results_equal_alone_under_overlap(T, pool):
    alone = _alone(T, pool)
    ctx = T.trig_create(0)
    try:
        g, thr = pool.geoms["km3"]
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        tickets = {}
        lock = threading.Lock()

        def producer(k):
            for i in range(k, len(pool.slices), 3):
                s = pool.slices[i][1]
                for rep in range(2):
                    st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params, tag=i)
                    assert st == 0
                    with lock:
                        tickets[(i, rep)] = tk

        ths = [threading.Thread(target=producer, args=(k,)) for k in range(3)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        for (i, rep), tk in tickets.items():
            st, r = T.trig_stream_poll(ctx, tk, -1, fire_cap=1 << 14, event_cap=1 << 14)
            assert st == 0 and r["tag"] == i
            assert np.array_equal(r["fires"], alone[i]["fires"])
            assert np.array_equal(r["events"], alone[i]["events"])
            assert r["n_seeds"] == alone[i]["n_seeds"]
        stats = T.trig_stream_stats_get(ctx)
        assert stats["completed"] == len(tickets) and stats["in_flight"] == 0
        assert stats["rounds"] >= 1
    finally:
        T.trig_destroy(ctx)


def test_admission_by_budget(T, pool):
    from gen import configs as C
    s = pool.slices[0][1]
    g, thr = pool.geoms["km3"]
    # a budget that holds a handful of slices of this size; rounds held back so
    # nothing completes while the budget fills
    ctx = T.trig_create(0, 64 << 20)
    try:
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        T.trig_stream_pause(ctx, True)
        got_again = False
        tks = []
        for _ in range(100):
            st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params)
            if st == T.TRIG_EAGAIN:
                got_again = True
                break
            assert st == 0
            tks.append(tk)
        assert got_again and len(tks) >= 2
        T.trig_stream_pause(ctx, False)
        for tk in tks:
            st, r = T.trig_stream_poll(ctx, tk, -1, fire_cap=1 << 14, event_cap=1 << 14)
            assert st == 0
        st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params)
        assert st == 0
        assert T.trig_stream_poll(ctx, tk, -1, fire_cap=1 << 14, event_cap=1 << 14)[0] == 0
        big = C.km3(seed=2).slices[0][1]
        st, _ = T.trig_stream_submit(ctx, gid, big.pmt, big.t, big.q, pool.params)
        assert st == T.TRIG_ENOMEM
    finally:
        T.trig_destroy(ctx)


def test_poll_overflow_then_deliver_and_errors(T, pool):
    s = pool.slices[1][1]
    g, thr = pool.geoms["km3"]
    ctx = T.trig_create(0)
    try:
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        prm = dict(pool.params, min_fold=1)
        st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, prm)
        assert st == 0
        st, r = T.trig_stream_poll(ctx, tk, -1, fire_cap=1, event_cap=1)
        assert st == T.TRIG_EOVERFLOW and r["n_fires"] > 1
        st, r2 = T.trig_stream_poll(ctx, tk, -1, fire_cap=r["n_fires"], event_cap=r["n_events"])
        assert st == 0 and r2["n_fires"] == r["n_fires"]
        assert T.trig_stream_poll(ctx, tk, 0)[0] == T.TRIG_EINVAL      # released
        bad = s.pmt.copy()
        bad[3] = 999
        st, tk = T.trig_stream_submit(ctx, gid, bad, s.t, s.q, prm)
        assert st == 0
        assert T.trig_stream_poll(ctx, tk, -1)[0] == T.TRIG_ERANGE
        st, _ = T.trig_stream_submit(ctx, 77, s.pmt, s.t, s.q, prm)
        assert st == T.TRIG_EINVAL
    finally:
        T.trig_destroy(ctx)


def test_destroy_with_tickets_in_flight(T, pool):
    g, thr = pool.geoms["km3"]
    ctx = T.trig_create(0)
    gid = T.trig_geom_load(ctx, g.floor_id, thr)
    for _, s in pool.slices[:8]:
        st, _ = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params)
        assert st == 0
    T.trig_destroy(ctx)      # drains running rounds, cancels the rest, frees everything


def test_next_done_reports_each_ticket_once(T, pool):
    """trig_stream_next_done hands out every finished ticket exactly once; the
    results then come from trig_stream_poll and equal the slices alone."""
    alone = _alone(T, pool)
    ctx = T.trig_create(0)
    try:
        g, thr = pool.geoms["km3"]
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        assert T.trig_stream_next_done(ctx, 0)[0] == T.TRIG_PENDING
        sub = {}
        for i, (_, s) in enumerate(pool.slices[:6]):
            st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params, tag=i)
            assert st == 0
            sub[tk] = i
        seen = []
        for _ in range(len(sub)):
            st, tk = T.trig_stream_next_done(ctx, -1)
            assert st == T.TRIG_OK and tk in sub and tk not in seen
            seen.append(tk)
            st, r = T.trig_stream_poll(ctx, tk, 0, fire_cap=1 << 14, event_cap=1 << 14)
            assert st == 0
            i = sub[tk]
            assert np.array_equal(r["fires"], alone[i]["fires"])
            assert np.array_equal(r["events"], alone[i]["events"])
        assert T.trig_stream_next_done(ctx, 1000)[0] == T.TRIG_PENDING
    finally:
        T.trig_destroy(ctx)


def test_long_result_lists_delivered_from_device(T, pool):
    """Fire lists longer than the pinned staging stay in the ticket's device region
    until the poll; they arrive whole and equal the slice triggered alone."""
    s = pool.slices[2][1]
    g, thr = pool.geoms["km3"]
    prm = dict(pool.params, q_seed=0, min_fold=1, half_event_ns=10)   # every hit fires
    with T.Trigger(0) as tr:
        gid = tr.load_geometry(g.floor_id, thr)
        ref = tr.slice(gid, s.pmt, s.t, s.q, prm)
    assert ref["n_fires"] == s.n
    ctx = T.trig_create(0)
    try:
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, prm)
        assert st == 0
        st, r = T.trig_stream_poll(ctx, tk, -1, fire_cap=16, event_cap=16)
        assert st == T.TRIG_EOVERFLOW and r is not None
        st, r = T.trig_stream_poll(ctx, tk, -1, fire_cap=s.n, event_cap=s.n)
        assert st == 0
        assert np.array_equal(r["fires"], ref["fires"])
        assert np.array_equal(r["events"], ref["events"])
    finally:
        T.trig_destroy(ctx)


def test_stream_submitter_equals_alone(T, pool):
    """Submissions through StreamSubmitter (descriptors built once, tag set per
    call) give each slice's own result, tags echoed."""
    alone = _alone(T, pool)
    ctx = T.trig_create(0)
    try:
        g, thr = pool.geoms["km3"]
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        sub = T.StreamSubmitter(ctx, [(gid, s.pmt, s.t, s.q) for _, s in pool.slices], pool.params)
        order = [3, 0, 7, 3, 11, 5]
        tickets = []
        for j, k in enumerate(order):
            rc, tk = sub(k, tag=100 + j)
            assert rc == T.TRIG_OK
            tickets.append((tk, k, 100 + j))
        for tk, k, tag in tickets:
            rc, r = T.trig_stream_poll(ctx, tk, timeout_us=-1, fire_cap=1 << 20, event_cap=1 << 20)
            assert rc == T.TRIG_OK and r["tag"] == tag
            assert r["n_fires"] == alone[k]["n_fires"] and r["n_events"] == alone[k]["n_events"]
            assert np.array_equal(r["fires"], alone[k]["fires"])
            assert np.array_equal(r["events"], alone[k]["events"])
    finally:
        T.trig_destroy(ctx)


def _oracle_lists(pool):
    from oracle import cpu as orc
    g, thr = pool.geoms["km3"]
    return [orc.run(s.pmt, s.t, s.q, g.floor_id, thr, pool.params, "blocked") for _, s in pool.slices]


def test_serving_pool_equals_oracle_alone_and_in_the_mix(T):
    """Every slice of a serving pool (rates 50-150 kHz per PMT, three slices at 5x
    rate) triggered through the stream loop, alone and with the whole pool in
    flight, gives the oracle's fires, events and seed count."""
    from gen import configs as C
    pool = C.serving_pool(seed=4, n_pool=10, length_ns=20_000_000, burst_frac=0.3)
    rates = [s.n for _, s in pool.slices]
    assert max(rates) > 3 * min(rates)          # the 5x slices are in the pool
    refs = _oracle_lists(pool)
    g, thr = pool.geoms["km3"]
    ctx = T.trig_create(0)
    try:
        gid = T.trig_geom_load(ctx, g.floor_id, thr)

        def check(k, st, r):
            assert st == 0
            assert r["n_seeds"] == int(refs[k]["seed"].sum())
            assert np.array_equal(r["fires"], refs[k]["fires"])
            assert np.array_equal(r["events"], refs[k]["events"])

        cap = max(max(len(r["fires"]), len(r["events"])) for r in refs) + 1
        for k, (_, s) in enumerate(pool.slices):          # alone: one ticket at a time
            st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params)
            assert st == 0
            check(k, *T.trig_stream_poll(ctx, tk, -1, fire_cap=cap, event_cap=cap))
        tks = []
        for rep in range(3):                                # in the mix: all in flight
            for k, (_, s) in enumerate(pool.slices):
                st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params)
                assert st == 0
                tks.append((tk, k))
        for tk, k in tks:
            check(k, *T.trig_stream_poll(ctx, tk, -1, fire_cap=cap, event_cap=cap))
    finally:
        T.trig_destroy(ctx)


def test_two_threads_polling_one_ticket(T, pool):
    """Two threads wait on the same ticket: exactly one receives the result, the
    other sees it pending or already delivered, and nothing is freed twice."""
    s = pool.slices[4][1]
    g, thr = pool.geoms["km3"]
    alone = _alone(T, pool)[4]
    ctx = T.trig_create(0)
    try:
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        for rep in range(12):
            T.trig_stream_pause(ctx, True)
            st, tk = T.trig_stream_submit(ctx, gid, s.pmt, s.t, s.q, pool.params)
            assert st == 0
            out = [None, None]

            def poller(j):
                out[j] = T.trig_stream_poll(ctx, tk, -1 if rep % 2 == 0 else 2_000_000,
                                            fire_cap=1 << 16, event_cap=1 << 16)

            ths = [threading.Thread(target=poller, args=(j,)) for j in range(2)]
            for th in ths:
                th.start()
            T.trig_stream_pause(ctx, False)
            for th in ths:
                th.join()
            codes = sorted(o[0] for o in out)
            assert codes.count(T.TRIG_OK) == 1, codes
            other = [c for c in codes if c != T.TRIG_OK][0]
            assert other in (T.TRIG_PENDING, T.TRIG_EINVAL), codes
            r = [o[1] for o in out if o[0] == T.TRIG_OK][0]
            assert np.array_equal(r["fires"], alone["fires"])
            assert np.array_equal(r["events"], alone["events"])
            # the ticket is gone for everybody now
            assert T.trig_stream_poll(ctx, tk, 0)[0] == T.TRIG_EINVAL
    finally:
        T.trig_destroy(ctx)


def test_slice_larger_than_a_chunk_after_the_arena_filled(T, pool):
    """The serving arena grows in chunks; once it has grown to the budget with
    small slices, a slice larger than any chunk is still admitted when the loop
    is idle (chunks holding no region are given back first) and gives the same
    result as alone."""
    from gen import configs as C
    g, thr = pool.geoms["km3"]
    small = pool.slices[0][1]
    big = C.km3(seed=5, length_ns=150_000_000, n_tracks=10).slices[0][1]   # ~700k hits
    with T.Trigger(0) as tr:
        gid0 = tr.load_geometry(g.floor_id, thr)
        ref = tr.slice(gid0, big.pmt, big.t, big.q, pool.params)
    budget = 512 << 20          # chunks of budget / 8 = 64 MiB
    ctx = T.trig_create(0, budget)
    try:
        gid = T.trig_geom_load(ctx, g.floor_id, thr)
        T.trig_stream_pause(ctx, True)
        tks = []
        while True:
            st, tk = T.trig_stream_submit(ctx, gid, small.pmt, small.t, small.q, pool.params)
            if st == T.TRIG_EAGAIN:
                break
            assert st == 0 and len(tks) < 200
            tks.append(tk)
        assert len(tks) >= 8
        st, _ = T.trig_stream_submit(ctx, gid, big.pmt, big.t, big.q, pool.params)
        assert st == T.TRIG_EAGAIN            # the small slices hold the arena
        T.trig_stream_pause(ctx, False)
        for tk in tks:
            assert T.trig_stream_poll(ctx, tk, -1, fire_cap=1 << 14, event_cap=1 << 14)[0] == 0
        st, tk = T.trig_stream_submit(ctx, gid, big.pmt, big.t, big.q, pool.params)
        assert st == 0, T.trig_last_error(ctx)
        st, r = T.trig_stream_poll(ctx, tk, -1, fire_cap=1 << 20, event_cap=1 << 20)
        assert st == 0
        assert np.array_equal(r["fires"], ref["fires"])
        assert np.array_equal(r["events"], ref["events"])
        assert T.trig_stream_stats_get(ctx)["device_bytes_peak"] <= budget
    finally:
        T.trig_destroy(ctx)
