"""GPU parity of the tagged-hit lists (the hits inside the merged event windows,
in (time, PMT, input index) order) against the oracle, on the ordinary, general
(shuffled input) orderings and a dense burst, in batches, with many events per tile,
and at full size; exact equality of the index lists."""
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
def tr(T):
    t = T.Trigger(0)
    yield t
    t.close()


@pytest.fixture(scope="module")
def orc():
    from oracle import cpu
    return cpu


def check_tagged(got, pmt, t, q, floor_id, thr, params, orc):
    ref = orc.run(pmt, t, q, floor_id, thr, params, "blocked")
    want = orc.tag(pmt, t, ref["fires"], params.get("half_event_ns", 3000))
    assert got["status"] == 0
    assert np.array_equal(got["fires"], ref["fires"]) and np.array_equal(got["events"], ref["events"])
    assert got["n_tagged"] == len(want)
    assert np.array_equal(got["tagged"], want)
    return ref, want


@pytest.mark.parametrize("order", ["runs", "shuffled"])
@pytest.mark.parametrize("key", ["nemo", "km3"])
def test_tower_slices(tr, orc, key, order):
    from gen import configs as C
    w = (C.nemo if key == "nemo" else C.km3)(seed=31, length_ns=30_000_000, n_tracks=6, order=order)
    g, thr = w.geoms[key]
    s = w.slices[0][1]
    gid = tr.load_geometry(g.floor_id, thr)
    got = tr.slice(gid, s.pmt, s.t, s.q, w.params, tagged=True)
    _, want = check_tagged(got, s.pmt, s.t, s.q, g.floor_id, thr, w.params, orc)
    assert len(want) > 0
    assert got["path"] == (1 if order == "shuffled" else 0)


@pytest.mark.parametrize("seed", range(6))
def test_random_slices(tr, orc, seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 40000))
    n_pmt = int(rng.integers(2, 40))
    floor_id = rng.integers(0, 5, size=n_pmt).astype(np.int32)
    thr = rng.integers(0, 4000, size=(n_pmt, n_pmt)).astype(np.uint32)
    pmt = rng.integers(0, n_pmt, size=n).astype(np.uint16)
    t = rng.integers(0, int(rng.integers(10_000, 5_000_000)), size=n).astype(np.int64) + 10**15
    q = rng.integers(0, 600, size=n).astype(np.uint16)
    params = dict(q_seed=400, t_floor_ns=20, w_ns=3000, min_fold=int(rng.integers(1, 5)),
                  half_event_ns=int(rng.integers(0, 4000)))
    gid = tr.load_geometry(floor_id, thr)
    got = tr.slice(gid, pmt, t, q, params, tagged=True)
    check_tagged(got, pmt, t, q, floor_id, thr, params, orc)


def test_many_events_in_one_tile(tr, orc):
    """Every hit a seed that fires, with windows of 1 ns and hits 3 ns apart: one
    event per hit, far more than the LDS list of a tile holds."""
    n = 5000
    pmt = (np.arange(n) % 7).astype(np.uint16)
    t = (np.arange(n, dtype=np.int64) * 3) + 77
    q = np.full(n, 500, np.uint16)
    floor_id = np.zeros(7, np.int32)
    thr = np.zeros((7, 7), np.uint32)
    params = dict(q_seed=300, t_floor_ns=-1, w_ns=0, min_fold=1, half_event_ns=1)
    gid = tr.load_geometry(floor_id, thr)
    got = tr.slice(gid, pmt, t, q, params, tagged=True)
    ref, want = check_tagged(got, pmt, t, q, floor_id, thr, params, orc)
    assert len(ref["events"]) == n and len(want) == n


def test_edge_cases(T, tr, orc):
    floor_id = np.zeros(4, np.int32)
    thr = np.full((4, 4), 100, np.uint32)
    gid = tr.load_geometry(floor_id, thr)
    e = np.zeros(0, np.uint16)
    got = tr.slice(gid, e, np.zeros(0, np.int64), e, None, tagged=True)
    assert got["status"] == 0 and got["n_tagged"] == 0 and len(got["tagged"]) == 0
    # no fires: nothing tagged
    rng = np.random.default_rng(3)
    n = 3000
    pmt = rng.integers(0, 4, size=n).astype(np.uint16)
    t = np.sort(rng.integers(0, 10**9, size=n)).astype(np.int64)
    q = np.zeros(n, np.uint16)
    got = tr.slice(gid, pmt, t, q, dict(t_floor_ns=-1), tagged=True)
    assert got["n_fires"] == 0 and got["n_tagged"] == 0
    # a window wider than the slice: every hit, in (time, PMT, index) order
    q2 = q.copy()
    q2[1234] = 500
    prm = dict(t_floor_ns=-1, min_fold=1, half_event_ns=2 * 10**9)
    got = tr.slice(gid, pmt, t, q2, prm, tagged=True)
    check_tagged(got, pmt, t, q2, floor_id, thr, prm, orc)
    assert got["n_tagged"] == n
    # a list longer than the caller's room: TRIG_EOVERFLOW with the count, no list
    got = tr.slice(gid, pmt, t, q2, prm, tagged=True, tagged_cap=10, raise_on_error=False)
    assert got["status"] == T.TRIG_EOVERFLOW and got["n_tagged"] == n


def test_dense_window(tr, orc):
    """A dense burst on one floor straddling a tile boundary: the tagged list
    follows its events."""
    from gen import configs as C
    w = C.nemo(seed=11, length_ns=20_000_000, n_tracks=2)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    rng = np.random.default_rng(5)
    k = 240
    floor0 = np.flatnonzero(g.floor_id == g.floor_id[0])[:4].astype(np.uint16)
    t0 = np.sort(s.t)[10240 - k // 2] + 1
    bt = t0 + np.sort(rng.integers(0, 400, size=k))
    bp = rng.choice(floor0, size=k).astype(np.uint16)
    bq = rng.integers(50, 400, size=k).astype(np.uint16)
    order = np.lexsort((bt, bp))
    pmt = np.concatenate([s.pmt, bp[order]])
    t = np.concatenate([s.t, bt[order]])
    q = np.concatenate([s.q, bq[order]])
    gid = tr.load_geometry(g.floor_id, thr)
    got = tr.slice(gid, pmt, t, q, w.params, tagged=True)
    check_tagged(got, pmt, t, q, g.floor_id, thr, w.params, orc)
    assert got["path"] == 0


def test_batch_mixed(tr, orc):
    """A batch of two tower types and uneven lengths; every slice's list equals
    the oracle's and the slice triggered alone."""
    from gen import configs as C
    items = []
    for i, (mk, key) in enumerate([(C.nemo, "nemo"), (C.km3, "km3"), (C.km3, "km3"), (C.nemo, "nemo")]):
        w = mk(seed=40 + i, length_ns=(10 + 7 * i) * 1_000_000, n_tracks=4)
        g, thr = w.geoms[key]
        items.append((w, g, thr, w.slices[0][1]))
    gids = [tr.load_geometry(g.floor_id, thr) for _, g, thr, _ in items]
    res = tr.batch([(gid, s.pmt, s.t, s.q) for gid, (_, _, _, s) in zip(gids, items)], items[0][0].params,
                   tagged=True)
    for gid, (w, g, thr, s), r in zip(gids, items, res):
        check_tagged(r, s.pmt, s.t, s.q, g.floor_id, thr, w.params, orc)
        alone = tr.slice(gid, s.pmt, s.t, s.q, w.params, tagged=True)
        assert np.array_equal(alone["tagged"], r["tagged"])


def test_full_size_km3(tr, orc):
    import torch
    from gen import configs as C
    w = C.km3()
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    gid = tr.load_geometry(g.floor_id, thr)
    d = torch.device("cuda:0")
    dp = torch.from_numpy(s.pmt.view(np.int16)).to(d)
    dt = torch.from_numpy(s.t).to(d)
    dq = torch.from_numpy(s.q.view(np.int16)).to(d)
    got = tr.slice(gid, dp, dt, dq, w.params, tagged=True)
    _, want = check_tagged(got, s.pmt, s.t, s.q, g.floor_id, thr, w.params, orc)
    assert len(want) > 1000
