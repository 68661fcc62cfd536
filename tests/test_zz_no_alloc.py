"""The allocation-free entry point (trig_slice_noalloc) against trig_slice on
the GPU: the same fires, events, seed flags and tagged hits on two calls in a
row (the second with a smaller slice), on the general and dense paths and a
tiny slice, and its errors (host inputs, a slice beyond the fixed scratch)."""
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


def dev(s):
    import torch
    d = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(s.pmt).view(np.int16)).to(d),
            torch.from_numpy(np.ascontiguousarray(s.t)).to(d),
            torch.from_numpy(np.ascontiguousarray(s.q).view(np.int16)).to(d))


def same(a, b, keys=("fires", "events")):
    assert a["status"] == b["status"] == 0
    assert (a["n_seeds"], a["n_fires"], a["n_events"], a["path"]) == (b["n_seeds"], b["n_fires"], b["n_events"],
                                                                      b["path"])
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


def test_two_calls_in_a_row_equal_trig_slice(T):
    """A full 84-PMT slice, then a smaller one: each equals trig_slice (with seed
    flags and the tagged-hit list), and the first equals it again afterwards."""
    from gen import configs as C
    big = C.km3(seed=1)
    small = C.km3(seed=7, length_ns=30_000_000, n_tracks=4)
    g, thr = big.geoms["km3"]
    with T.Trigger(0) as tr:
        gid = tr.load_geometry(g.floor_id, thr)
        outs = []
        for w in (big, small, big):
            d = dev(w.slices[0][1])
            ref = tr.slice(gid, *d, w.params, seed_flags=True, tagged=True)
            got = T.trig_slice_noalloc(tr.ctx, gid, *d, w.params, seed_flags=True, tagged=True)
            same(got, ref, ("fires", "events", "seed_flags", "tagged"))
            outs.append(got)
        assert outs[1]["n_hits"] < outs[0]["n_hits"]


def _dense_window_slice():
    """A NEMO-like slice with a short burst on one floor, far denser than the
    slice's mean (causal windows over several tiles' seed lists)."""
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
    return (g, thr, np.concatenate([s.pmt, bp[order]]), np.concatenate([s.t, bt[order]]),
            np.concatenate([s.q, bq[order]]))


def test_general_dense_and_tiny_paths(T):
    """A shuffled slice (general ordering), level 0 on it, a slice with a dense
    burst, and a shuffled slice of at most 30 hits: all
    equal trig_slice."""
    import torch
    from gen import configs as C
    gk, thk = C.geometry("km3")
    shuffled = C.km3(seed=3, length_ns=40_000_000, n_tracks=4, order="shuffled").slices[0][1]
    tiny = C.km3(seed=4, length_ns=5_000, n_tracks=0, order="shuffled").slices[0][1]
    assert 0 < tiny.n <= 30
    prm = dict(C.DEFAULT_PARAMS)
    gn, thn, dp, dt, dq = _dense_window_slice()
    d0 = torch.device("cuda:0")
    dense = (torch.from_numpy(dp.view(np.int16)).to(d0), torch.from_numpy(dt).to(d0),
             torch.from_numpy(dq.view(np.int16)).to(d0))
    with T.Trigger(0) as tr:
        gid = tr.load_geometry(gk.floor_id, thk)
        gid_n = tr.load_geometry(gn.floor_id, thn)
        cases = ((gid, dev(shuffled), prm, 1), (gid, dev(shuffled), dict(prm, l0_n=7, l0_tw_ns=500), 1),
                 (gid_n, dense, prm, 0), (gid, dev(tiny), dict(prm, q_seed=0, min_fold=1), None))
        for g_id, d, p, path in cases:
            ref = tr.slice(g_id, *d, p, seed_flags=True)
            got = T.trig_slice_noalloc(tr.ctx, g_id, *d, p, seed_flags=True)
            same(got, ref, ("fires", "events", "seed_flags"))
            assert path is None or got["path"] == path


def test_errors(T):
    """Host inputs are refused; a slice larger than the fixed scratch gets
    TRIG_ENOMEM with the sizes in the message, and the next call still works."""
    import torch
    from gen import configs as C
    w = C.km3(seed=2, length_ns=10_000_000, n_tracks=2)
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    n_big = 2_800_000
    d0 = torch.device("cuda:0")
    big = (torch.zeros(n_big, dtype=torch.int16, device=d0),
           torch.arange(n_big, dtype=torch.int64, device=d0) + 1_400_000_000_000_000_000,
           torch.zeros(n_big, dtype=torch.int16, device=d0))
    with T.Trigger(0) as tr:
        gid = tr.load_geometry(g.floor_id, thr)
        r = T.trig_slice_noalloc(tr.ctx, gid, s.pmt, s.t, s.q, w.params, raise_on_error=False)
        assert r["status"] == T.TRIG_EINVAL
        r = T.trig_slice_noalloc(tr.ctx, gid, *big, w.params, raise_on_error=False)
        assert r["status"] == T.TRIG_ENOMEM
        assert "fixed scratch" in T.trig_last_error(tr.ctx)
        d = dev(s)
        same(T.trig_slice_noalloc(tr.ctx, gid, *d, w.params), tr.slice(gid, *d, w.params))
