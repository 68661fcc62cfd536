"""Pins of the synthetic input generator against the paper's workload facts."""
import math

import numpy as np

from gen import configs as C
from gen import geometry as G
from gen.slices import concat_runs_order, make_slice


def test_tower_geometry_matches_paper():
    g = G.nemo_tower()                          # Sec. 2: 8 floors x 4 DUs, 40 m apart, 6 m floor
    assert g.n_pmt == 32 and len(set(g.floor_id.tolist())) == 8
    z = sorted(set(np.round(g.pos[:, 2] - (g.pos[:, 2] % 40.0 > 20) * 0, 3).tolist()))
    assert abs(g.height - 280.0) < 1e-9
    assert np.allclose(np.abs(g.pos[:, :2]).max(), 3.0)
    k = G.km3net_it_tower()                     # Sec. 5: 14 floors, 20 m apart, 84 DUs
    assert k.n_pmt == 84 and len(set(k.floor_id.tolist())) == 14
    b = G.block()
    assert b.n_pmt == 2688 and len(set(b.floor_id.tolist())) == 32 * 14
    assert len(z) > 0


def test_thr_table_properties():
    for key in ("nemo", "km3"):
        g, thr = C.geometry(key)
        assert thr.dtype == np.uint32 and thr.shape == (g.n_pmt, g.n_pmt)
        assert np.array_equal(thr, thr.T)
        assert np.all(np.diag(thr) == 20) and thr.min() == 20
        d = np.linalg.norm(g.pos[0] - g.pos[-1])
        assert thr[0, -1] == math.ceil(1.35 * d / 0.299792458) + 20
    g, thr = C.geometry("block")
    assert 3000 < thr.max() < 3500 and 0.005 < (thr > 3000).mean() < 0.02


def test_hit_rates_match_paper():
    # Sec. 3: about 1.7 Mhits/s per 32-PMT tower and 4.6 Mhits/s per 84-PMT tower at 55 kHz
    for key, mhz in (("nemo", 1.76), ("km3", 4.62)):
        g, _ = C.geometry(key)
        s = make_slice(g, 50_000_000, 55_000.0, 3)
        expect = g.n_pmt * 55_000.0 * 0.05
        assert abs(s.n - expect) < 5 * math.sqrt(expect)
        assert abs(s.n / 0.05 / 1e6 - mhz) < 0.05
        assert concat_runs_order(s)


def test_bioluminescence_burst_plus_40_percent():
    # Sec. 4.1: two PMTs at 1 MHz among 84 at 55 kHz raise the hit count by about 40 %
    g, _ = C.geometry("km3")
    T = 20_000_000
    base = make_slice(g, T, 55_000.0, 4)
    burst = make_slice(g, T, 55_000.0, 4, bursts=[(3, 1e6, 0, T), (40, 1e6, 0, T)])
    ratio = burst.n / base.n
    assert abs(ratio - (84 * 55e3 + 2e6) / (84 * 55e3)) < 0.02
    assert 1.35 < ratio < 1.48


def test_generator_is_seeded_and_orders():
    g, _ = C.geometry("nemo")
    a = make_slice(g, 2_000_000, 55e3, 9, n_tracks=2)
    b = make_slice(g, 2_000_000, 55e3, 9, n_tracks=2)
    assert np.array_equal(a.t, b.t) and np.array_equal(a.q, b.q) and np.array_equal(a.pmt, b.pmt)
    c = make_slice(g, 2_000_000, 55e3, 9, n_tracks=2, order="shuffled")
    assert sorted(zip(a.t.tolist(), a.pmt.tolist(), a.q.tolist())) == sorted(zip(c.t.tolist(), c.pmt.tolist(), c.q.tolist()))
    for ta, tc in zip(a.tracks, c.tracks):
        assert np.array_equal(np.sort(ta.t), np.sort(c.t[tc.hit_index]))


def test_full_size_counts():
    s = C.km3().slices[0][1]
    assert abs(s.n - 924_000) < 5000 and len(s.tracks) == 20
    specs = C.batch_specs()
    assert len(specs) == 256
    tot = sum((32 if sp["key"] == "nemo" else 84) * sp["rate_hz"] * sp["length_ns"] * 1e-9 for sp in specs)
    assert 1.2e8 < tot < 2.5e8
    assert 10 <= sum(1 for sp in specs if sp["bursts"]) <= 45


def test_bar_end_groups():
    """Groups are the PMTs at one end of one floor's bar: half a floor each, one
    floor and one horizontal position per group."""
    from gen import geometry as G
    for geom, per_floor in ((G.nemo_tower(), 4), (G.km3net_it_tower(), 6)):
        grp = G.bar_end_groups(geom)
        assert len(np.unique(grp)) == 2 * len(np.unique(geom.floor_id))
        for k in np.unique(grp):
            m = grp == k
            assert m.sum() == per_floor // 2
            assert len(np.unique(geom.floor_id[m])) == 1
            assert np.allclose(geom.pos[m, :2], geom.pos[m, :2][0])


def test_block_floors_consecutive_only_within_a_tower():
    """In the 32-tower block, two PMTs whose floor ids differ by exactly 1 (an AFC
    pair) always belong to one tower, and every tower's own floors are
    consecutive; the same-floor (FC) pairs never cross towers either."""
    from gen import geometry as G
    g = G.block()
    f = g.floor_id.astype(np.int64)
    d = np.abs(f[:, None] - f[None, :])
    same_tower = g.tower_id[:, None] == g.tower_id[None, :]
    assert same_tower[d == 1].all()
    assert same_tower[d == 0].all()
    for k in np.unique(g.tower_id):
        fl = np.unique(f[g.tower_id == k])
        assert len(fl) == 14 and (np.diff(fl) == 1).all()
