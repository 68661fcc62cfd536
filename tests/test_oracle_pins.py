"""Pins of the oracle against facts outside itself.

* hand-worked boundary slices (tests/golden/hand_cases.json);
* the literal pure-Python rule, the strict all-pairs C form and the blocked C
  form agree on random and adversarial slices;
* closed forms: the floor-coincidence seed count of Poisson streams and the
  N-fold fire count of thinned Poisson seeds (Palm / Slivnyak);
* physics: injected Cherenkov tracks always fire and are covered by a window;
* invariances: time shift, input permutation, PMT relabelling.
"""
import math

import numpy as np
import pytest
from scipy import stats

from conftest import events_as_tuples, fires_as_tuples, load_hand_cases
from oracle import literal

HAND = load_hand_cases()


# ------------------------------------------------------------- hand cases

@pytest.mark.parametrize("case", HAND, ids=[c["name"] for c in HAND])
def test_hand_case_literal(case):
    r = literal.run(case["pmt"], case["t"], case["q"], list(case["floor_id"]), case["thr"].tolist(), **case["params"])
    assert r["status"] == case["status"], case["cite"]
    if case["status"] != 0:
        return
    assert r["seed"] == case["seed"]
    assert r["fold"] == case["fold"]
    assert [list(f) for f in r["fires"]] == case["fires"]
    assert [list(e) for e in r["events"]] == case["events"]


@pytest.mark.parametrize("form", ["strict", "blocked"])
@pytest.mark.parametrize("case", HAND, ids=[c["name"] for c in HAND])
def test_hand_case_c(oracle_lib, case, form):
    r = oracle_lib.run(case["pmt"], case["t"], case["q"], case["floor_id"], case["thr"], case["params"], form)
    assert r["status"] == case["status"], case["cite"]
    if case["status"] != 0:
        return
    assert r["seed"].tolist() == case["seed"]
    assert r["fold"].tolist() == case["fold"]
    assert [list(f) for f in fires_as_tuples(r["fires"])] == case["fires"]
    assert [list(e) for e in events_as_tuples(r["events"])] == case["events"]


# ------------------------------------------------- three forms agree

def _random_case(rng, n, n_pmt, n_floor, span, dense_frac=0.0, tie_frac=0.0):
    floor_id = rng.integers(0, n_floor, size=n_pmt).astype(np.int32)
    thr = rng.integers(0, 4000, size=(n_pmt, n_pmt)).astype(np.uint32)    # asymmetric on purpose
    pmt = rng.integers(0, n_pmt, size=n).astype(np.uint16)
    t = rng.integers(-span // 2, span // 2, size=n).astype(np.int64) + int(rng.integers(-10**17, 10**17))
    k = int(dense_frac * n)
    if k:
        t[:k] = t[0] + rng.integers(0, 200, size=k)                         # a dense burst
    k = int(tie_frac * n)
    if k:
        t[-k:] = t[-1] + rng.integers(0, 3, size=k)                         # many equal times
    q = rng.integers(0, 600, size=n).astype(np.uint16)
    params = dict(q_seed=int(rng.integers(200, 700)), t_floor_ns=int(rng.integers(-1, 60)),
                  w_ns=int(rng.integers(0, 5000)), min_fold=int(rng.integers(0, 7)),
                  half_event_ns=int(rng.integers(0, 5000)))
    return pmt, t, q, floor_id, thr, params


@pytest.mark.parametrize("seed", range(12))
def test_literal_strict_blocked_agree(oracle_lib, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 500))
    pmt, t, q, floor_id, thr, params = _random_case(rng, n, int(rng.integers(1, 12)), int(rng.integers(1, 4)),
                                                     int(rng.integers(10, 200000)), dense_frac=0.2 * (seed % 3 == 1),
                                                     tie_frac=0.3 * (seed % 3 == 2))
    lit = literal.run(pmt, t, q, floor_id.tolist(), thr.tolist(), **params)
    s = oracle_lib.run(pmt, t, q, floor_id, thr, params, "strict")
    b = oracle_lib.run(pmt, t, q, floor_id, thr, params, "blocked")
    assert lit["status"] == s["status"] == b["status"] == 0
    assert lit["seed"] == s["seed"].tolist() == b["seed"].tolist()
    assert lit["fold"] == s["fold"].tolist() == b["fold"].tolist()
    assert [tuple(f) for f in lit["fires"]] == fires_as_tuples(s["fires"]) == fires_as_tuples(b["fires"])
    assert [tuple(e) for e in lit["events"]] == events_as_tuples(s["events"]) == events_as_tuples(b["events"])


@pytest.mark.parametrize("seed", range(4))
def test_strict_blocked_agree_mid_size(oracle_lib, seed):
    rng = np.random.default_rng(2000 + seed)
    pmt, t, q, floor_id, thr, params = _random_case(rng, 20000, 30, 6, 3_000_000, dense_frac=0.02, tie_frac=0.02)
    s = oracle_lib.run(pmt, t, q, floor_id, thr, params, "strict")
    b = oracle_lib.run(pmt, t, q, floor_id, thr, params, "blocked")
    for k in ("seed", "fold", "fires", "events"):
        assert np.array_equal(s[k], b[k]), k


def test_strict_blocked_agree_nemo_slice(oracle_lib):
    from gen import configs as C
    w = C.nemo(seed=5, length_ns=40_000_000)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    a = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "strict")
    b = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    for k in ("seed", "fold", "fires", "events"):
        assert np.array_equal(a[k], b[k]), k
    assert len(a["fires"]) > 0


def test_point_oracle_matches_full(oracle_lib):
    from gen import configs as C
    w = C.km3(seed=3, length_ns=10_000_000)
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    full = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    rng = np.random.default_rng(9)
    ks = np.concatenate([rng.choice(s.n, 150, replace=False), np.nonzero(full["seed"])[0][:100]])
    seed, fold = oracle_lib.point(s.pmt, s.t, s.q, g.floor_id, thr, ks, w.params)
    assert np.array_equal(seed, full["seed"][ks])
    assert np.array_equal(fold, full["fold"][ks])


# ------------------------------------------------------------ closed forms

def _poisson_stream(rng, rate_per_ns, T):
    k = rng.poisson(rate_per_ns * T)
    return np.sort(rng.integers(0, T, size=k)).astype(np.int64)


def test_floor_coincidence_seed_rate_closed_form(oracle_lib):
    """Charge rule off, four PMTs on one floor at 1 MHz for 1 s.

    For independent Poisson streams at integer-ns times, a hit on PMT p has
    no partner within +-tau (inclusive) with probability
    exp(-(2 tau + 1) * sum_{p' != p} R_p'), so
    E[#seeds] = sum_p N_p (1 - exp(-(2 tau + 1) sum_{p' != p} N_p' / T)).
    The (2 tau + 1) versus 2 tau difference (an exclusive window) is >10 sigma.
    """
    rng = np.random.default_rng(77)
    T, R, tau = 1_000_000_000, 1e-3, 20
    streams = [_poisson_stream(rng, R, T) for _ in range(4)]
    pmt = np.concatenate([np.full(len(s), i, np.uint16) for i, s in enumerate(streams)])
    t = np.concatenate(streams)
    q = np.zeros(len(t), np.uint16)
    floor_id = np.zeros(4, np.int32)
    thr = np.full((4, 4), 20, np.uint32)
    r = oracle_lib.run(pmt, t, q, floor_id, thr, dict(q_seed=65536, t_floor_ns=tau, w_ns=3000, min_fold=99),
                       "blocked")
    N = np.array([len(s) for s in streams], dtype=np.float64)

    def expect(width):
        return sum(N[p] * (1 - math.exp(-width * (N.sum() - N[p]) / T)) for p in range(4))

    obs = int(r["seed"].sum())
    e_ok, e_excl = expect(2 * tau + 1), expect(2 * tau)
    sigma = math.sqrt(2.0 * e_ok)           # seeds come in correlated pairs: variance ~ 2 E
    assert abs(obs - e_ok) < 4 * sigma, (obs, e_ok, sigma)
    assert abs(obs - e_excl) > 6 * sigma     # the pin tells the two window conventions apart
    # pairs: (2 tau + 1) R1 R2 T per PMT pair
    pairs_expected = 6 * (2 * tau + 1) * R * R * T
    assert obs > 0.9 * pairs_expected


def test_nfold_fire_rate_closed_form(oracle_lib):
    """Floor rule off; charge seeds an independent thinning of Poisson streams.

    Given a seed on PMT p (Palm / Slivnyak), the other seeds within
    +-L_pp' (L = min(thr[p][p'], W), inclusive) of it are Poisson with mean
    mu_p = sum_p' R^s_p' (2 L_pp' + 1) (p' = p included), so
    E[#fires on p] = N^s_p * P(Poisson(mu_p) >= N - 1).
    The strongly asymmetric table makes a transposed lookup fail per PMT.
    """
    rng = np.random.default_rng(78)
    P, T, Rs = 8, 1_000_000_000, 5e-5
    W = 2500
    thr = np.where(np.arange(P)[:, None] > np.arange(P)[None, :], 2800, 150).astype(np.uint32)
    np.fill_diagonal(thr, 60)
    streams = [_poisson_stream(rng, Rs * 2, T) for _ in range(P)]
    pmt = np.concatenate([np.full(len(s), i, np.uint16) for i, s in enumerate(streams)])
    t = np.concatenate(streams)
    q = np.where(rng.random(len(t)) < 0.5, 400, 100).astype(np.uint16)
    r = oracle_lib.run(pmt, t, q, np.arange(P, dtype=np.int32), thr,
                       dict(q_seed=300, t_floor_ns=-1, w_ns=W, min_fold=4), "blocked")
    seeds = r["seed"].astype(bool)
    Ns = np.array([np.sum(seeds & (pmt == p)) for p in range(P)], dtype=np.float64)
    L = np.minimum(thr, W).astype(np.float64)

    def expected(table):
        mu = ((2 * table + 1) * (Ns / T)[None, :]).sum(1)
        return Ns * stats.poisson.sf(2, mu)           # P(X >= 3)

    e = expected(L)
    e_t = expected(L.T)
    fires_p = np.bincount(r["fires"]["pmt_id"], minlength=P).astype(np.float64)
    sig = np.sqrt(4.0 * e) + 5                         # fires cluster: generous variance
    assert np.all(np.abs(fires_p - e) < 5 * sig), (fires_p, e)
    assert np.any(np.abs(fires_p - e_t) > 10 * sig)     # transposed table is rejected
    assert fires_p.sum() > 5000


# ------------------------------------------------------------- physics

def test_injected_tracks_fire_and_are_covered(oracle_lib):
    """Every track with >= N charge-seeded hits that are pairwise causal fires, and
    one event window covers all those hits (Sec. 3: Cherenkov hits of one muon
    are correlated in time and space within 3 us)."""
    from gen import configs as C
    w = C.nemo(seed=0)
    g, thr = w.geoms["nemo"]
    s = w.slices[0][1]
    r = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked")
    fired = set(int(x) for x in r["fires"]["hit_index"])
    ev = r["events"]
    W, N = w.params["w_ns"], w.params["min_fold"]
    checked = 0
    pair_ok = pair_all = 0
    for tr in s.tracks:
        for a in range(len(tr.pmt)):
            for b in range(a + 1, len(tr.pmt)):
                pair_all += 1
                pair_ok += abs(int(tr.t[a]) - int(tr.t[b])) <= int(thr[tr.pmt[a], tr.pmt[b]])
        sel = [i for i in range(len(tr.pmt)) if tr.q[i] >= w.params["q_seed"]]
        if len(sel) < N:
            continue
        causal = all(abs(int(tr.t[a]) - int(tr.t[b])) <= min(int(thr[tr.pmt[a], tr.pmt[b]]), W)
                     for a in sel for b in sel if a != b)
        if not causal:
            continue
        checked += 1
        for i in sel:
            assert int(tr.hit_index[i]) in fired
        lo, hi = min(int(tr.t[i]) for i in sel), max(int(tr.t[i]) for i in sel)
        assert any(e["t_begin"] <= lo and hi <= e["t_end"] for e in ev)
    assert checked >= 3
    # jitter-free track pairs satisfy |dt| <= n d / c <= thr - 20; 3 ns jitter rarely breaks it
    assert pair_ok >= 0.99 * pair_all


# ----------------------------------------------------------- invariances

@pytest.fixture(scope="module")
def mid_slice():
    from gen import configs as C
    w = C.km3(seed=11, length_ns=8_000_000, n_tracks=6)
    g, thr = w.geoms["km3"]
    return w, g, thr, w.slices[0][1]


def test_time_shift_invariance(oracle_lib, mid_slice):
    w, g, thr, s = mid_slice
    a = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params)
    d = -1_400_000_000_000_000_000 - 123_457
    b = oracle_lib.run(s.pmt, s.t + d, s.q, g.floor_id, thr, w.params)
    assert np.array_equal(a["seed"], b["seed"]) and np.array_equal(a["fold"], b["fold"])
    assert np.array_equal(a["fires"]["t_ns"] + d, b["fires"]["t_ns"])
    assert np.array_equal(a["fires"]["hit_index"], b["fires"]["hit_index"])
    for k in ("t_trig", "t_begin", "t_end"):
        assert np.array_equal(a["events"][k] + d, b["events"][k])


def test_permutation_invariance(oracle_lib, mid_slice):
    w, g, thr, s = mid_slice
    a = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params)
    perm = np.random.default_rng(5).permutation(s.n)
    b = oracle_lib.run(s.pmt[perm], s.t[perm], s.q[perm], g.floor_id, thr, w.params)
    assert np.array_equal(a["seed"][perm], b["seed"]) and np.array_equal(a["fold"][perm], b["fold"])
    fb = b["fires"].copy()
    fb["hit_index"] = perm[fb["hit_index"]]
    # equal (t, pmt) keys may reorder with the input positions; compare as sorted records
    key = lambda f: np.lexsort((f["hit_index"], f["pmt_id"], f["t_ns"]))
    assert np.array_equal(a["fires"][key(a["fires"])], fb[key(fb)])
    assert np.array_equal(a["events"], b["events"])


def test_pmt_relabel_invariance(oracle_lib, mid_slice):
    w, g, thr, s = mid_slice
    a = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params)
    P = g.n_pmt
    pi = np.random.default_rng(6).permutation(P)           # old id -> new id
    floor2 = np.empty(P, np.int32)
    floor2[pi] = g.floor_id
    thr2 = np.empty_like(thr)
    thr2[np.ix_(pi, pi)] = thr
    b = oracle_lib.run(pi[s.pmt].astype(np.uint16), s.t, s.q, floor2, thr2, w.params)
    assert np.array_equal(a["seed"], b["seed"]) and np.array_equal(a["fold"], b["fold"])
    sa = sorted(zip(a["fires"]["hit_index"].tolist(), a["fires"]["t_ns"].tolist(), a["fires"]["fold"].tolist()))
    sb = sorted(zip(b["fires"]["hit_index"].tolist(), b["fires"]["t_ns"].tolist(), b["fires"]["fold"].tolist()))
    assert sa == sb
    assert np.array_equal(a["events"], b["events"])


# ------------------------------------------------------------- tagged hits

def _fires(rows):
    from oracle.cpu import FIRE_DTYPE
    f = np.zeros(len(rows), FIRE_DTYPE)
    for i, (t, k, fold, p) in enumerate(rows):
        f[i]["t_ns"], f[i]["hit_index"], f[i]["fold"], f[i]["pmt_id"] = t, k, fold, p
    return f


def test_tag_hand_example(oracle_lib):
    """Worked by hand: fires at 10 000, 10 500 and 30 000 ns with H = 3000 ns
    tag [7000, 13500] and [27000, 33000] (both ends inclusive); equal times
    order by PMT, then input position."""
    hits = [(5, 6999), (4, 7000), (1, 10000), (3, 10500), (0, 13500), (0, 13501), (2, 20000), (2, 30000),
            (7, 33000), (7, 33001), (2, 7000), (4, 7000), (6, 27000), (6, 26999)]
    pmt = np.array([h[0] for h in hits], np.uint16)
    t = np.array([h[1] for h in hits], np.int64)
    fires = _fires([(10000, 2, 4, 1), (10500, 3, 4, 3), (30000, 7, 5, 2)])
    got = oracle_lib.tag(pmt, t, fires, 3000)
    assert got.tolist() == [10, 1, 11, 2, 3, 4, 12, 7, 8]


def test_tag_equals_hits_inside_the_event_windows(oracle_lib, mid_slice):
    """The tagged hits are exactly those inside a merged event window (the
    events come from the separate merge walk over the fires)."""
    w, g, thr, s = mid_slice
    r = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params)
    assert len(r["events"]) > 0
    got = oracle_lib.tag(s.pmt, s.t, r["fires"], w.params["half_event_ns"])
    ev = r["events"]
    i = np.searchsorted(ev["t_begin"], s.t, side="right") - 1
    inside = (i >= 0) & (s.t <= ev["t_end"][np.maximum(i, 0)])
    idx = np.flatnonzero(inside)
    want = idx[np.lexsort((idx, s.pmt[idx], s.t[idx]))]
    assert np.array_equal(got, want.astype(np.uint32))
    assert len(got) > r["fires"].shape[0]


def test_tag_special_cases(oracle_lib, mid_slice):
    w, g, thr, s = mid_slice
    r = oracle_lib.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params)
    f = r["fires"]
    # no fires: nothing tagged
    assert len(oracle_lib.tag(s.pmt, s.t, f[:0], 3000)) == 0
    # a window wider than the slice around one fire: every hit, in (t, pmt, index) order
    allh = oracle_lib.tag(s.pmt, s.t, f[:1], 2**31 - 1)
    assert np.array_equal(allh, np.lexsort((np.arange(s.n), s.pmt, s.t)).astype(np.uint32))
    # H = 0: the hits at a fire's exact time (the fires among them)
    z = oracle_lib.tag(s.pmt, s.t, f, 0)
    assert set(z.tolist()) == set(np.flatnonzero(np.isin(s.t, f["t_ns"])).tolist())
    assert set(f["hit_index"].tolist()) <= set(z.tolist())


# ------------------------------------------------------------- level 0 (N hits in TW)

def _l0_flags(oracle_lib, pmt, t, n_pmt, form="strict", **l0):
    """Level-0 pass flags read through the seed rule: every charge is over a zero
    threshold and the floor rule is off, so a hit is a seed exactly when it passes."""
    pmt = np.asarray(pmt, np.uint16)
    t = np.asarray(t, np.int64)
    prm = dict(q_seed=0, t_floor_ns=-1, w_ns=0, min_fold=1, half_event_ns=0, **l0)
    r = oracle_lib.run(pmt, t, np.zeros(len(t), np.uint16), np.zeros(n_pmt, np.int32),
                       np.zeros((n_pmt, n_pmt), np.uint32), prm, form)
    assert r["status"] == 0
    return r["seed"].astype(bool)


@pytest.mark.parametrize("form", ["strict", "blocked"])
def test_l0_hand_example(oracle_lib, form):
    """Worked by hand, N = 3, TW = 100 ns: the windows [0, 100) and [260, 360)
    hold three hits each, and so do the three equal times at 1000; the hit at
    150 sees at most two (the window is half-open)."""
    t = [0, 40, 99, 150, 260, 300, 330, 1000, 1000, 1000]
    got = _l0_flags(oracle_lib, [0, 1, 2, 3, 0, 1, 2, 0, 1, 1], t, 4, form, l0_n=3, l0_tw_ns=100)
    assert got.tolist() == [True, True, True, False, True, True, True, True, True, True]
    # strict window: two hits 100 ns apart are not within TW = 100, 99 ns apart are
    assert _l0_flags(oracle_lib, [0, 1], [0, 100], 2, form, l0_n=2, l0_tw_ns=100).tolist() == [False, False]
    assert _l0_flags(oracle_lib, [0, 1], [0, 99], 2, form, l0_n=2, l0_tw_ns=100).tolist() == [True, True]


@pytest.mark.parametrize("form", ["strict", "blocked"])
def test_l0_distinct_pmts_hand_example(oracle_lib, form):
    """DN with N = 3, TW = 100 ns: four hits of two PMTs do not pass; a hit of a
    third PMT inside the window lets all five pass.  Counting hits (not PMTs),
    the four already pass."""
    pmt, t = [1, 1, 2, 2], [0, 10, 20, 50]
    assert not _l0_flags(oracle_lib, pmt, t, 4, form, l0_n=3, l0_tw_ns=100, l0_distinct=1).any()
    assert _l0_flags(oracle_lib, pmt, t, 4, form, l0_n=3, l0_tw_ns=100).all()
    assert _l0_flags(oracle_lib, pmt + [3], t + [90], 4, form, l0_n=3, l0_tw_ns=100, l0_distinct=1).all()


def test_l0_restricts_floor_partners(oracle_lib):
    """Floor coincidences count only between hits that pass level 0: E and F
    (t = 400, 410; the same floor) are partners but fail N = 3 in TW = 50 ns."""
    hits = [(0, 0), (10, 1), (20, 2), (400, 0), (410, 1), (1000, 0), (1005, 2), (1010, 3)]
    t = np.array([h[0] for h in hits], np.int64)
    pmt = np.array([h[1] for h in hits], np.uint16)
    floor_id = np.array([0, 0, 1, 1], np.int32)
    thr = np.zeros((4, 4), np.uint32)
    base = dict(q_seed=300, t_floor_ns=20, w_ns=0, min_fold=1, half_event_ns=0)
    q = np.zeros(len(t), np.uint16)
    for form in ("strict", "blocked"):
        on = oracle_lib.run(pmt, t, q, floor_id, thr, dict(base, l0_n=3, l0_tw_ns=50), form)
        off = oracle_lib.run(pmt, t, q, floor_id, thr, base, form)
        assert on["seed"].tolist() == [1, 1, 0, 0, 0, 0, 1, 1]
        assert off["seed"].tolist() == [1, 1, 0, 1, 1, 0, 1, 1]


@pytest.mark.parametrize("seed", range(4))
def test_l0_equals_consecutive_hits_form(oracle_lib, seed):
    """Counting hits, a hit passes exactly when it lies in some run of N hits
    that are consecutive in time order and span less than TW (the sliding form
    t[i + N - 1] - t[i] < TW), computed here with numpy on the sorted times."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(200, 3000))
    N, TW = int(rng.integers(2, 9)), int(rng.integers(50, 2000))
    t = rng.integers(0, n * 300, size=n).astype(np.int64)
    t[: n // 10] = t[0] + rng.integers(0, 3, size=n // 10)      # ties
    pmt = rng.integers(0, 8, size=n).astype(np.uint16)
    got = _l0_flags(oracle_lib, pmt, t, 8, "blocked", l0_n=N, l0_tw_ns=TW)
    order = np.lexsort((np.arange(n), pmt, t))
    ts = t[order]
    ok = np.zeros(n, bool)
    if n >= N:
        ok[: n - N + 1] = ts[N - 1:] - ts[: n - N + 1] < TW
    run_pass = np.convolve(ok.astype(int), np.ones(N, int))[:n] > 0   # some window start in [j-N+1, j]
    want = np.zeros(n, bool)
    want[order] = run_pass
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(4))
def test_l0_strict_blocked_and_variants_agree(oracle_lib, seed):
    """Strict (all windows, all members) and blocked forms agree; the distinct
    variant passes a subset; N = 1 is the same as no level 0."""
    rng = np.random.default_rng(950 + seed)
    n = int(rng.integers(100, 1500))
    P = 12
    t = rng.integers(0, n * 200, size=n).astype(np.int64) + 10**12
    pmt = rng.integers(0, P, size=n).astype(np.uint16)
    q = rng.integers(0, 600, size=n).astype(np.uint16)
    floor_id = rng.integers(0, 3, size=P).astype(np.int32)
    thr = rng.integers(0, 3000, size=(P, P)).astype(np.uint32)
    base = dict(q_seed=400, t_floor_ns=30, w_ns=3000, min_fold=2, half_event_ns=500)
    for l0 in (dict(l0_n=4, l0_tw_ns=800), dict(l0_n=4, l0_tw_ns=800, l0_distinct=1), dict(l0_n=7, l0_tw_ns=1000)):
        a = oracle_lib.run(pmt, t, q, floor_id, thr, dict(base, **l0), "strict")
        b = oracle_lib.run(pmt, t, q, floor_id, thr, dict(base, **l0), "blocked")
        assert np.array_equal(a["seed"], b["seed"]) and np.array_equal(a["fold"], b["fold"])
        assert np.array_equal(a["fires"], b["fires"]) and np.array_equal(a["events"], b["events"])
    dn = _l0_flags(oracle_lib, pmt, t, P, "blocked", l0_n=4, l0_tw_ns=800, l0_distinct=1)
    nn = _l0_flags(oracle_lib, pmt, t, P, "blocked", l0_n=4, l0_tw_ns=800)
    assert not (dn & ~nn).any() and dn.sum() < nn.sum()
    one = oracle_lib.run(pmt, t, q, floor_id, thr, dict(base, l0_n=1, l0_tw_ns=1), "blocked")
    off = oracle_lib.run(pmt, t, q, floor_id, thr, base, "blocked")
    assert np.array_equal(one["seed"], off["seed"]) and np.array_equal(one["fires"], off["fires"])


# ------------------------------------------------------------- seed menu (SC, FC, AFC)

# three floors x two bar ends x two PMTs; PMT = 4 floor + 2 end + j; adjacency group = bar end
MENU_FLOOR = np.repeat(np.arange(3), 4).astype(np.int32)
MENU_ADJ = np.repeat(np.arange(6), 2).astype(np.int32)
MENU_WIN = dict(q_seed=300, t_floor_ns=100, t_adj_ns=20, t_afloor_ns=250, w_ns=0, min_fold=1, half_event_ns=0)


@pytest.mark.parametrize("form", ["strict", "blocked"])
def test_seed_menu_hand_example(oracle_lib, form):
    """Worked by hand (SC 20 ns adjacent PMTs, FC 100 ns same floor, AFC 250 ns
    consecutive floors, all inclusive):
      h0 p0 t1000, h1 p1 t1015: SC (15), FC, AFC with h3      -> any / combination
      h2 p2 t1080: FC with h0 (80), AFC with h3 (120)          -> any / combination
      h3 p4 t1200: AFC only (floor 1 has no partner)           -> any
      h4 p8 t5000, h5 p9 t5010: SC and FC; h6 p5 t5300 too far  -> any (h4, h5)
      h7 p10 t9000, h8 p11 t9021: not SC (21 > 20) but FC       -> any / combination
      h9 p6 t9250: AFC with h7 at exactly 250                  -> any"""
    hits = [(0, 1000), (1, 1015), (2, 1080), (4, 1200), (8, 5000), (9, 5010), (5, 5300),
            (10, 9000), (11, 9021), (6, 9250)]
    pmt = np.array([h[0] for h in hits], np.uint16)
    t = np.array([h[1] for h in hits], np.int64)
    q = np.zeros(len(t), np.uint16)
    thr = np.zeros((12, 12), np.uint32)
    anyr = oracle_lib.run(pmt, t, q, MENU_FLOOR, thr, MENU_WIN, form, adj_id=MENU_ADJ)
    comb = oracle_lib.run(pmt, t, q, MENU_FLOOR, thr, dict(MENU_WIN, seed_mode=1), form, adj_id=MENU_ADJ)
    assert anyr["seed"].tolist() == [1, 1, 1, 1, 1, 1, 0, 1, 1, 1]
    assert comb["seed"].tolist() == [1, 1, 1, 0, 0, 0, 0, 1, 1, 0]
    # FC off: h4 and h5 are seeds through SC alone, and lose it without the
    # adjacency groups; AFC still holds for the others
    nofc = dict(MENU_WIN, t_floor_ns=-1)
    sc = oracle_lib.run(pmt, t, q, MENU_FLOOR, thr, nofc, form, adj_id=MENU_ADJ)
    noadj = oracle_lib.run(pmt, t, q, MENU_FLOOR, thr, nofc, form)
    assert sc["seed"].tolist() == [1, 1, 1, 1, 1, 1, 0, 1, 1, 1]
    assert noadj["seed"].tolist() == [1, 1, 1, 1, 0, 0, 0, 1, 1, 1]


def test_adjacent_floor_seed_rate_closed_form(oracle_lib):
    """Only the AFC rule, two PMTs on each of floors 0 and 1 at 1 MHz for 0.5 s:
    a hit on floor f has no partner on the other floor within +-tau with
    probability exp(-(2 tau + 1) R_other), so
    E[#seeds] = sum_p N_p (1 - exp(-(2 tau + 1) N_other(p) / T)).
    A same-floor partner must not count (the floors' own pairs are 3x as many)."""
    rng = np.random.default_rng(78)
    T, R, tau = 500_000_000, 1e-3, 30
    streams = [_poisson_stream(rng, R, T) for _ in range(4)]
    pmt = np.concatenate([np.full(len(s), i, np.uint16) for i, s in enumerate(streams)])
    t = np.concatenate(streams)
    q = np.zeros(len(t), np.uint16)
    floor_id = np.array([0, 0, 1, 1], np.int32)
    thr = np.full((4, 4), 20, np.uint32)
    prm = dict(q_seed=65536, t_floor_ns=-1, t_afloor_ns=tau, w_ns=0, min_fold=99)
    r = oracle_lib.run(pmt, t, q, floor_id, thr, prm, "blocked")
    N = np.array([len(s) for s in streams], dtype=np.float64)
    other = {0: N[2] + N[3], 1: N[2] + N[3], 2: N[0] + N[1], 3: N[0] + N[1]}
    e = sum(N[p] * (1 - math.exp(-(2 * tau + 1) * other[p] / T)) for p in range(4))
    obs = int(r["seed"].sum())
    sigma = math.sqrt(2.0 * e)
    assert abs(obs - e) < 4 * sigma, (obs, e, sigma)


@pytest.mark.parametrize("seed", range(4))
def test_seed_menu_strict_blocked_and_modes(oracle_lib, seed):
    rng = np.random.default_rng(970 + seed)
    n = int(rng.integers(200, 2000))
    P = 24
    floor_id = (np.arange(P) // 4).astype(np.int32)
    adj = (np.arange(P) // 2).astype(np.int32)
    thr = rng.integers(0, 3000, size=(P, P)).astype(np.uint32)
    t = rng.integers(0, n * 400, size=n).astype(np.int64) + 7 * 10**15
    pmt = rng.integers(0, P, size=n).astype(np.uint16)
    q = rng.integers(0, 600, size=n).astype(np.uint16)
    base = dict(q_seed=500, t_floor_ns=int(rng.integers(-1, 120)), t_adj_ns=int(rng.integers(-1, 40)),
                t_afloor_ns=int(rng.integers(-1, 300)), w_ns=3000, min_fold=2, half_event_ns=400)
    for extra in (dict(), dict(seed_mode=1), dict(seed_mode=1, l0_n=3, l0_tw_ns=600)):
        prm = dict(base, **extra)
        a = oracle_lib.run(pmt, t, q, floor_id, thr, prm, "strict", adj_id=adj)
        b = oracle_lib.run(pmt, t, q, floor_id, thr, prm, "blocked", adj_id=adj)
        assert np.array_equal(a["seed"], b["seed"]) and np.array_equal(a["fold"], b["fold"])
        assert np.array_equal(a["fires"], b["fires"]) and np.array_equal(a["events"], b["events"])
    any_ = oracle_lib.run(pmt, t, q, floor_id, thr, base, "blocked", adj_id=adj)["seed"]
    comb = oracle_lib.run(pmt, t, q, floor_id, thr, dict(base, seed_mode=1), "blocked", adj_id=adj)["seed"]
    assert not (comb.astype(bool) & ~any_.astype(bool)).any()
