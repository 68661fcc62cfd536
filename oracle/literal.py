"""Literal trigger oracle in plain Python loops (tiny inputs only).

TEST INFRASTRUCTURE ONLY: used by the tests to pin the C oracle; the product
library never imports it.  It shares no code with the C oracle or with the
HIP library: it is the rule, written out once more from the paper.

Paper: Bouhadef, Morganti, Terreni, "Parallel Neutrino Triggers using GPUs
for an Underwater Telescope" (GPUHEP2014).

* seed (Sec. 4.2 trigger list: QTRIG charge over threshold and FC floor
  coincidence; Sec. 3 charge trigger): a hit is a seed if its charge reaches
  ``q_seed``, or if another PMT on the same floor has a hit within
  ``t_floor_ns`` of it (inclusive; ``t_floor_ns < 0`` switches this off).
* fold (Sec. 3 space-time correlation within less than 3 us): a seed's fold
  is one (itself) plus the number of other seeds whose time differs from its
  own by at most ``min(thr[own pmt][their pmt], w_ns)``.
* fire: a seed with fold >= ``min_fold``; fires are listed by time, then
  PMT, then input position.
* events (Sec. 2: 6 us window centred on the trigger seed; Sec. 4.2: hits
  within +-3 us are tagged): each fire spans [t - H, t + H]; consecutive
  fires whose spans meet or overlap belong to one event.

Inputs are Python sequences; ``thr`` is a list of rows.  Returns a dict with
``status`` (0, or -2 when the input is outside the accepted range),
``seed``, ``fold`` (per input position), ``fires`` as tuples
``(t, hit_index, fold, pmt)`` and ``events`` as tuples
``(t_trig, t_begin, t_end, n_fire, max_fold)``.
"""
from __future__ import annotations

INT64_MIN = -(2 ** 63)
INT64_MAX = 2 ** 63 - 1


def in_range(pmt, t, n_pmt, half_event_ns):
    """The accepted input range: PMT below P, time span below 2^31 ns, windows fit int64."""
    if len(t) >= 2 ** 32:
        return False
    for p in pmt:
        if p >= n_pmt:
            return False
    if not t:
        return True
    lo, hi = min(t), max(t)
    if hi - lo >= 2 ** 31:
        return False
    return lo - half_event_ns >= INT64_MIN and hi + half_event_ns <= INT64_MAX


def is_seed(k, pmt, t, q, floor_id, q_seed, t_floor_ns):
    if q[k] >= q_seed:
        return True
    if t_floor_ns < 0:
        return False
    for m in range(len(t)):
        if pmt[m] != pmt[k] and floor_id[pmt[m]] == floor_id[pmt[k]] and abs(t[k] - t[m]) <= t_floor_ns:
            return True
    return False


def fold_of(k, pmt, t, seed, thr, w_ns):
    count = 1
    for m in range(len(t)):
        if m == k or not seed[m]:
            continue
        if abs(t[k] - t[m]) <= min(thr[pmt[k]][pmt[m]], w_ns):
            count += 1
    return count


def run(pmt, t, q, floor_id, thr, q_seed=300, t_floor_ns=20, w_ns=3000, min_fold=4, half_event_ns=3000):
    pmt, t, q = [int(x) for x in pmt], [int(x) for x in t], [int(x) for x in q]
    n_pmt = len(floor_id)
    if not in_range(pmt, t, n_pmt, half_event_ns):
        return dict(status=-2, seed=[], fold=[], fires=[], events=[])
    n = len(t)
    seed = [is_seed(k, pmt, t, q, floor_id, q_seed, t_floor_ns) for k in range(n)]
    fold = [fold_of(k, pmt, t, seed, thr, w_ns) if seed[k] else 0 for k in range(n)]
    fires = sorted((t[k], k, fold[k], pmt[k]) for k in range(n) if seed[k] and fold[k] >= min_fold)
    fires.sort(key=lambda f: (f[0], f[3], f[1]))
    events = []
    for (tf, _k, fd, _p) in fires:
        if events and tf - half_event_ns <= events[-1][2]:
            t_trig, begin, _end, nfire, mx = events[-1]
            events[-1] = (t_trig, begin, tf + half_event_ns, nfire + 1, max(mx, fd))
        else:
            events.append((tf, tf - half_event_ns, tf + half_event_ns, 1, fd))
    return dict(status=0, seed=[int(s) for s in seed], fold=fold, fires=fires, events=events)
