"""Benchmark of the trigger hot path on one MI355X.

One step = one pass of the whole path (ingest, time-order merge, L1 seeds,
causal N-fold count, fire compaction, event windows, results to host) over one
synthetic 200 ms slice of a KM3Net-It-like tower (84 PMTs on 14 floors x 6,
55 kHz per PMT, about 924k hits, 20 injected muon tracks), inputs resident in
HBM before the timed region.  Prints one JSON line.

``--gpus N`` with N > 1 exits: the benchmark drives one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per input hit of each kernel (what its function must move,
# each byte counted once).
ALGO_BYTES_PER_HIT = {
    "k_ingest": 20.0,      # read t (8) + pmt (2) + q (2), write the packed word (8)
    "k_bounds": 8.0,       # read t (8); the boundary table is counted separately
    "k_segsort": 20.0,     # read the packed word (8) + write ordered t, pmt|q, index (12)
    "k_segsort_w": 20.0,   # the same, one wave per segment
    "k_tile": 8.0,         # read ordered t + pmt|q (8): seeds and causal folds; fires are per fire
    "k_tag_bits": 4.125,   # read ordered t (4) + write one tag bit; the few event windows are per event
}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` on this workload from the committed counter
    summary (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated with a plain copy), or
    None when there is none or the kernel's sources changed since it was taken."""
    import hashlib
    fn = os.path.join(ROOT, "profiles", "hbm_traffic_km3.json")
    if not os.path.exists(fn):
        return None
    with open(fn) as f:
        rec = json.load(f).get("kernels", {}).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, "paper_1411_3968_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return rec["traffic_bytes"] if h.hexdigest()[:16] == rec["sources_sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB once (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--batch-slices", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-form leg")
    ap.add_argument("--serve-pool", type=int, default=48, help="distinct pre-generated slices replayed")
    ap.add_argument("--serve-slices", type=int, default=10000, help="slices of the saturating run")
    ap.add_argument("--serve-inflight", type=int, default=32)
    ap.add_argument("--serve-pollers", type=int, default=4, help="threads delivering finished tickets")
    ap.add_argument("--serve-paced-slices", type=int, default=800, help="slices of the real-time run")
    return ap.parse_args()


def _dev_slice(torch, dev, s):
    return (torch.from_numpy(s.pmt.view(np.int16)).to(dev), torch.from_numpy(s.t).to(dev),
            torch.from_numpy(s.q.view(np.int16)).to(dev))


def _pct(x, p):
    return round(float(np.percentile(np.asarray(x), p)), 4) if len(x) else None


def bench_tagging(T, torch, tr, gid, pmt, t, q, params, n, steps, warmup, stream):
    """The same slice with the tagged-hit list asked for (hits inside the event
    windows, extracted to the host): step time and the tagging kernels."""
    run = T.SliceRunner(tr.ctx, gid, pmt, t, q, params, stream=stream, tagged=True)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    tagged = r["tagged"].copy()
    T.trig_profile_enable(tr.ctx, True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    prof = T.trig_profile_read(tr.ctx)
    T.trig_profile_enable(tr.ctx, False)
    kernels = {}
    for p in prof:
        if not p["name"].startswith("k_tag"):
            continue
        avg_us = p["total_ms"] / max(1, p["launches"]) * 1e3
        e = dict(avg_us=round(avg_us, 3), launches=int(p["launches"]))
        if p["name"] in ALGO_BYTES_PER_HIT:
            e["gbs"] = round(ALGO_BYTES_PER_HIT[p["name"]] * n / (avg_us * 1e-6) / 1e9, 1)
        kernels[p["name"]] = e
    return dict(value=round(n / el, 1), unit="hits/s", ms_per_step=round(el * 1e3, 4), n_tagged=int(r["n_tagged"]),
                kernels=kernels), tagged


# the paper's settings for the 84-PMT tower: level 0 N7TW500, then the candidate
# selection [SC and AFC] or [FC and AFC] (SC 20 ns, FC 100 ns, AFC 250 ns)
LEVEL0 = dict(l0_n=7, l0_tw_ns=500)
SEED_MENU = dict(LEVEL0, t_adj_ns=20, t_floor_ns=100, t_afloor_ns=250, seed_mode=1)


def bench_variant(T, torch, tr, gid, pmt, t, q, prm, n, steps, warmup, stream, prefix, setting):
    """The same slice with one of the paper's rule variants on: step time and the
    kernels whose names start with prefix."""
    run = T.SliceRunner(tr.ctx, gid, pmt, t, q, prm, stream=stream)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    out = dict(fires=r["fires"].copy(), events=r["events"].copy())
    T.trig_profile_enable(tr.ctx, True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    prof = T.trig_profile_read(tr.ctx)
    T.trig_profile_enable(tr.ctx, False)
    kernels = {}
    for p in prof:
        if p["name"].startswith(prefix):
            kernels[p["name"]] = dict(avg_us=round(p["total_ms"] / max(1, p["launches"]) * 1e3, 3),
                                      launches=int(p["launches"]))
    return dict(setting=setting, value=round(n / el, 1), unit="hits/s", ms_per_step=round(el * 1e3, 4),
                n_seeds=int(r["n_seeds"]), n_fires=int(r["n_fires"]), kernels=kernels), out


def bench_batch(T, torch, dev, a):
    """Batched form: many uneven slices of two tower types in one launch sequence,
    against the same slices triggered one call each."""
    from gen import configs as C
    g0 = time.perf_counter()
    w = C.batch(seed=2, n_slices=a.batch_slices)
    gen_s = time.perf_counter() - g0
    tr = T.Trigger(0)
    gids = {k: tr.load_geometry(g.floor_id, thr) for k, (g, thr) in w.geoms.items()}
    dsl = [(gids[k],) + _dev_slice(torch, dev, s) for k, s in w.slices]
    n = int(sum(s.n for _, s in w.slices))
    torch.cuda.synchronize()
    # ordering-stage launch parameters from the autotuner, tuned on this batch
    # (one class for both tower types)
    from paper_1411_3968_amd import autotune
    tuned = autotune.tune_class(tr.ctx, 84, dsl, w.params, reps=5, time_budget_s=30.0)
    first = tr.batch(dsl, w.params)
    assert all(r["status"] == 0 for r in first)
    caps = [(max(1, r["n_fires"]), max(1, r["n_events"])) for r in first]
    run = T.BatchRunner(tr.ctx, dsl, w.params, caps=caps)
    for _ in range(2):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.batch_steps):
        res = run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / a.batch_steps
    # the same slices, one plain per-slice call each
    runners = [T.SliceRunner(tr.ctx, *d, w.params, fire_cap=c[0], event_cap=c[1]) for d, c in zip(dsl, caps)]
    for r in runners:
        r()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = True
    for r, b in zip(runners, res):
        x = r()
        same &= x["n_fires"] == b["n_fires"] and np.array_equal(x["fires"], b["fires"]) \
            and np.array_equal(x["events"], b["events"])
    torch.cuda.synchronize()
    el_loop = time.perf_counter() - t0
    assert same, "batched and per-slice results differ"
    T.trig_profile_enable(tr.ctx, True)
    run()
    torch.cuda.synchronize()
    prof = T.trig_profile_read(tr.ctx)
    T.trig_profile_enable(tr.ctx, False)
    # per kernel over the whole pass: a kernel that also reruns single slices
    # (general ordering, dense windows) has more launches than one per pass, so
    # its algorithmic rate is taken over its total time
    kernels = {}
    for p in prof:
        tot_us = p["total_ms"] * 1e3
        e = dict(total_us=round(tot_us, 2), launches=int(p["launches"]))
        if p["name"] in ALGO_BYTES_PER_HIT:
            e["gbs"] = round(ALGO_BYTES_PER_HIT[p["name"]] * n / (tot_us * 1e-6) / 1e9, 1)
        kernels[p["name"]] = e
    tr.close()
    return dict(workload="batch-256-mixed-32/84pmt-50-200ms", slices=len(dsl), hits=n,
                value=round(n / el, 1), unit="hits/s", ms_per_batch=round(el * 1e3, 3),
                per_slice_loop=dict(value=round(n / el_loop, 1), ms=round(el_loop * 1e3, 3)),
                speedup_vs_per_slice=round(el_loop / el, 3), results_equal_per_slice=bool(same),
                fires=int(sum(r["n_fires"] for r in res)), kernels=kernels, gen_seconds=round(gen_s, 1),
                autotune=dict({k: tuned["best"][k] for k in ("seg_cap", "seg_target", "grid_per_cu")},
                              candidates=len(tuned["trials"]), seconds=round(tuned["seconds"], 1),
                              trials_ms=[[t["seg_cap"], t["seg_target"], t["grid_per_cu"], round(t["s"] * 1e3, 3)]
                                         for t in tuned["trials"]]))


def bench_serving(T, torch, dev, a):
    """Serving form: slices submitted to the stream loop as they arrive (device
    resident), results polled; every result is checked against the same slice
    triggered alone."""
    from gen import configs as C
    w = C.serving_pool(seed=4, n_pool=a.serve_pool)
    g, thr = w.geoms["km3"]
    tr = T.Trigger(0, hbm_budget_bytes=32 << 30)
    gid = tr.load_geometry(g.floor_id, thr)
    pool = [_dev_slice(torch, dev, s) for _, s in w.slices]
    ns = [int(s.n) for _, s in w.slices]
    alone = [tr.slice(gid, *d, w.params) for d in pool]
    torch.cuda.synchronize()
    cap = max(max(r["n_fires"] for r in alone), max(r["n_events"] for r in alone), 1)
    bufs = [T.ResultBuffers(cap, cap, 0, False) for _ in range(max(a.serve_inflight, 64))]

    def ref_bytes(ref):
        """The reference lists as bytes (every field and the zeroed padding of a
        record), whole up to 2^16 records, else every 61st record plus both ends."""
        out = []
        for key in ("fires", "events"):
            b2 = ref[key]
            if len(b2) <= 1 << 16:
                out.append((True, b2.tobytes()))
            else:
                out.append((False, (b2[::61].tobytes(), b2[:256].tobytes(), b2[-256:].tobytes())))
        return out

    alone_b = [ref_bytes(r) for r in alone]

    def same_as_alone(r, k):
        """Counts always; the lists byte for byte against the slice triggered alone,
        whole up to 2^16 records, else every 61st record plus both ends (a burst
        slice's 2M fires would otherwise cost the single submitting thread more
        than the GPU spends on a dozen slices)."""
        ref = alone[k]
        if (r["n_fires"], r["n_events"], r["n_seeds"]) != (ref["n_fires"], ref["n_events"], ref["n_seeds"]):
            return False
        for key, (whole, rb) in zip(("fires", "events"), alone_b[k]):
            a = r[key]
            if whole:
                if a.tobytes() != rb:
                    return False
            elif (a[::61].tobytes(), a[:256].tobytes(), a[-256:].tobytes()) != rb:
                return False
        return True

    submit = T.StreamSubmitter(tr.ctx, [(gid,) + d for d in pool], w.params)

    # finished tickets are delivered (polled into their buffers and checked) by a
    # few threads: the copy of a result's lists runs with Python's lock released,
    # so one thread's copies no longer cap the rate
    from concurrent.futures import ThreadPoolExecutor
    pollers = ThreadPoolExecutor(max_workers=max(1, a.serve_pollers))

    def deliver(tk, arr, k, bi, t_start):
        rc, r = T.trig_stream_poll(tr.ctx, tk, timeout_us=0, buffers=bufs[bi], copy=False)
        lat = time.perf_counter() - t_start - arr
        return lat, rc == T.TRIG_OK and same_as_alone(r, k), bi

    def run(order, arrivals, inflight_max):
        """Submit pool[order[i]] at arrivals[i] (None: as soon as fewer than
        inflight_max are outstanding); returns (latencies s, wall s, mismatches)."""
        lat, bad = [], 0
        pending = {}          # ticket -> (arrival, pool index, buffer): submitted, not finished
        delivering = []       # deliveries in progress (still counted as outstanding)
        free = list(range(len(bufs)))
        i, n_tot = 0, len(order)
        t_start = time.perf_counter()

        def collect(wait):
            nonlocal bad
            still = []
            for f in delivering:
                if wait or f.done():
                    l, ok, bi = f.result()
                    lat.append(l)
                    bad += 0 if ok else 1
                    free.append(bi)
                else:
                    still.append(f)
            delivering[:] = still

        while i < n_tot or pending or delivering:
            collect(False)
            now = time.perf_counter() - t_start
            while i < n_tot and len(pending) + len(delivering) < inflight_max and \
                    (arrivals is None or arrivals[i] <= now):
                k = order[i]
                rc, tk = submit(k, i)
                if rc == T.TRIG_EAGAIN:
                    break
                if rc != T.TRIG_OK:
                    raise T.TrigError(rc, T.trig_last_error(tr.ctx))
                pending[tk] = (now if arrivals is None else float(arrivals[i]), k, free.pop())
                i += 1
            # wait for whichever ticket finishes first (until the next arrival is due)
            wait_us = -1 if (arrivals is None or i >= n_tot) else \
                max(0, int((arrivals[i] - (time.perf_counter() - t_start)) * 1e6))
            if not pending:
                if delivering and (wait_us < 0 or len(delivering) >= inflight_max):
                    collect(True)
                else:
                    time.sleep(max(0.0, wait_us * 1e-6) if wait_us >= 0 else 0.0005)
                continue
            rc, tk = T.trig_stream_next_done(tr.ctx, wait_us)
            if rc != T.TRIG_OK:
                continue
            arr, k, bi = pending.pop(tk)
            delivering.append(pollers.submit(deliver, tk, arr, k, bi, t_start))
        collect(True)
        return lat, time.perf_counter() - t_start, bad

    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([4, 99])))
    # saturating: arrivals as fast as admission and the in-flight cap allow
    order = rng.integers(0, len(pool), a.serve_slices)
    run(order[:min(64, len(order))], None, a.serve_inflight)          # warm-up
    lat, wall, bad = run(order, None, a.serve_inflight)
    hits = int(sum(ns[k] for k in order))
    sat = dict(slices=int(len(order)), hits=hits, value=round(hits / wall, 1), unit="hits/s",
               latency_ms=dict(p50=_pct(np.array(lat) * 1e3, 50), p99=_pct(np.array(lat) * 1e3, 99)),
               inflight=a.serve_inflight, pollers=a.serve_pollers, mismatches=bad)
    # paced: 16 towers, slice k of a tower arrives at k * 200 ms + Exp(10 ms)
    m = a.serve_paced_slices
    k_of = np.arange(m) // 16
    arr = k_of * 0.2 + rng.exponential(0.010, m)
    ordp = np.argsort(arr, kind="stable")
    arr = arr[ordp]
    porder = rng.integers(0, len(pool), m)
    lat_p, wall_p, bad_p = run(porder, arr, 1 << 30)
    hits_p = int(sum(ns[k] for k in porder))
    paced = dict(slices=m, hits=hits_p, offered=round(hits_p / float(arr[-1] + 1e-9), 1),
                 sustained=round(hits_p / wall_p, 1), unit="hits/s",
                 latency_ms=dict(p50=_pct(np.array(lat_p) * 1e3, 50), p99=_pct(np.array(lat_p) * 1e3, 99),
                                 max=_pct(np.array(lat_p) * 1e3, 100)),
                 mismatches=bad_p)
    pollers.shutdown(wait=True)
    stats = T.trig_stream_stats_get(tr.ctx)
    tr.close()
    assert bad == 0 and bad_p == 0, "serving results differ from the slices triggered alone"
    return dict(workload="serving-16x84pmt-200ms-50-150kHz", pool=len(pool), saturating=sat, paced=paced,
                rounds=stats.get("rounds"), device_bytes_peak=stats.get("device_bytes_peak"))


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py drives a single MI355X: multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)
    import torch

    from gen import configs as C
    from paper_1411_3968_amd import trig as T

    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    w = C.km3(seed=1)
    g, thr = w.geoms["km3"]
    s = w.slices[0][1]
    n = s.n
    pmt = torch.from_numpy(s.pmt.view(np.int16)).to(dev)
    t = torch.from_numpy(s.t).to(dev)
    q = torch.from_numpy(s.q.view(np.int16)).to(dev)
    torch.cuda.synchronize()
    tr = T.Trigger(0)
    gid = tr.load_geometry(g.floor_id, thr)
    stream = torch.cuda.current_stream()
    first = tr.slice(gid, pmt, t, q, w.params, stream=stream)
    assert first["status"] == 0
    run = T.SliceRunner(tr.ctx, gid, pmt, t, q, w.params, stream=stream)
    for _ in range(a.warmup):
        run()
    # timed region: the production path (launch sequence replayed as a HIP graph)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        r = run()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert r["n_fires"] == first["n_fires"] and np.array_equal(r["fires"], first["fires"])
    # per-kernel durations: the same launch sequence, launched kernel by kernel with
    # HIP events between the kernels on the launching stream (event nodes inside a
    # replayed graph do not order with its kernels), right after the timed region
    T.trig_profile_enable(tr.ctx, True)
    for _ in range(a.steps):
        run()
    torch.cuda.synchronize()
    prof = T.trig_profile_read(tr.ctx)
    T.trig_profile_enable(tr.ctx, False)
    if a.calib_copy_mib:
        x = torch.empty(a.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    kern = {p["name"]: p for p in prof}
    per_kernel = {}
    for name, p in kern.items():
        avg_ms = p["total_ms"] / max(1, p["launches"])
        entry = dict(avg_us=round(avg_ms * 1e3, 3), launches=p["launches"])
        if name in ALGO_BYTES_PER_HIT:
            entry["gbs"] = round(ALGO_BYTES_PER_HIT[name] * n / (avg_ms * 1e-3) / 1e9, 1)
        per_kernel[name] = entry
    timed = {k: v for k, v in per_kernel.items() if k in ALGO_BYTES_PER_HIT}
    dom = max(timed, key=lambda k: timed[k]["avg_us"])
    dom_gbs = timed[dom]["gbs"]
    roofline = dict(bound="hbm", kernel=dom, achieved=dom_gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(dom_gbs / HBM_PEAK_GBS, 4), traffic=measured_traffic(dom),
                    bytes_per_hit=ALGO_BYTES_PER_HIT[dom], hits_per_launch=n)

    tagging, tagged = bench_tagging(T, torch, tr, gid, pmt, t, q, w.params, n, a.steps, a.warmup, stream)
    l0_prm = dict(w.params, **LEVEL0)
    level0, l0_out = bench_variant(T, torch, tr, gid, pmt, t, q, l0_prm, n, a.steps, a.warmup, stream, "k_l0",
                                   "N7TW500")
    from gen.geometry import bar_end_groups
    adj = bar_end_groups(g)
    gid_adj = tr.load_geometry(g.floor_id, thr, adj)
    menu_prm = dict(w.params, **SEED_MENU)
    seed_menu, menu_out = bench_variant(T, torch, tr, gid_adj, pmt, t, q, menu_prm, n, a.steps, a.warmup, stream,
                                        "k_tile", "N7TW500 then [SC and AFC] or [FC and AFC]")

    cpu = None
    if not a.no_cpu:
        from oracle import cpu as orc
        threads = os.cpu_count() or 1
        reps, tc = 0, 0.0
        ref = None
        while tc < a.cpu_seconds or reps == 0:
            c0 = time.perf_counter()
            ref = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, w.params, "blocked", threads=threads)
            tc += time.perf_counter() - c0
            reps += 1
        assert np.array_equal(ref["fires"], r["fires"]) and np.array_equal(ref["events"], r["events"])
        tagging["equals_oracle"] = bool(np.array_equal(orc.tag(s.pmt, s.t, ref["fires"], w.params["half_event_ns"]),
                                                       tagged))
        ref0 = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, l0_prm, "blocked", threads=threads)
        level0["equals_oracle"] = bool(np.array_equal(ref0["fires"], l0_out["fires"]) and
                                       np.array_equal(ref0["events"], l0_out["events"]))
        refm = orc.run(s.pmt, s.t, s.q, g.floor_id, thr, menu_prm, "blocked", threads=threads, adj_id=adj)
        seed_menu["equals_oracle"] = bool(np.array_equal(refm["fires"], menu_out["fires"]) and
                                          np.array_equal(refm["events"], menu_out["events"]))
        cpu = dict(value=round(n * reps / tc, 1), unit="hits/s", cores=threads, kind="oracle",
                   sample=f"blocked form, whole {n}-hit slice x {reps} runs ({tc:.1f} s)")

    tr.close()
    batch = None if a.no_batch else bench_batch(T, torch, dev, a)
    serving = None if a.no_serve else bench_serving(T, torch, dev, a)

    lat_ms = np.array(lat) * 1e3
    out = dict(
        metric="hits/s triggered on 1 MI355X",
        value=round(n * a.steps / el, 1),
        unit="hits/s",
        n_gpus=1,
        steps=a.steps,
        warmup=a.warmup,
        ms_per_step=round(el / a.steps * 1e3, 4),
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="u32",
        data="synthetic",
        config=dict(workload="km3net-it-84pmt-200ms", n_pmt=84, hits=n, slice_ms=200, rate_khz=55,
                    tracks=20, inputs="device-resident", params=w.params),
        latency_ms=dict(p50=round(float(np.percentile(lat_ms, 50)), 4),
                        p99=round(float(np.percentile(lat_ms, 99)), 4)),
        roofline=roofline,
        kernels=per_kernel,
        cpu_baseline=cpu,
        results=dict(n_seeds=r["n_seeds"], n_fires=r["n_fires"], n_events=r["n_events"], path=r["path"]),
        tagging=tagging,
        level0=level0,
        seed_menu=seed_menu,
        batched=batch,
        serving=serving,
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()
