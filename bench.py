"""Benchmark of the trigger hot path on one MI355X.

One step = one pass of the whole path (ingest, time-order merge, L1 seeds,
causal N-fold count, fire compaction, event windows, results to host) over one
synthetic 200 ms slice of a KM3Net-It-like tower (84 PMTs on 14 floors x 6,
55 kHz per PMT, about 924k hits, 20 injected muon tracks), inputs resident in
HBM before the timed region.  Prints one JSON line.

``--gpus N`` with N > 1 exits: this build drives one GPU.
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
    "k_ingest": 10.0,      # read t (8) + pmt (2)
    "k_bounds": 8.0,       # read t (8); the boundary table is counted separately
    "k_segsort": 24.0,     # read t, pmt, q (12) + write ordered t, pmt|q, index (12)
    "k_seed": 8.125,       # read ordered t + pmt|q (8) + write one seed bit
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB once (counter calibration)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py drives a single MI355X: multi-GPU runs are not part of this build", file=sys.stderr)
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
    # per-kernel durations: the same steps launched eagerly with HIP events around
    # every kernel on the launching stream
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
                    frac=round(dom_gbs / HBM_PEAK_GBS, 4), traffic=None,
                    bytes_per_hit=ALGO_BYTES_PER_HIT[dom], hits_per_launch=n)

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
        cpu = dict(value=round(n * reps / tc, 1), unit="hits/s", cores=threads, kind="oracle",
                   sample=f"blocked form, whole {n}-hit slice x {reps} runs ({tc:.1f} s)")

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
    )
    tr.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
