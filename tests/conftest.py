import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import cpu
    cpu.build(force=False)
    return cpu


def load_hand_cases():
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        doc = json.load(f)
    out = []
    for c in doc["cases"]:
        params = dict(doc["params"])
        params.update(c.get("params", {}))
        thr = np.asarray(c.get("thr", doc["thr"]), dtype=np.uint32)
        floor_id = np.asarray(c.get("floor_id", doc["floor_id"]), dtype=np.int32)
        hits = c["hits"]
        pmt = np.asarray([h[0] for h in hits], dtype=np.uint16)
        t = np.asarray([h[1] for h in hits], dtype=np.int64)
        q = np.asarray([h[2] for h in hits], dtype=np.uint16)
        out.append(dict(name=c["name"], cite=c["cite"], params=params, thr=thr, floor_id=floor_id,
                        pmt=pmt, t=t, q=q, status=c.get("status", 0), seed=c.get("seed"),
                        fold=c.get("fold"), fires=c.get("fires"), events=c.get("events")))
    return out


def fires_as_tuples(fires):
    """Structured fire array -> list of (t, hit_index, fold, pmt)."""
    return [(int(f["t_ns"]), int(f["hit_index"]), int(f["fold"]), int(f["pmt_id"])) for f in fires]


def events_as_tuples(events):
    return [(int(e["t_trig"]), int(e["t_begin"]), int(e["t_end"]), int(e["n_fire"]), int(e["max_fold"]))
            for e in events]
