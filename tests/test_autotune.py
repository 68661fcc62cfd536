"""Autotuner candidates and cache format (no GPU needed)."""
import json
import os

from conftest import ROOT


def test_candidates_are_valid_tunings():
    from paper_1411_3968_amd import autotune
    src = open(os.path.join(ROOT, "paper_1411_3968_amd", "csrc", "api.hip")).read()
    assert "WAVE_CAP" in src
    seen = set()
    for cap, tgt, g in autotune.DEFAULT_CANDIDATES:
        assert cap in (autotune.WAVE_CAP, autotune.WAVE_CAP_SMALL, 2048, 4096, 8192)
        assert 0 < tgt <= cap and 1 <= g <= 16
        assert (cap, tgt, g) not in seen
        seen.add((cap, tgt, g))
    assert any(c[0] == autotune.WAVE_CAP for c in seen) and any(c[0] == autotune.WAVE_CAP_SMALL for c in seen)
    assert any(c[0] > autotune.WAVE_CAP for c in seen)


def test_count_candidates_are_valid_tunings():
    from paper_1411_3968_amd import autotune
    assert len(set(autotune.COUNT_CANDIDATES)) == len(autotune.COUNT_CANDIDATES)
    for g, h in autotune.COUNT_CANDIDATES:
        assert g in (1, 2, 4) and h in (512, 2048)


def test_cache_roundtrip_format(tmp_path):
    from paper_1411_3968_amd import autotune
    res = [dict(n_pmt_max=84, best=dict(seg_cap=512, seg_target=256, grid_per_cu=3, tile_group=2, window_cap=512,
                                        s=0.01), trials=[])]
    path = str(tmp_path / "tune.json")
    autotune.save(path, res, device="test")
    doc = json.load(open(path))
    assert doc["device"] == "test"
    assert doc["classes"] == [dict(n_pmt_max=84, seg_cap=512, seg_target=256, grid_per_cu=3, tile_group=2,
                                   window_cap=512)]
