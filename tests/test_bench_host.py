"""Host-side logic of bench.py (CPU only): the one-GPU refusal, the roofline
object, the per-pass table and the source-hash gate on recorded traffic."""
import json

import bench
from paper_1810_12707_amd.profile_summary import source_sha256


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_world_size_above_one_is_refused(monkeypatch, capsys):
    monkeypatch.setenv("WORLD_SIZE", "4")
    assert bench.main([]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_roofline_object():
    prof = {"xb": {"ms": 2.0, "launches": 4, "bytes": 4 * 1.0e9}}
    r = bench.roofline_from(prof, "xb", {"xb": 1.05e9, "zrhs": 7.0})
    # 1e9 bytes per launch in 0.5 ms = 2000 GB/s of the 8000 GB/s peak
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == 2000.0 and r["peak"] == 8000.0 and r["frac"] == 0.25
    assert r["traffic"] == 1.05e9
    assert r["bytes_per_launch"] == 1.0e9 and r["ms_per_launch"] == 0.5
    assert bench.roofline_from(prof, "xb", None)["traffic"] is None
    assert bench.roofline_from(prof, "xb", {"xa": 1.0})["traffic"] is None


def test_pass_table_skips_idle_classes():
    prof = {k: {"ms": 0.0, "launches": 0, "bytes": 0.0} for k in bench.PASS_NAMES}
    prof["zrhs"] = {"ms": 1.0, "launches": 10, "bytes": 4.0e9}
    t = bench.pass_table(prof, steps=10)
    assert list(t) == ["zrhs"]
    assert t["zrhs"] == {"ms_per_step": 0.1, "GBps": 4000.0, "frac_hbm": 0.5}


def test_traffic_needs_the_current_source_hash(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic(64) is None  # nothing recorded
    rec = {"source_sha256": "0" * 64, "bytes_per_launch": {"xb": 1.0}}
    (tmp_path / "profiles" / "traffic_64.json").write_text(json.dumps(rec))
    assert bench.load_traffic(64) is None  # recorded for other sources
    rec["source_sha256"] = source_sha256()
    (tmp_path / "profiles" / "traffic_64.json").write_text(json.dumps(rec))
    assert bench.load_traffic(64) == {"xb": 1.0}
