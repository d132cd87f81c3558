"""Host logic of bench.py's roofline traffic: counter bytes stored with a
hash of the kernel source are used only while that source is unchanged."""
import json

import bench


def _store(tmp_path, monkeypatch, entries):
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(entries))
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(p))


def test_matching_hash_gives_the_stored_bytes(tmp_path, monkeypatch):
    _store(tmp_path, monkeypatch, {"wl": {"collide_stream": {
        "source_hash": bench._kernel_hash(), "bytes_per_launch": 123.0}}})
    assert bench._traffic("wl", "collide_stream") == 123.0


def test_changed_kernel_source_gives_none(tmp_path, monkeypatch):
    _store(tmp_path, monkeypatch, {"wl": {"collide_stream": {
        "source_hash": "0" * 16, "bytes_per_launch": 123.0}}})
    assert bench._traffic("wl", "collide_stream") is None


def test_missing_workload_kernel_or_file_gives_none(tmp_path, monkeypatch):
    _store(tmp_path, monkeypatch, {"wl": {}})
    assert bench._traffic("other", "collide_stream") is None
    assert bench._traffic("wl", "collide_stream") is None
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(tmp_path / "absent.json"))
    assert bench._traffic("wl", "collide_stream") is None


def test_committed_counters_cover_both_bench_workloads():
    """The stored counter runs name the 3D and the 2D workload's
    collide-stream, each with positive fetch and write bytes."""
    with open(bench.PROFILE_COUNTERS) as fh:
        d = json.load(fh)
    for wl in ("3d_d3q19_fp32_256x256x512", "2d_fp32_shifted_s_1024x2048"):
        e = d[wl]["collide_stream"]
        assert e["fetch_bytes"] > 0 and e["write_bytes"] > 0
        assert abs(e["bytes_per_launch"] - e["fetch_bytes"] - e["write_bytes"]) < 1.0
