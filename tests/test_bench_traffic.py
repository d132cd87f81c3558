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
    collide-stream and transport phases, each with positive fetch and write
    bytes."""
    with open(bench.PROFILE_COUNTERS) as fh:
        d = json.load(fh)
    for wl in ("3d_d3q19_fp32_256x256x512", "2d_fp32_shifted_s_1024x2048"):
        for phase in ("collide_stream", "transport"):
            e = d[wl][phase]
            assert e["fetch_bytes"] > 0 and e["write_bytes"] > 0
            assert abs(e["bytes_per_launch"] - e["fetch_bytes"] - e["write_bytes"]) < 1.0


def test_transport_hash_is_separate(tmp_path, monkeypatch):
    _store(tmp_path, monkeypatch, {"wl": {"transport": {
        "source_hash": bench._kernel_hash("transport"), "bytes_per_launch": 7.0},
        "collide_stream": {"source_hash": bench._kernel_hash("transport"), "bytes_per_launch": 1.0}}})
    assert bench._traffic("wl", "transport") == 7.0
    assert bench._traffic("wl", "collide_stream") is None


def test_algorithmic_bytes_of_the_workloads():
    from paper_2106_07694_amd import workloads as W
    ab = bench._alg_bytes(W.C3)
    assert (ab["step"], ab["collide_stream"], ab["transport"]) == (160, 156, 68)
    ab = bench._alg_bytes(W.C2)           # D2Q9 FP32 with S: 72 + 16; stages 2D
    assert (ab["step"], ab["collide_stream"], ab["transport"]) == (88, 80, 8 * 4 + 3 * 8 + 8)


def test_ingest_counters_scales_by_the_copy_kernel(tmp_path, monkeypatch):
    """Two counter CSVs in rocprofv3's layout: each kernel's mean counter per
    dispatch is scaled by the copy kernel's reading of its known 256 MiB."""
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(tmp_path / "t.json"))
    import csv
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float>>()"
    cs = "void lbw::(anonymous namespace)::k_collide_stream<19, float, true, false, true>(lbw::RunDev)"
    st = "void lbw::(anonymous namespace)::k_stage_tiled<float, 3, 0, {}, 64, 8, true, false, false>(x)"
    rows = {"FETCH_SIZE": [(copy, 131072), (cs, 1000), (cs, 3000)],
            "WRITE_SIZE": [(copy, 262144), (cs, 500), (cs, 500)]}
    for k in (1, 2, 3):
        rows["FETCH_SIZE"].append((st.format(k), 10))
        rows["WRITE_SIZE"].append((st.format(k), 20))
    for fname, counter in (("f.csv", "FETCH_SIZE"), ("w.csv", "WRITE_SIZE")):
        with open(tmp_path / fname, "w", newline="") as fh:
            w = csv.writer(fh)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for i, (name, val) in enumerate(rows[counter]):
                w.writerow([i, name, counter, val])
    e = bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "wl", cells=1024)
    name = "k_collide_stream<19, float, true, false, true>"
    k = e["kernels"][name]
    assert k["fetch_bytes"] == 2000 * 1024 * 2.0 and k["write_bytes"] == 500 * 1024
    assert k["launches"] == 2
    assert bench._traffic("wl", "collide_stream") == k["bytes_per_launch"]
    assert bench._traffic("wl", "transport") == 3 * (10 * 1024 * 2.0 + 20 * 1024)
