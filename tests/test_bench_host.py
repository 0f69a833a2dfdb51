"""CPU checks of bench.py's host logic: counter summaries are used only for
the sources and the workload seed they were taken on."""
import json

import bench


def test_traffic_is_gated_by_source_hash_and_seed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    h = bench.kernel_source_hash()
    (tmp_path / "p.json").write_text(json.dumps({"kernel_hash": h, "seed": 0, "hbm_bytes_per_launch": 123}))
    assert bench.traffic_from_profile("p.json", h, 0) == 123
    assert bench.traffic_from_profile("p.json", h, 1) is None
    assert bench.traffic_from_profile("p.json", "0" * 16, 0) is None
    assert bench.traffic_from_profile("missing.json", h, 0) is None
    # summaries without a seed count as seed 0
    (tmp_path / "q.json").write_text(json.dumps({"kernel_hash": h, "hbm_bytes_per_launch": 7}))
    assert bench.traffic_from_profile("q.json", h) == 7


def test_committed_headline_summary_matches_the_sources():
    """The committed counter summary of the headline workload was taken on
    the current kernels, layout and runtime (else bench reports no traffic)."""
    d = json.load(open(bench.PROFILE_DIR + "/sweep_f32_poiseuille256_pmc.json"))
    assert d["kernel_hash"] == bench.kernel_source_hash()
    assert 1.0 <= d["traffic_over_algorithmic"] < 1.1
