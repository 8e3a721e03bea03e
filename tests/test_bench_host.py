"""Host logic of bench.py that needs no GPU: the recorded traffic figure is
used only for the kernel source it was measured on, the recorded campaign
summary parses, and more than one GPU is refused before anything starts."""
import os
import subprocess
import sys

import bench


def test_traffic_is_read_for_the_measured_source_only(tmp_path, monkeypatch):
    v = bench.measured_traffic("k_grad_forces<8,fp32,2>")
    assert v is not None and 3e8 < v < 2e9
    assert bench.measured_traffic("k_grad_forces<3,fp32,9>") is None
    # a different kernel source: the figure no longer applies
    src = tmp_path / "pairs.hip"
    src.write_text(open(os.path.join(bench.ROOT, bench.TRAFFIC_SOURCES[0])).read() + "\n// x\n")
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", (str(src),) + bench.TRAFFIC_SOURCES[1:])
    assert bench.measured_traffic("k_grad_forces<8,fp32,2>") is None


def test_traffic_file_missing_gives_none(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "none.md"))
    assert bench.measured_traffic("k_grad_forces<8,fp32,2>") is None


def test_recorded_campaign_summary():
    c = bench.recorded_campaign()
    assert c is not None and c["source"].startswith("profiles")
    assert c["compared"] == c["held_out_cases"] == len(c["cases"])
    assert c["sims_net"] < c["sims_bisect"]
    assert c["sims_per_case_bisect"] == c["sims_bisect"] / c["compared"]
    for r in c["cases"]:
        assert abs(r["q_rd_net"] / r["q_rd_bisect"] - 1.0) <= c["q_rd_max_rel_diff"] + 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
