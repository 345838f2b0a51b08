"""Host-side checks of bench.py's bookkeeping (no GPU): the committed HBM-traffic
record is filed under the benchmarked workload's name, so the bench line can
find it, and it names the kernels the roofline uses."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2011_13517_amd import synth  # noqa: E402


def test_traffic_record_is_filed_under_the_headline_workload():
    name = synth.config(2).name
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{name}.json")
    assert os.path.exists(path), path
    with open(path) as f:
        rec = json.load(f)
    assert rec["workload"] == name
    for k in ("cheb_adjoint64_kernel", "cheb_forward_kernel"):
        assert k in rec["kernels"] and k in bench.KERNEL_SOURCES
        assert rec["kernels"][k]["fetch_bytes"] > 0 and rec["kernels"][k]["write_bytes"] > 0


def test_traffic_record_is_ignored_for_other_sources(tmp_path, monkeypatch):
    name = synth.config(2).name
    rec = {"workload": name, "kernels": {"cheb_forward_kernel": {
        "fetch_bytes": 1.0, "write_bytes": 2.0, "source_sha256": "0" * 64}}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / f"hbm_traffic_{name}.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel: "f" * 64)
    assert bench.recorded_traffic("cheb_forward_kernel", name) is None
    rec["kernels"]["cheb_forward_kernel"]["source_sha256"] = "f" * 64
    (tmp_path / "profiles" / f"hbm_traffic_{name}.json").write_text(json.dumps(rec))
    assert bench.recorded_traffic("cheb_forward_kernel", name)["bytes"] == 3.0
