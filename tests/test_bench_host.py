"""Host-side contract of bench.py and of the binding (no GPU needed).

* ``bench.py --gpus N`` with N > 1 exits with a message and status 2: the
  measured path is one GPU.
* The roofline's HBM traffic is reported only from a counter record of the
  same kernel sources and of launches of the same algorithmic size.
* The binding fails loudly when the library is missing: there is no
  fallback path.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_needs_matching_sources_and_size(tmp_path, monkeypatch):
    alg = 5.0e9
    rec = {"source_sha256": bench.kernel_source_hash(), "algorithmic_bytes_per_launch": alg,
           "bytes_per_launch": 5.1e9}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.recorded_traffic(alg) == 5.1e9
    # launches of another size: no figure
    assert bench.recorded_traffic(alg * 1.01) is None
    # kernel sources changed since the counters were taken: no figure
    rec["source_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.recorded_traffic(alg) is None
    # no record at all
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.recorded_traffic(alg) is None


def test_committed_traffic_record_is_consistent():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    if rec["source_sha256"] != bench.kernel_source_hash():
        pytest.skip("product kernel sources changed since the counters were taken "
                    "(bench.py then reports no traffic)")
    # the stem is read once and written once: counted bytes at or a little
    # above the algorithmic ones, both scaled by the copy calibration
    assert 1.0 <= rec["bytes_per_launch"] / rec["algorithmic_bytes_per_launch"] < 1.2
    cal = rec["copy_calibration"]
    assert cal["fetch_factor"] * cal["fetch_kib"] == pytest.approx(cal["bytes_copied"] / 1024,
                                                                   rel=1e-3)
    assert cal["write_factor"] * cal["write_kib"] == pytest.approx(cal["bytes_copied"] / 1024,
                                                                   rel=1e-3)
    per = (cal["fetch_factor"] * rec["fetch_kib_sum"] + cal["write_factor"] * rec["write_kib_sum"]) \
        * 1024 / rec["launches"]
    assert per == pytest.approx(rec["bytes_per_launch"], rel=1e-6)


def test_binding_without_the_library_raises(monkeypatch, tmp_path):
    from paper_2005_06787_amd import _capi as C

    monkeypatch.setattr(C, "LIB_PATH", str(tmp_path / "libstemgpu.so"))
    monkeypatch.setattr(C, "_lib", None)
    with pytest.raises(ImportError, match="no fallback"):
        C.lib()
