"""Host logic of bench.py (no GPU): the roofline object names the Lanczos-form
H.v class with the most time, prices its algorithmic bytes per launch by the
live HIP-event durations, and takes `traffic` from the class's committed
counter summary only while that summary's kernel-source hash matches."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _stat(launches, ms, nbytes):
    return {"launches": launches, "sampled": launches, "sampled_ms": ms, "sampled_bytes": nbytes}


def _summary(path, sha, line):
    with open(path, "w") as f:
        f.write(f"kernel_source_sha1: {sha}  (source)\n\n{line}\n")


def test_roofline_takes_the_dominant_hv_class(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1109_1205_amd", "csrc", "hamiltonian.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    fused = tmp_path / "fused.md"
    _summary(fused, sha, "traffic_bytes_per_algorithmic_byte.hv_up_lanczos: 1.5\n"
                         "traffic_bytes_per_algorithmic_byte.hv_rows_lanczos: 1.25")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"hv_up_lanczos": str(fused), "hv_rows_lanczos": str(fused)})
    stats = {
        "combine": _stat(1, 400.0, 1e12),             # the most time overall, but not an H.v class
        "hv_rows_lanczos": _stat(20, 160.0, 20 * 2e10),
        "hv_up_lanczos": _stat(20, 200.0, 20 * 4e10),
    }
    roof, kernels = bench.roofline_of(stats)
    assert roof["kernel"] == "hv_up_lanczos" and roof["dominant_class"] == "combine"
    assert roof["avg_launch_algorithmic_bytes"] == 4e10
    assert abs(roof["avg_launch_ms"] - 10.0) < 1e-12
    assert abs(roof["achieved"] - 4000.0) < 1e-6                   # 4e10 B per 10 ms
    assert abs(roof["frac"] - 0.5) < 1e-12
    assert roof["traffic"] == round(1.5 * 4e10)
    assert set(kernels) == set(stats)


def test_traffic_is_null_for_another_source_or_no_summary(tmp_path, monkeypatch):
    stale = tmp_path / "stale.md"
    _summary(stale, "0" * 40, "traffic_bytes_per_algorithmic_byte: 3.0")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"hv_lanczos": str(stale)})
    assert bench.measured_traffic("hv_lanczos") is None
    assert bench.measured_traffic("hv_up_lanczos") is None          # no summary for the class
    roof, _ = bench.roofline_of({"hv_lanczos": _stat(4, 8.0, 4 * 1e9)})
    assert roof["kernel"] == "hv_lanczos" and roof["traffic"] is None


def test_committed_summaries_parse():
    for kernel in bench.TRAFFIC_FILES:
        assert os.path.exists(bench.TRAFFIC_FILES[kernel])
        r = bench.measured_traffic(kernel)
        assert r is None or 0.9 < r < 5.0, (kernel, r)
