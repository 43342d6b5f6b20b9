"""bench.py's host-side contract (CPU): one GPU only, the counter-summary
parser, the digest guard that turns traffic to null after a kernel change,
and the algorithmic work counts it reports."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2 and "one GPU" in out.stderr


def test_traffic_summary_parsing_and_digest_guard(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_x.txt").write_text(
        "# comment\nkernel: factor_redo\nworkload: wl\nsource_digest: abc\n"
        "fetch_bytes_per_launch: 100\nwrite_bytes_per_launch: 20\ncopy_scale_fetch: 2.0\ncopy_scale_write: 1.0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tr = bench.read_traffic("factor_redo", "wl", "abc")
    assert tr["fetch_bytes"] == 100 and tr["write_bytes"] == 20 and tr["copy_scale_fetch"] == 2.0
    assert bench.read_traffic("factor_redo", "wl", "other") is None        # kernel changed since the counters
    assert bench.read_traffic("factor_sparse", "wl", "abc") is None


def test_committed_traffic_summaries_parse():
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt")):
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("#", " ")):
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip()
        if "kernel" in kv:
            assert float(kv["fetch_bytes_per_launch"]) > 0 and float(kv["write_bytes_per_launch"]) > 0
            assert len(kv["source_digest"]) == 16


@pytest.mark.parametrize("k,kind,refine,expected", [(32, 2, True, 29674.666666666664), (32, 2, False, 19706.666666666664)])
def test_flop_counts(k, kind, refine, expected):
    assert bench.factor_flops_per_point(k, kind, refine) == pytest.approx(expected)


def test_byte_counts():
    assert bench.apply_bytes_per_point(32, 4) == 396
    assert bench.factor_bytes_per_point(32, 4) == 656
