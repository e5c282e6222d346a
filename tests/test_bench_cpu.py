"""Host logic of bench.py, on the CPU: the one-GPU guard, the timing
statistics, the algorithmic bytes behind the roofline figure, and the source
hash that ties a committed HBM-traffic summary to the kernel code it was
measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_stats_us():
    t = [float(v) for v in range(1, 102)]  # 1 .. 101
    st = bench.stats_us(list(reversed(t)))
    assert st["median"] == 51.0 and st["p10"] == 11.0 and st["p90"] == 91.0
    assert st["mean"] == 51.0 and st["n"] == 101
    assert bench.stats_us([7.0]) == {"median": 7.0, "p10": 7.0, "p90": 7.0, "mean": 7.0, "n": 1}


def test_algorithmic_bytes_of_the_headline():
    # 8 B read + 8 B written per complex point (two FP32 planes each way)
    assert 16 * bench.N * bench.BATCH == 268435456
    assert bench.N == 1024 and bench.BATCH == 16384


def test_code_hash_ignores_comments_and_blank_lines_only():
    a = "int f(int x)\n{\n    return x + 1;  // one more\n}\n"
    b = "// f: the successor\nint f(int x)\n{\n\n    return x + 1;\n}   \n"
    c = "int f(int x)\n{\n    return x + 2;\n}\n"
    assert bench.code_hash([a]) == bench.code_hash([b])
    assert bench.code_hash([a]) != bench.code_hash([c])
    # the files are hashed in order, as separate texts
    assert bench.code_hash([a, c]) != bench.code_hash([c, a])


def test_traffic_summary_is_read_only_for_its_own_source(tmp_path, monkeypatch):
    summary = tmp_path / "summary.md"
    summary.write_text("    kernel_source_sha256: %s\n    traffic_bytes_per_launch: 268551197\n"
                       % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    assert bench.measured_traffic() == 268551197
    summary.write_text("    kernel_source_sha256: %s\n    traffic_bytes_per_launch: 268551197\n" % ("0" * 64))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None
