"""Host-side checks of the benchmark script: it refuses more than one GPU
before touching a device, and it attaches the committed counter profile only
to the kernel source the profile was taken on (comments aside)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_source_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    k0, k1 = tmp_path / "k0.hip", tmp_path / "k1.hip"
    k0.write_text("int f(int x) {\n  return x + 1;  // one more\n}\n")
    k1.write_text("/* block\n comment */ float g;\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(k0), str(k1)])
    h0 = bench.kernel_source_hash()
    k0.write_text("// header\nint f(int x) {\n    return x + 1;\n}\n")
    k1.write_text("float g;  /* other */\n")
    assert bench.kernel_source_hash() == h0
    k0.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_hash() != h0


def test_counters_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int f() { return 1; }\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    prof = tmp_path / "prof.md"
    prof.write_text("# summary\n\ntraffic_bytes_per_launch: 1234\nvalu_issue_utilisation: 0.5\n"
                    f"active_lane_fraction: 0.25\nkernel_source_sha256: {bench.kernel_source_hash()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.committed_counters() == {"traffic_bytes_per_launch": 1234.0,
                                          "valu_issue_utilisation": 0.5, "active_lane_fraction": 0.25}
    assert bench.committed_traffic() == 1234.0
    src.write_text("int f() { return 2; }\n")
    assert bench.committed_counters() == {}
    assert bench.committed_traffic() is None
