"""Host logic of the benchmark script that needs no GPU: the one-GPU
contract (more GPUs exit with a message), and the traffic figure, which is
reported only while the kernel sources hash as in the committed profile."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 64
    prof = tmp_path / "p.md"
    prof.write_text(f"source_sha256: {h}\ntraffic_bytes_per_launch: 12345\n")
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.measured_traffic() == 12345.0
    prof.write_text("source_sha256: " + "0" * 64 + "\ntraffic_bytes_per_launch: 12345\n")
    assert bench.measured_traffic() is None
    # comments do not change the hash; code does
    assert bench._code_tokens("int a; // note\n/* x */ int b;") == bench._code_tokens("int a;\nint b;")
    assert bench._code_tokens("int a;") != bench._code_tokens("int b;")
