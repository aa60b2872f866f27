"""Host-side pieces of bench.py that need no GPU: the one-GPU refusal and
the rule that a committed rocprofv3 traffic figure is used only for the
kernel source and schedule it was taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_needs_the_same_source_and_schedule(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel text\n")
    import hashlib
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text("schedule: A+B\nsha `%s`\ntraffic_bytes_per_launch: 1.5e8\n" % h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k.hip", "k.md", "A+B") == 1.5e8
    assert bench.measured_traffic("k.hip", "k.md", "A+C") is None      # other schedule
    src.write_text("kernel text, edited\n")
    assert bench.measured_traffic("k.hip", "k.md", "A+B") is None      # other source
    assert bench.measured_traffic("k.hip", "missing.md", "A+B") is None

