"""bench.py's contract on the CPU: more than one GPU is refused with a
message before any GPU is touched; the counter traffic is read only while
the kernel sources match the ones it was taken on; the oracle baseline
reports the fields the bench line carries."""
import hashlib
import os
import subprocess
import sys

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_read_only_for_the_recorded_sources(tmp_path):
    digest = hashlib.sha256(b"".join(open(p, "rb").read() for p in bench.KERNEL_SOURCES)).hexdigest()
    good = tmp_path / "good.md"
    good.write_text(f"traffic_bytes_per_launch: 123456\nkernel sources sha256 {digest}\n")
    stale = tmp_path / "stale.md"
    stale.write_text(f"traffic_bytes_per_launch: 123456\nkernel sources sha256 {'0' * 64}\n")
    assert bench.measured_traffic(str(good)) == 123456.0
    assert bench.measured_traffic(str(good), xcd=True) is None  # no figure for the XCD numbering
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None
    both = tmp_path / "both.md"
    both.write_text(f"traffic_bytes_per_launch: 123456\ntraffic_bytes_per_launch_xcd: 120000\n"
                    f"kernel sources sha256 {digest}\n")
    assert bench.measured_traffic(str(both)) == 123456.0
    assert bench.measured_traffic(str(both), xcd=True) == 120000.0
    assert bench.measured_traffic(str(both), lanes16=True) is None


def test_oracle_baseline_fields():
    csc, b = W.tiny_tridiagonal()
    out = bench.cpu_baseline(csc, b, 3)
    assert out["kind"] == "oracle" and out["cores"] == 1
    assert out["unit"] == "amplitude updates/s"
    assert out["value"] > 0 and "3 walk steps" in out["sample"]
