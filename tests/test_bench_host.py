"""bench.py's host-side parts, on the CPU: the one-GPU rule and the oracle
baseline leg (timed on a bounded window of the ring workload)."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.lstrip().startswith("{")


def test_cpu_baseline_reports_the_oracle_on_a_window():
    import bench
    import fvinputs as F
    case = F.make_case(2, n=1024)
    out = bench.cpu_baseline(case, seconds=0.2)
    assert out["kind"] == "oracle" and out["cores"] == 1
    assert out["unit"] == "cell-updates/s" and out["value"] > 0
    assert "96x96 window" in out["sample"]
    host = out["host"]
    assert host["logical_cpus"] == os.cpu_count()
    assert host["model"] is None or isinstance(host["model"], str)


def test_kernel_source_hash_is_stable():
    import bench
    assert bench.kernel_source_hash() == bench.kernel_source_hash()
    assert len(bench.kernel_source_hash()) == 16
