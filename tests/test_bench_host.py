"""bench.py's host-side parts, on the CPU: the one-GPU rule, the oracle
baseline leg (timed on a bounded window of the workload) and the check that
ties committed counter summaries to the kernel source they were taken on."""
import os
import shutil
import subprocess
import sys

import numpy as np
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


@pytest.mark.parametrize("which", ["ring", "impact3d"])
def test_cpu_baseline_reports_the_oracle_on_a_window(which):
    import bench
    n = 1024 if which == "ring" else 48
    cases, _, window = bench.make_workload(which, n)
    out = bench.cpu_baseline(cases[0], window[0], window[1], seconds=0.2)
    assert out["kind"] == "oracle" and out["cores"] == 1
    assert out["unit"] == "cell-updates/s" and out["value"] > 0
    w = window[1]
    shape = "x".join([str(w)] * cases[0].dim)
    assert out["sample"].startswith(f"{shape} window")
    host = out["host"]
    assert host["logical_cpus"] == os.cpu_count()
    assert host["model"] is None or isinstance(host["model"], str)


def test_window_is_the_workload_restricted():
    """The baseline window holds the workload's own fields and phi0."""
    import bench
    cases, _, window = bench.make_workload("impact3d", 48)
    c = cases[0]
    sub = bench._window(c, window[0], window[1])
    (x0, y0, z0), w = window
    assert np.array_equal(sub.prim, c.prim[:, z0:z0 + w, y0:y0 + w, x0:x0 + w])
    assert np.array_equal(sub.phi0, c.phi0[z0:z0 + w, y0:y0 + w, x0:x0 + w])
    assert sub.lo[0] == pytest.approx(c.lo[0] + x0 * c.dx[0])
    assert sub.dx == pytest.approx(c.dx)


def test_counter_summary_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    """A summary whose hash is not that of the current sources is ignored
    (its traffic figure reads as None), and editing any source changes the
    hash."""
    import bench
    srcs = []
    for p in bench.KERNEL_SOURCES:
        if os.path.exists(p):
            q = tmp_path / os.path.basename(p)
            shutil.copy(p, q)
            srcs.append(str(q))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", srcs)
    h0 = bench.kernel_source_hash()
    summary = tmp_path / "summary.txt"
    summary.write_text(f"kernel_source_hash: {h0}\nbytes_per_launch_fp32: 123.0\n")
    monkeypatch.setitem(bench.TRAFFIC_FILES, "ring", str(summary))
    assert bench.profile_value("ring", "bytes_per_launch_fp32") == 123.0
    for q in srcs:
        orig = open(q).read()
        with open(q, "a") as f:
            f.write("\n// edit\n")
        assert bench.kernel_source_hash() != h0, q
        assert bench.profile_value("ring", "bytes_per_launch_fp32") is None
        with open(q, "w") as f:
            f.write(orig)
    assert bench.kernel_source_hash() == h0
