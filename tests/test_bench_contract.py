"""Host-side checks of bench.py's command line (no GPU needed): more than
one GPU is refused with a message before anything touches a device, the
learned-chemistry leg can be skipped, and the kernel-source hash
that ties the committed counter summaries to the kernel ignores comments."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "single" in r.stderr and "GPU" in r.stderr


def test_surrogate_leg_can_be_skipped():
    # the learned-chemistry comparison runs by default; the flag that skips
    # it parses (the GPU-count check then refuses the run before any device
    # work)
    r = run("--no-surrogate", "--gpus", "2")
    assert r.returncode == 2
    assert "single" in r.stderr


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    h0 = bench.kernel_hash()
    src = tmp_path / "k.hip"
    src.write_text("int a; // one\n/* two */ int b;\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", [str(src)])
    h1 = bench.kernel_hash()
    src.write_text("int a; // changed\n/* also changed */ int b;\n")
    assert bench.kernel_hash() == h1
    src.write_text("int a; int c;\n")
    assert bench.kernel_hash() != h1
    assert isinstance(h0, str) and len(h0) == 16


def test_committed_traffic_summaries_name_their_kernel_hash():
    for name in ("m1_step_cosmo1024_traffic.json", "m1_step_hll_cosmo1024_traffic.json"):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            d = json.load(fh)
        assert len(d["kernel_sha"]) == 16
        assert d["bytes_per_launch"] == pytest.approx(d["fetch_bytes"] + d["write_bytes"])
