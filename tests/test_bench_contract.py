"""bench.py's host-side contract (no GPU): the one-GPU guard, the committed counter figures it
reports and how it turns them into the counter view of a roofline."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_follows_the_kernel_source_and_workload(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        table = json.load(f)
    assert table and set(table) <= {"lj", "scale"}, "no committed counter figures"
    for workload, kinds in table.items():
        other = "scale" if workload == "lj" else "lj"
        for kernel, entry in kinds.items():
            monkeypatch.setattr(bench, "kernel_source_hash",
                                lambda h=entry["kernel_source_sha256_16"]: h)
            got = bench.committed_traffic(kernel, workload)
            assert got == entry["bytes_per_launch"] and got > 0
            # one workload's counters are never reported for the other's launches
            if kernel not in table.get(other, {}):
                assert bench.committed_traffic(kernel, other) is None
            # figures taken on another kernel source are not reported
            monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
            assert bench.committed_traffic(kernel, workload) is None
    assert bench.committed_traffic("no_such_kernel", "lj") is None


def test_committed_profiles_describe_one_kernel_source():
    """The kernel-time summaries, the memory-counter summary and traffic.json were taken on the
    same kernel source."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        hashes = {e["kernel_source_sha256_16"] for kinds in json.load(f).values()
                  for e in kinds.values()}
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.endswith(".md"):
            with open(os.path.join(ROOT, "profiles", name)) as f:
                hashes |= set(re.findall(r"sha256\[:16\] = `([0-9a-f]{16})`", f.read()))
    assert len(hashes) == 1, hashes


def test_counter_view_of_a_roofline():
    rl = {"bound": "hbm", "peak": 8000.0, "avg_launch_us": 250.0,
          "algorithmic_bytes_per_launch": 1.0e9, "traffic": 1.5e9}
    out = bench.with_counters(dict(rl))
    assert out["counter_achieved"] == pytest.approx(1.5e9 / 250e-6 / 1e9)
    assert out["counter_frac"] == pytest.approx(out["counter_achieved"] / 8000.0)
    assert out["traffic_over_algorithmic"] == pytest.approx(1.5)
    # no counter figures: the roofline is left as it is
    assert "counter_frac" not in bench.with_counters({"traffic": None, "peak": 1.0})
    assert bench.with_counters(None) is None
