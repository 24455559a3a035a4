"""Host logic of bench.py that needs no GPU: the counter-traffic summaries are
used only for the kernel source they were taken on, the one-GPU limit is
enforced before any device work, and the CPU baseline reports what it ran."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

import bench

WORKLOADS = ("c2", "c3i32", "c3u8", "c4")


def summary_fields(workload):
    path = os.path.join(bench.ROOT, "profiles", "traffic_k_persistent_%s.txt" % workload)
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


@pytest.mark.parametrize("workload", WORKLOADS)
def test_traffic_used_only_for_its_kernel_source(workload, monkeypatch):
    kv = summary_fields(workload)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: kv["kernel_source_sha256"])
    assert bench.load_traffic(workload) == float(kv["traffic_bytes_per_launch"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic(workload) is None


@pytest.mark.parametrize("workload", WORKLOADS)
def test_traffic_summary_is_consistent(workload):
    kv = summary_fields(workload)
    fetch = float(kv["fetch_bytes_per_launch"])
    write = float(kv["write_bytes_per_launch"])
    algo = float(kv["algorithmic_bytes_per_launch"])
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx(fetch + write, rel=1e-9, abs=1)
    assert float(kv["traffic_over_algorithmic"]) == pytest.approx((fetch + write) / algo,
                                                                  abs=1e-3)
    # the workload's algorithmic bytes: read I and J, write R, sizeof(T) each
    if workload == "c4":
        assert algo > 0  # 256 images of uneven size
    else:
        side = 4096 if workload == "c2" else 32768
        per_px = 12 if workload == "c3i32" else 3
        assert algo == per_px * side * side
    # the calibration scale turns the counters' KiB into bytes
    kib = [float(x) for x in kv["worker_fetch_kib_per_dispatch"].split(",")]
    assert min(kib) > 0
    assert fetch == pytest.approx(sum(kib) / len(kib) * 1024 / float(kv["scale_fetch"]), rel=1e-3)
    wkib = [float(x) for x in kv["worker_write_kib_per_dispatch"].split(",")]
    assert write == pytest.approx(sum(wkib) / len(wkib) * 1024 / float(kv["scale_write"]),
                                  rel=1e-3)


@pytest.mark.parametrize("workload", WORKLOADS)
def test_counter_scale_does_not_depend_on_the_copy_size(workload):
    # the copy of 64 MiB stays inside the 256 MB Infinity Cache, the copy of
    # 1024 MiB does not; the counters read the same fraction of the true bytes
    lines = open(os.path.join(bench.ROOT, "profiles",
                              "traffic_k_persistent_%s.txt" % workload)).read().splitlines()
    ratios = [l.split("counter/true")[1].split("/") for l in lines if "counter/true" in l]
    assert len(ratios) == 4
    for a, b in ratios:
        assert float(a) == pytest.approx(float(b), rel=0.01)


def test_traffic_missing_summary_is_none():
    assert bench.load_traffic("no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_reports_its_sample():
    cb = bench.cpu_baseline("c1", budget_s=0.05)
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["unit"] == "Mpixel/s"
    assert cb["value"] > 0
    assert cb["sample"].startswith("whole 512x512 image")


def test_pooled_oracle_task_matches_the_batch_recipe():
    # one task of the all-core batch baseline reconstructs image k of the
    # whole batch recipe
    import synth

    px, dt = bench._oracle_task(("c4", 3))
    (I, _), = synth.c4(only=[3])
    assert px == I.size and dt > 0
    assert synth.sha256(*synth.c4(only=[3])[0]) == synth.sha256(*synth.c4()[3])


def test_cv_protocol():
    assert bench.cv_protocol([1.0] * 10) == {"runs": 10, "cv": 0.0, "bound": 0.01, "held": True}
    assert not bench.cv_protocol([1.0] * 9)["held"]
    assert not bench.cv_protocol([1.0, 1.1] * 5)["held"]


def test_golden_digests_cover_every_workload():
    g = bench.golden()
    for name in ("c1", "c2", "c3i32", "c3u8"):
        assert name in g
    assert all("c4/%d" % k in g for k in range(256))
    assert all("c5/%d" % k in g for k in range(256))
