"""The bench line's traffic figures come from committed counter summaries and
are dropped once the kernel they describe has changed (CPU only)."""
import json
import os

import pytest

import bench

SUMMARIES = ["hbm_traffic_T300_K256.json", "hbm_traffic_full_chip_T300_K256.json"]
KERNEL = "lm_kernel<float, false, false, false>"


@pytest.mark.parametrize("summary", SUMMARIES)
def test_summary_matches_recorded_bytes_or_is_stale(summary):
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", summary)))
    k = rec["kernels"][KERNEL]
    assert k["bytes_per_launch"] > 0
    got = bench.measured_traffic(KERNEL, summary)
    if k["sources_sha"] == bench.kernel_sources_sha(k["sources"]):
        assert got is not None and got["bytes_per_launch"] == k["bytes_per_launch"]
    else:
        assert got is None


@pytest.mark.parametrize("summary", SUMMARIES)
def test_changed_sources_drop_the_figure(summary, monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda files: "0" * 16)
    assert bench.measured_traffic(KERNEL, summary) is None


def test_missing_summary_or_kernel_gives_none():
    assert bench.measured_traffic(KERNEL, "no_such_summary.json") is None
    assert bench.measured_traffic("no_such_kernel", SUMMARIES[0]) is None


def test_full_chip_traffic_exceeds_single_plan():
    # 256 plans cannot move fewer bytes than one; the counters gave about 70x
    # more per plan once the factors no longer fit in the L2
    one = json.load(open(os.path.join(bench.ROOT, "profiles", SUMMARIES[0])))["kernels"][KERNEL]
    full = json.load(open(os.path.join(bench.ROOT, "profiles", SUMMARIES[1])))["kernels"][KERNEL]
    assert full["plans"] == 256
    assert full["bytes_per_launch"] / full["plans"] >= one["bytes_per_launch"]
