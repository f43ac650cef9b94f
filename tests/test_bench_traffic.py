"""The bench line's traffic figures come from committed counter summaries and
are dropped once the kernel they describe has changed (CPU only)."""
import json
import os

import pytest

import bench

SUMMARY = "hbm_traffic_serving.json"
KEYS = ["serving:lm", "serving:dp_lists"]


@pytest.mark.parametrize("key", KEYS)
def test_summary_matches_recorded_bytes_or_is_stale(key):
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", SUMMARY)))
    k = rec["kernels"][key]
    assert k["bytes_per_unit"] > 0 and k["units"] > 0
    got = bench.measured_traffic(key, SUMMARY)
    if k["sources_sha"] == bench.kernel_sources_sha(k["sources"]):
        assert got is not None and got["bytes_per_unit"] == k["bytes_per_unit"]
    else:
        assert got is None


@pytest.mark.parametrize("key", KEYS)
def test_changed_sources_drop_the_figure(key, monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda files: "0" * 16)
    assert bench.measured_traffic(key, SUMMARY) is None


def test_missing_summary_or_kernel_gives_none():
    assert bench.measured_traffic(KEYS[0], "no_such_summary.json") is None
    assert bench.measured_traffic("no_such_kernel", SUMMARY) is None


def test_recorded_bytes_follow_from_the_counters():
    """bytes per unit = (FETCH_SIZE x fetch scale + WRITE_SIZE x write scale)
    KiB x 1024 / units, with the scales from the copy calibration (a copy's
    FETCH_SIZE reads half the bytes it moves)."""
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", SUMMARY)))
    assert rec["fetch_scale"] == pytest.approx(2.0, rel=0.01)
    assert rec["write_scale"] == pytest.approx(1.0, rel=0.01)
    for key in KEYS:
        k = rec["kernels"][key]
        b = (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024
        assert k["bytes_per_unit"] == pytest.approx(b / k["units"], rel=1e-12)
