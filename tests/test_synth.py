"""Seeded workload generator: determinism, shapes, float32 exactness."""
import numpy as np

from paper_2309_09102_amd import synth


def test_deterministic_and_float32_exact():
    a = synth.config2()
    b = synth.config2()
    assert np.array_equal(a.cand, b.cand) and np.array_equal(a.q_star, b.q_star)
    for arr in (a.cand, a.q_star, a.robot.a, a.robot.d, a.robot.alpha):
        assert np.array_equal(arr, arr.astype(np.float32).astype(np.float64))
    assert a.cand.shape == (256, 300, 7) and a.T == 300 and a.K == 256


def test_limits_and_branch_offsets():
    p = synth.config1()
    assert p.cand.shape == (16, 50, 7)
    assert np.all(p.cand <= p.robot.q_hi) and np.all(p.cand >= p.robot.q_lo)
    # 4 candidates carry a +-pi/2 offset on joints 2, 4 and 6 (1-based)
    dev = np.abs(p.cand - p.q_star[None]).mean(axis=1)        # [K][n]
    offset = dev[:, [1, 3, 5]].min(axis=1) > 0.5
    assert offset.sum() == 4
    assert np.all(dev[~offset].max(axis=1) < 0.2)


def test_ground_truth_inside_limits():
    for i in range(8):
        p = synth.config4_problem(i)
        assert 100 <= p.T <= 1000 and 64 <= p.K <= 512
        assert np.all(np.abs(p.q_star) <= 1.5 + 1e-6)


def test_serving_stream_shapes():
    arr = synth.config5_arrivals(duration_s=5.0)
    assert np.all(np.diff(arr) > 0) and 600 < len(arr) < 1400
    r = synth.config5_request(3)
    assert r.K in (128, 256, 512) and 50 <= r.T <= 2000
    assert 0.02 <= r.sigma <= 0.15


def test_targets_rounded():
    p = synth.config1()
    p2 = p.with_targets(np.full((p.T, 12), 0.1))
    assert np.all(p2.targets == np.float32(0.1))
