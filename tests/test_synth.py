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


def test_prismatic_robot_and_its_inputs():
    """The prismatic robot is the revolute robot of the same seed with one
    joint marked prismatic over [0, 0.4] m; its path, candidates and random
    configurations stay inside that travel and are float32-exact, and the
    revolute joints' inputs are unchanged by the mapping."""
    import math
    rb0 = synth.make_robot(3)
    rb = synth.make_robot_prismatic(3)
    assert list(rb.joint_type) == [1, 0, 0, 0, 0, 0, 0] and rb0.joint_type is None
    assert np.array_equal(rb.a, rb0.a) and np.array_equal(rb.d, rb0.d)
    assert rb.q_lo[0] == 0.0 and rb.q_hi[0] == np.float32(0.4)
    p = synth.make_problem(rb, seed=5, T=40, K=16, sigma=0.3, branch_frac=0.25)
    p0 = synth.make_problem(rb0, seed=5, T=40, K=16, sigma=0.3, branch_frac=0.25)
    for x in (p.q_star[:, 0], p.cand[..., 0]):
        assert x.min() >= 0.0 and x.max() <= rb.q_hi[0]
    assert np.array_equal(p.cand[..., 1:], p0.cand[..., 1:])
    assert np.array_equal(p.cand.astype(np.float32).astype(np.float64), p.cand)
    q = synth.random_configs(2, 500, rb)
    assert q[:, 0].min() >= 0.0 and q[:, 0].max() <= rb.q_hi[0]
    assert np.abs(q[:, 1:]).max() <= math.pi
    extra = synth.more_candidates(p, 8)
    assert extra[..., 0].min() >= 0.0 and extra[..., 0].max() <= rb.q_hi[0]


def test_serving_requests_distinct_and_distributed():
    """Each request of the stream has its own shape, path and noise: the
    candidates are float32 values inside the limits; the candidates without
    a branch offset scatter around q* with the request's sigma; round(frac K)
    candidates carry the +-pi/2 offset on joints 2, 4 and 6."""
    reqs = [synth.config5_request(i) for i in range(6)]
    assert len({(r.T, r.K, r.sigma) for r in reqs}) == 6
    for r in reqs:
        assert r.cand.dtype == np.float32 and r.cand.shape == (r.K, r.T, 7)
        assert np.all(r.cand <= r.robot.q_hi) and np.all(r.cand >= r.robot.q_lo)
        dev = r.cand.astype(np.float64) - r.q_star[None]
        shifted = np.abs(dev[:, :, [1, 3, 5]]).mean(axis=(1, 2)) > 0.8
        assert shifted.sum() == round(r.branch_frac * r.K)
        plain = dev[~shifted]
        inside = np.abs(r.q_star[None] + plain) < 2.8 - 1e-6   # not clamped
        z = plain[inside]
        assert abs(z.mean()) < 0.05 * r.sigma
        assert abs(z.std() / r.sigma - 1.0) < 0.05
    # requests are distinct (different paths and noise)
    a, b = reqs[0], reqs[1]
    assert not np.array_equal(a.q_star[:min(a.T, b.T)], b.q_star[:min(a.T, b.T)])
