"""Pins of the oracle's closed-loop rollout (ray policy + goal attractor, Sec. III-A Eq. 1 and
Sec. III-C Eqs. 3-4, integrated step by step): closed forms of the integrator and the attractor,
geometric invariants of the path measure, and collision detection."""
import numpy as np
import pytest

import oracle
from paper_2301_08068_amd import workloads as W

P = W.params("static", max_range=3.0)
ALPHA, BETA, DT = 10.0, 15.0, 0.01


@pytest.fixture(scope="module")
def empty():
    vm = W.VoxelMap("empty", np.ones((40, 40, 40), np.float32), 0.1, np.zeros(3), [], 0.3)
    return oracle.OracleMap.from_voxelmap(vm)


def test_attractor_closed_forms():
    # s(0) = 0: at the goal only the damping acts
    v = np.array([0.3, -1.2, 2.0])
    assert np.array_equal(oracle.attractor([1.0, 2.0, 3.0], [1.0, 2.0, 3.0], v, ALPHA, BETA, 0.2), -BETA * v)
    # far from the goal log1p(exp(-2 c |u|)) vanishes and s is the unit vector
    g = np.array([0.0, 0.0, 1e6])
    f = oracle.attractor(g, [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], ALPHA, BETA, 0.2)
    assert np.allclose(f, [0.0, 0.0, ALPHA], rtol=0, atol=1e-12)


def test_far_goal_follows_the_discrete_closed_form(empty):
    """Free space, goal 1e6 m away along +x: a_k = alpha - beta v_k exactly, so
    v_k = (alpha/beta)(1 - q^k) and x_k - x_0 = dt sum_{j=1..k} v_j with q = 1 - beta dt."""
    x0 = np.array([0.5, 2.0, 2.0])
    r = oracle.rollout(empty, x0, [0, 0, 0], 256, P, [1e6, 2.0, 2.0], ALPHA, BETA, DT, 30, 0.01)
    assert r["status"] == oracle.ROLLOUT_TIMEOUT and r["n_steps"] == 30
    q = 1.0 - BETA * DT
    k = np.arange(31)
    v_cf = ALPHA / BETA * (1.0 - q ** k)
    x_cf = x0[0] + DT * np.concatenate([[0.0], np.cumsum(v_cf[1:])])
    assert np.allclose(r["v"][:, 0], v_cf, rtol=1e-12, atol=1e-14)
    assert np.allclose(r["x"][:, 0], x_cf, rtol=1e-12, atol=1e-12)
    assert np.all(r["x"][:, 1:] == x0[1:]) and np.all(r["v"][:, 1:] == 0.0)


def test_empty_map_reaches_goal_on_a_straight_line(empty):
    x0, goal = np.array([0.55, 2.05, 2.0]), np.array([3.5, 2.05, 2.0])
    r = oracle.rollout(empty, x0, [0, 0, 0], 256, P, goal, ALPHA, BETA, DT, 1000, 0.05)
    assert r["status"] == oracle.ROLLOUT_GOAL
    assert np.linalg.norm(r["x"][-1] - goal) <= 0.05
    assert np.all(r["x"][:, 1:] == x0[1:])
    assert r["smoothness"] == 1.0
    assert abs(r["path_length"] - np.linalg.norm(r["x"][-1] - x0)) < 1e-12


def test_start_at_goal_takes_no_step(empty):
    r = oracle.rollout(empty, [1.0, 1.0, 1.0], [0.4, 0, 0], 64, P, [1.0, 1.0, 1.0], ALPHA, BETA, DT, 10, 0.01)
    assert r["status"] == oracle.ROLLOUT_GOAL and r["n_steps"] == 0


def test_smoothness_of_known_paths():
    assert oracle.smoothness([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]]) == 1.0
    assert oracle.smoothness([[0, 0, 0], [1, 0, 0], [1, 1, 0]]) == pytest.approx(0.5, abs=1e-15)
    assert oracle.smoothness([[0, 0, 0], [1, 0, 0], [0, 0, 0]]) == pytest.approx(0.0, abs=1e-15)
    # zero-length segments are skipped
    assert oracle.smoothness([[0, 0, 0], [1, 0, 0], [1, 0, 0], [2, 0, 0]]) == 1.0


def test_collision_is_detected():
    """A wall at x = 2.0..2.1 m and no obstacle force (zero gains): the walk toward a goal
    behind the wall enters the wall and stops there with a collision."""
    t = np.ones((40, 40, 40), np.float32)
    t[:, :, 20] = -0.05
    om = oracle.OracleMap(t, 0.1, np.zeros(3), "f32")
    p = dict(P, eta_rep=0.0, eta_damp=0.0)
    r = oracle.rollout(om, [0.55, 2.05, 2.05], [0, 0, 0], 64, p, [3.5, 2.05, 2.05], ALPHA, BETA, DT, 2000, 0.05)
    assert r["status"] == oracle.ROLLOUT_COLLISION
    assert 2.0 <= r["x"][-1][0] < 2.1
    # the full static-map policy keeps the same start out of the wall
    r2 = oracle.rollout(om, [0.55, 2.05, 2.05], [0, 0, 0], 256, P, [3.5, 2.05, 2.05], ALPHA, BETA, DT, 600, 0.05)
    assert r2["status"] != oracle.ROLLOUT_COLLISION
    assert r2["x"][:, 0].max() < 2.0


def test_zero_ray_weight_ignores_obstacles():
    """ray_weight = 0 removes the ray policy: the flight toward a goal behind a wall is the
    free-space flight (bit for bit) until it enters the wall."""
    t = np.ones((40, 40, 40), np.float32)
    t[:, :, 20] = -0.05
    om = oracle.OracleMap(t, 0.1, np.zeros(3), "f32")
    free = oracle.OracleMap(np.ones((40, 40, 40), np.float32), 0.1, np.zeros(3), "f32")
    x0, goal = [0.55, 2.05, 2.05], [3.5, 2.05, 2.05]
    r = oracle.rollout(om, x0, [0, 0, 0], 256, P, goal, ALPHA, BETA, DT, 2000, 0.05, ray_weight=0.0)
    f = oracle.rollout(free, x0, [0, 0, 0], 256, P, goal, ALPHA, BETA, DT, r["n_steps"], 0.05)
    assert r["status"] == oracle.ROLLOUT_COLLISION
    assert np.array_equal(r["x"], f["x"][: r["n_steps"] + 1])


def test_smoothness_sampling_stride():
    # a zigzag of right angles at every point is straight when every second point is kept
    zig = [[0, 0, 0], [1, 1, 0], [2, 0, 0], [3, 1, 0], [4, 0, 0]]
    assert oracle.smoothness(zig) == pytest.approx(0.5, abs=1e-15)
    assert oracle.smoothness(zig, every=2) == 1.0
    # a trailing partial stride is not sampled: 0, 3 and 6 are kept, the turn at 7 is not seen
    pts = [[i, 0, 0] for i in range(7)] + [[6, 5, 0]]
    assert oracle.smoothness(pts, every=3) == 1.0
    assert oracle.smoothness(pts) < 1.0
