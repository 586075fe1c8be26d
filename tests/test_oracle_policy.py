"""Pins of the oracle's per-ray policy, combination and resolve (Sec. III-A Eq. 1,
Sec. III-C Eqs. 4-9, Sec. III-E Eq. 11, Sec. III-G) against closed forms, invariants and
library routines."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2301_08068_amd import workloads as W

P = W.params("static", max_range=5.0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "single_ray_worked.json")


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------- soft normalisation, weight

def test_soft_normalize_limits_and_direction(rng):
    assert np.array_equal(oracle.soft_normalize([0, 0, 0], 0.2), np.zeros(3))
    prev = 0.0
    for m in np.geomspace(1e-6, 1e4, 200):
        v = m * _unit(rng.normal(size=3))
        s = oracle.soft_normalize(v, 0.2)
        n = np.linalg.norm(s)
        assert n <= 1.0 and (n < 1.0 or m > 60)              # |s| < 1 up to rounding
        assert n >= prev - 4e-16 and (n > prev or m > 60)    # monotone in |v|
        prev = n
        # parallel to v: the denominator is a scalar (reading R1)
        assert np.linalg.norm(np.cross(s, v)) <= 1e-12 * n * m
    assert 1.0 - prev < 1e-12                                # -> 1 as |v| -> inf
    # small |v|: s(v) ~ v / (c log 2)
    v = np.array([1e-9, 0, 0])
    assert abs(oracle.soft_normalize(v, 0.5)[0] / (1e-9 / (0.5 * math.log(2))) - 1) < 1e-8


def test_weight_endpoints_and_shape():
    """w(0) = 1, w(r) = 0, zero slope at r, zero beyond r: these three conditions fix the
    printed quadratic (reading R3)."""
    r = 2.4
    assert oracle.weight(0.0, r) == 1.0
    assert abs(oracle.weight(r, r)) < 1e-15
    e = 1e-5
    assert abs((oracle.weight(r, r) - oracle.weight(r - e, r)) / e) < 1e-4
    assert abs((oracle.weight(e, r) - oracle.weight(0, r)) / e + 2 / r) < 1e-4
    ds = np.linspace(0, r, 1001)
    ws = np.array([oracle.weight(d, r) for d in ds])
    assert np.all(np.diff(ws) <= 1e-15) and np.all(ws >= -1e-15) and np.all(ws <= 1.0)
    assert oracle.weight(r * 1.0000001, r) == 0.0 and oracle.weight(100.0, r) == 0.0


# ---------------------------------------------------------------- per-ray policy

def test_single_ray_worked_values():
    g = json.load(open(GOLDEN))
    for case in g["cases"]:
        d, v = case["d"], case["v"]
        A, b = oracle.rmp_ray(P, [0, 0, 1], d, [0, 0, v])
        r = oracle.combine(P, np.array([[0.0, 0, 1]]), np.array([d]), np.array([0]), [0, 0, v])
        if "S_zz" in case:
            assert abs(A[2, 2] - case["S_zz"]) < 1e-11
            assert abs(b[2] - case["b_z"]) < 1e-9
            assert abs(r["f"][2] - case["f_z"]) < 1e-8
        if "phi" in case:
            assert abs(-r["f"][2] - case["phi"]) < 1e-8 * case["phi"]
        if "w" in case and "sigma" in case:
            assert abs(A[2, 2] - case["w"] * case["sigma"] ** 2) < 1e-11
        if "sigma" in case and "w" not in case:
            w = oracle.weight(d, P["radius"])
            assert abs(math.sqrt(A[2, 2] / w) - case["sigma"]) < 1e-9
        assert np.count_nonzero(A - np.diag(np.diag(A))) == 0 and A[0, 0] == 0 and A[1, 1] == 0
        assert r["rank"] == 1 and np.allclose(r["f"][:2], 0)


def test_single_ray_force_is_independent_of_metric(rng):
    """One contributing unit ray: (a r r^T)^+ (-a phi r) = -phi r for any weight a > 0."""
    for _ in range(50):
        r = _unit(rng.normal(size=3))
        v = r * rng.uniform(0.1, 3) + 0.3 * rng.normal(size=3)
        if v @ r <= 0.05:
            continue
        d = rng.uniform(0.05, 2.3)
        res = oracle.combine(P, r[None, :], np.array([d]), np.array([0]), v)
        p = max(0.0, v @ r) ** 2
        phi = P["eta_rep"] * math.exp(-d / P["nu_rep"]) + P["eta_damp"] * p / (d / P["nu_damp"] + P["eps"])
        assert np.allclose(res["f"], -phi * r, rtol=1e-9, atol=1e-9 * phi)
        assert res["rank"] == 1
        # S is rank one along r
        assert np.allclose(res["S"], res["S"][2, 2] / r[2] ** 2 * np.outer(r, r), rtol=1e-9, atol=1e-15)


def test_policy_scaling_laws(rng):
    """Structure of f_rep + f_damp: with eta_rep = 0 the force scales as 1/(d/nu + eps) and
    as the squared approach speed; with eta_damp -> small the repulsive part dominates."""
    r = _unit([0.3, -0.2, 0.9])
    p0 = dict(P, eta_rep=0.0)
    f = lambda d, s, pp: oracle.combine(pp, r[None], np.array([d]), np.array([0]), s * r)["f"]
    for d in (0.1, 0.5, 1.7):
        f1 = f(d, 1.0, p0)
        assert np.allclose(f(d, 2.0, p0), 4.0 * f1, rtol=1e-12)
        assert np.allclose(f1 * (d / p0["nu_damp"] + p0["eps"]), -p0["eta_damp"] * r, rtol=1e-12)
    # repulsive term decays as exp(-d / nu_rep) and points away from the obstacle
    pr = dict(P, eta_damp=1e-9)
    fa, fb = f(0.4, 1.0, pr), f(1.4, 1.0, pr)
    assert np.allclose(fb / fa, math.exp(-1.0 / P["nu_rep"]), rtol=1e-6)
    assert fa @ r < 0


def test_three_orthogonal_rays_decouple():
    """Rays along +x, +y, +z with different d: S is diagonal and each axis resolves alone."""
    rh = np.eye(3)
    d = np.array([0.4, 1.1, 1.9])
    v = np.array([0.7, 1.3, 2.1])
    res = oracle.combine(P, rh, d, np.array([0, 1, 2]), v)
    for a in range(3):
        single = oracle.combine(P, rh[a:a + 1], d[a:a + 1], np.array([0]), v)
        assert abs(res["S"][a, a] - single["S"][a, a]) <= 1e-15 * single["S"][a, a]
        assert abs(res["f"][a] - single["f"][a]) <= 1e-12 * abs(single["f"][a])
    assert np.count_nonzero(res["S"] - np.diag(np.diag(res["S"]))) == 0
    assert res["rank"] == 3


def test_zero_velocity_is_exactly_zero(tiny_map):
    """x_dot = 0 gives g_obs = 0, f_damp = 0, s = 0 and A_i = 0 exactly, so f = 0."""
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    for seed in range(100, 110):
        x, _ = W.free_state(tiny_map, seed)
        res = oracle.query(om, x, [0, 0, 0], 1024, P)
        assert np.all(res["S"] == 0) and np.all(res["b"] == 0) and np.all(res["f"] == 0)
        assert res["rank"] == 0 and res["n_contrib"] == 0


def test_rays_away_from_velocity_contribute_zero(rng):
    """A ray with x_dot . r <= 0 has zero metric and zero force (Sec. III-E)."""
    for _ in range(100):
        r = _unit(rng.normal(size=3))
        v = rng.normal(size=3)
        v -= (v @ r) * r + rng.uniform(0, 2) * r            # x_dot . r <= 0
        A, b = oracle.rmp_ray(P, r, rng.uniform(0.01, 2.0), v)
        assert np.all(A == 0) and np.all(b == 0)


def test_beyond_radius_contributes_zero(rng):
    for _ in range(50):
        r = _unit(rng.normal(size=3))
        A, b = oracle.rmp_ray(P, r, P["radius"] * rng.uniform(1.0000001, 3), 2 * r)
        assert np.all(A == 0) and np.all(b == 0)


def test_per_ray_metric_is_symmetric_psd_rank_one(rng):
    for _ in range(200):
        r = _unit(rng.normal(size=3))
        v = rng.normal(size=3) * 2
        A, b = oracle.rmp_ray(P, r, rng.uniform(0.0, 2.4), v)
        assert np.allclose(A, A.T, rtol=4e-16, atol=0)
        lam = np.linalg.eigvalsh(A)
        assert lam[0] >= -1e-15 * max(lam[2], 1e-300) and lam[1] <= 1e-12 * max(lam[2], 1e-300)
        # b = A (f_rep + f_damp) lies in range(A), i.e. along r
        assert np.linalg.norm(np.cross(b, r)) <= 1e-12 * max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- resolve

def test_sym3_eig_matches_library(rng):
    for _ in range(300):
        M = rng.normal(size=(3, 3)) * 10 ** rng.uniform(-3, 4)
        S = M @ M.T if rng.uniform() < 0.5 else M + M.T
        lam, Q = oracle.sym3_eig(S)
        ref = np.linalg.eigvalsh(S)
        scale = np.max(np.abs(ref))
        assert np.allclose(lam, ref, rtol=0, atol=1e-13 * scale)
        assert np.allclose(Q @ np.diag(lam) @ Q.T, S, rtol=0, atol=1e-13 * scale)
        assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-13)


def test_resolve_matches_library_pinv(rng):
    for k in range(300):
        Qr, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        lam = np.sort(10 ** rng.uniform(-4, 3, size=3))
        if k % 3 == 0:
            lam[0] = 0.0                                      # rank 2
        if k % 9 == 0:
            lam[1] = 0.0                                      # rank 1
        S = Qr @ np.diag(lam) @ Qr.T
        b = rng.normal(size=3) * 100
        f, lam_o, rank, flags = oracle.resolve(S, b, 1e-6)
        ref = np.linalg.pinv(S, rcond=1e-6, hermitian=True) @ b
        if flags & oracle.Q_ILL:
            continue
        assert np.allclose(f, ref, rtol=1e-8, atol=1e-8 * np.linalg.norm(ref))
        assert rank == int(np.sum(lam > 1e-6 * lam[2] * (1 + 1e-9)))


def test_resolve_zero_and_ill_flags():
    f, lam, rank, flags = oracle.resolve(np.zeros(9), np.zeros(3), 1e-6)
    assert np.all(f == 0) and rank == 0 and flags == 0
    S = np.diag([1.0, 1e-6 * 1.5, 0.0])                     # an eigenvalue next to the cut
    f, lam, rank, flags = oracle.resolve(S, np.ones(3), 1e-6)
    assert flags & oracle.Q_ILL
    S = np.diag([1.0, 1e-4, 0.5])                            # condition number 1e4
    assert oracle.resolve(S, np.ones(3), 1e-6)[3] & oracle.Q_ILL


# ---------------------------------------------------------------- full query invariants

def test_query_invariants(tiny_map):
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    n_checked = 0
    for seed in range(100, 140):
        x, v = W.free_state(tiny_map, seed)
        res = oracle.query(om, x, v, 1024, P)
        S, b, f = res["S"], res["b"], res["f"]
        assert np.allclose(S, S.T, rtol=0, atol=1e-14 * np.abs(S).max())
        lam = np.linalg.eigvalsh(S)
        if lam[2] == 0:
            continue
        assert lam[0] >= -1e-12 * lam[2]
        # b lies in range(S): S f reproduces b
        assert np.linalg.norm(S @ f - b) <= 1e-10 * np.linalg.norm(b)
        # f is orthogonal to the dropped eigenvectors
        ev, Q = np.linalg.eigh(S)
        for j in range(3):
            if ev[j] <= 1e-6 * ev[2]:
                assert abs(Q[:, j] @ f) <= 1e-9 * np.linalg.norm(f)
        assert res["n_contrib"] <= res["n_hit"] <= 1024
        n_checked += 1
    assert n_checked > 30


def test_sum_is_order_independent(tiny_map, rng):
    """The combination is a sum: permuting the rays changes S and b only by rounding."""
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    x, v = W.free_state(tiny_map, 123)
    dirs = oracle.directions(1024)
    g = oracle.grid_start(om, x)
    tr = oracle.trace(om, g, dirs, P["max_range"])
    a = oracle.combine(P, dirs.astype(np.float64), tr["d"], tr["hit"], v)
    perm = rng.permutation(1024)
    b = oracle.combine(P, dirs[perm].astype(np.float64), tr["d"][perm], tr["hit"][perm], v)
    assert np.allclose(a["S"], b["S"], rtol=1e-14, atol=1e-14 * np.abs(a["S"]).max())
    assert np.allclose(a["b"], b["b"], rtol=1e-14, atol=1e-14 * np.abs(a["b"]).max())
    q = oracle.query(om, x, v, 1024, P)
    assert np.array_equal(q["S"], a["S"]) and np.array_equal(q["f"], a["f"])


# ---------------------------------------------------------------- LiDAR scan path

def test_scan_reproduces_grid_query(tiny_map):
    """Feeding a grid query's hit points (r_i d_i) to the scan path with the same parameters
    reproduces S and b; the gap is the float32 rounding of the points and of |r_i| - 1."""
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    dirs = oracle.directions(1024)
    for seed in range(100, 110):
        x, v = W.free_state(tiny_map, seed)
        g = oracle.grid_start(om, x)
        tr = oracle.trace(om, g, dirs, P["max_range"])
        hit = tr["hit"] >= 0
        pts = (dirs[hit].astype(np.float64) * tr["d"][hit, None]).astype(np.float32)
        pts = np.concatenate([pts, np.zeros((7, 3), np.float32)])   # dropouts
        q = oracle.query(om, x, v, 1024, P)
        s = oracle.scan(pts, v, dict(P, min_range=1e-9))
        scale_S = max(np.abs(q["S"]).max(), 1e-300)
        scale_b = max(np.abs(q["b"]).max(), 1e-300)
        assert np.max(np.abs(s["S"] - q["S"])) <= 1e-6 * scale_S
        assert np.max(np.abs(s["b"] - q["b"])) <= 1e-6 * scale_b
        assert s["n_hit"] == q["n_hit"]


def test_scan_skips_dropouts_and_close_points(rng):
    v = np.array([1.0, 0.5, -0.2])
    good = rng.normal(size=(50, 3)).astype(np.float32)
    good *= (rng.uniform(0.3, 2.0, size=(50, 1)) / np.linalg.norm(good, axis=1, keepdims=True)).astype(np.float32)
    bad = np.array([[0, 0, 0], [np.nan, 1, 1], [np.inf, 0, 0], [0.05, 0, 0]], np.float32)
    L = W.params("lidar")
    a = oracle.scan(good, v, L)
    b = oracle.scan(np.concatenate([bad[:2], good, bad[2:]]), v, L)
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["b"], b["b"])
    assert a["n_hit"] == 50 and b["n_hit"] == 50
    e = oracle.scan(np.zeros((0, 3), np.float32), v, L)
    assert np.all(e["f"] == 0) and e["rank"] == 0
