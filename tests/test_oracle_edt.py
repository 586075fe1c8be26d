"""Pins of the oracle's exact distance transform (the ESDF behind the single-lookup policy of
Sec. III-D, reading R21): brute force over all occupied voxels, scipy's exact Euclidean
distance transform, and closed forms."""
import numpy as np
import pytest

import oracle
from paper_2301_08068_amd import workloads as W


def _omap(occ):
    t = np.where(occ, -0.05, 0.3).astype(np.float32)
    return oracle.OracleMap(t, 0.1, np.zeros(3), "f32")


def test_brute_force_small():
    rng = np.random.default_rng(4)
    occ = rng.uniform(size=(9, 10, 12)) < 0.04
    got = oracle.edt(_omap(occ))
    pts = np.argwhere(occ)                          # (k, j, i)
    kk, jj, ii = np.indices(occ.shape)
    want = np.full(occ.shape, np.iinfo(np.int64).max)
    for k, j, i in pts:
        want = np.minimum(want, (kk - k) ** 2 + (jj - j) ** 2 + (ii - i) ** 2)
    assert np.array_equal(got, want)


def test_matches_scipy_on_tiny_map(tiny_map):
    ndimage = pytest.importorskip("scipy.ndimage")
    occ = tiny_map.tsdf <= 0
    got = oracle.edt(oracle.OracleMap.from_voxelmap(tiny_map))
    d = ndimage.distance_transform_edt(~occ)
    assert np.array_equal(got, np.rint(d * d).astype(np.int64))


def test_closed_forms():
    occ = np.zeros((7, 8, 9), bool)
    assert np.all(oracle.edt(_omap(occ)) == -1)
    assert np.all(oracle.edt(_omap(~occ)) == 0)
    occ[2, 5, 1] = True
    kk, jj, ii = np.indices(occ.shape)
    assert np.array_equal(oracle.edt(_omap(occ)), (kk - 2) ** 2 + (jj - 5) ** 2 + (ii - 1) ** 2)


def test_encodings_agree(tiny_map):
    a = oracle.edt(oracle.OracleMap.from_voxelmap(tiny_map))
    b = oracle.edt(oracle.OracleMap(W.encode_f16(tiny_map.tsdf), 0.1, np.zeros(3), "f16"))
    c = oracle.edt(oracle.OracleMap(W.encode_u8(tiny_map.tsdf), 0.1, np.zeros(3), "u8"))
    assert np.array_equal(a, b) and np.array_equal(a, c)


def _plane_world(n=40, h=0.1):
    """Occupied half-space x >= 3.05 m (voxel columns i >= 30) of a 40^3 grid."""
    occ = np.zeros((n, n, n), bool)
    occ[:, :, 30:] = True
    return occ, h


def test_esdf_policy_faces_the_wall():
    """In front of a wall the distance is the centre-to-centre distance to it, the gradient
    points away from it, and the policy equals the obstacle policy of that single ray."""
    occ, h = _plane_world()
    m = oracle.OracleMap(np.where(occ, -0.05, 0.3).astype(np.float32), h, np.zeros(3), "f32")
    sq = oracle.edt(m)
    p = W.params("static")
    x, v = np.array([1.23, 2.0, 2.0]), np.array([0.7, 0.1, -0.2])
    q = oracle.esdf_query(m, sq, x, v, p)
    d = (30 - 12) * h                                   # voxel 12 to column 30, centre to centre
    A, b = oracle.rmp_ray(p, [1.0, 0.0, 0.0], d, v)
    assert np.allclose(q["S"], A.reshape(3, 3), rtol=0, atol=1e-12)
    assert np.allclose(q["b"], b, rtol=0, atol=1e-12)
    assert q["n_hit"] == 1 and q["n_contrib"] == 1
    # moving away from the wall: zero metric, nothing contributes
    q2 = oracle.esdf_query(m, sq, x, -v, p)
    assert q2["n_contrib"] == 0 and np.all(q2["S"] == 0)


def test_esdf_policy_degenerate_cases():
    p = W.params("static")
    free = oracle.OracleMap(np.full((8, 8, 8), 0.3, np.float32), 0.1, np.zeros(3), "f32")
    q = oracle.esdf_query(free, oracle.edt(free), [0.4, 0.4, 0.4], [1, 0, 0], p)
    assert q["n_hit"] == 0 and np.all(q["S"] == 0) and np.all(q["f"] == 0)
    occ, h = _plane_world(12)
    occ[:] = False
    occ[6, 6, 6] = True
    m = oracle.OracleMap(np.where(occ, -0.05, 0.3).astype(np.float32), h, np.zeros(3), "f32")
    q = oracle.esdf_query(m, oracle.edt(m), [0.65, 0.65, 0.65], [1, 0, 0], p)
    assert q["flags"] & oracle.Q_IN_COLLISION
