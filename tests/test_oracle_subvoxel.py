"""Pins of the oracle's sub-voxel hit distance (reading R20: one secant step on the trilinearly
interpolated TSDF across the entry point of the hit voxel).  Trilinear interpolation reproduces
a linear field exactly, so on a plane the refined distance is the analytic one; on a sphere the
error is second order in the voxel size, against first order for the walk's face distance."""
import numpy as np
import pytest

import oracle

H, N = 0.05, 48


def _grid_centres(n=N, h=H):
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h], -1)


def _map(sd, dtype="f32"):
    t = np.clip(sd, -0.3, 0.3).astype(np.float32)
    if dtype == "f16":
        from paper_2301_08068_amd import workloads as W
        return oracle.OracleMap(W.encode_f16(t), H, np.zeros(3), "f16"), t
    return oracle.OracleMap(t, H, np.zeros(3), "f32"), t


def _interior(p, margin=2.5):
    return np.all(p >= margin) and np.all(p <= N - margin)


@pytest.fixture(scope="module")
def plane():
    nrm = np.array([0.3, 0.5, 0.81])
    nrm /= np.linalg.norm(nrm)
    c = 1.6
    m, _ = _map(c - _grid_centres() @ nrm)
    return m, nrm, c


def test_field_at_centres_is_the_stored_value(plane):
    m, _, _ = plane
    rng = np.random.default_rng(3)
    for _ in range(50):
        i, j, k = rng.integers(0, N, size=3)
        assert oracle.field(m, [i + 0.5, j + 0.5, k + 0.5]) == float(m.data[k, j, i])
    # outside the centres' hull the indices clamp to the grid
    assert oracle.field(m, [-3.0, 0.2, 0.1]) == float(m.data[0, 0, 0])


def test_plane_distance_is_exact(plane):
    m, nrm, c = plane
    x = np.array([0.6, 0.7, 0.5])
    g = (x / H).astype(np.float32)
    dirs = oracle.directions(2048)
    tr = oracle.trace(m, g, dirs, 10.0)
    n_ok, worst_walk = 0, 0.0
    for r, d in zip(dirs, tr["d"]):
        rd = r.astype(np.float64)
        den = rd @ nrm
        if not np.isfinite(d) or den <= 0.05:
            continue
        true = (c - (g.astype(np.float64) * H) @ nrm) / den
        hit = g.astype(np.float64) + true / H * rd
        if not _interior(hit):
            continue
        ref = oracle.subvoxel(m, g, r, d)
        # float32 storage of the field is the only error left
        assert abs(ref - true) <= 1e-6, (r, d, ref, true)
        worst_walk = max(worst_walk, abs(d - true))
        n_ok += 1
    assert n_ok > 300
    assert worst_walk > 0.5 * H          # the walk's face distance is off by up to ~1.8 voxels


def test_sphere_error_is_second_order():
    R, ctr = 0.8, np.array([1.2, 1.2, 1.2])
    m, _ = _map(np.linalg.norm(_grid_centres() - ctr, axis=-1) - R)
    x = np.array([0.3, 0.4, 0.35])
    g = (x / H).astype(np.float32)
    dirs = oracle.directions(4096)
    tr = oracle.trace(m, g, dirs, 10.0)
    e_ref, e_walk = [], []
    for r, d in zip(dirs, tr["d"]):
        if not np.isfinite(d):
            continue
        o = g.astype(np.float64) * H
        rd = r.astype(np.float64)
        b = rd @ (o - ctr)
        disc = b * b - ((o - ctr) @ (o - ctr) - R * R)
        if disc <= 0.05:                  # keep rays that cross the sphere clearly
            continue
        true = -b - np.sqrt(disc)
        e_ref.append(abs(oracle.subvoxel(m, g, r, d) - true))
        e_walk.append(abs(d - true))
    assert len(e_ref) > 200
    assert max(e_ref) <= H * H / R            # second order: h^2 / R = 3.1 mm here
    assert np.median(e_walk) > 10 * np.median(e_ref)


def test_fallbacks(plane):
    m, _, _ = plane
    g = np.array([12.0, 14.0, 10.0], np.float32)
    r = np.array([1.0, 0.0, 0.0], np.float32)
    assert oracle.subvoxel(m, g, r, float("inf")) == float("inf")
    assert oracle.subvoxel(m, g, r, 0.0) == 0.0
    # no sign change in the sampled window: the walk's distance is kept
    free = oracle.OracleMap(np.full((N, N, N), 0.3, np.float32), H, np.zeros(3), "f32")
    assert oracle.subvoxel(free, g, r, 0.4) == 0.4
    # occupancy bytes have no field: unchanged
    occ = oracle.OracleMap(np.zeros((N, N, N), np.uint8), H, np.zeros(3), "u8")
    assert oracle.subvoxel(occ, g, r, 0.4) == 0.4


def test_f16_field_matches_its_decoded_values(plane):
    _, nrm, c = plane
    m16, t32 = _map(c - _grid_centres() @ nrm, "f16")
    bits = m16.data
    dec = bits.view(np.float16).astype(np.float64)
    for (i, j, k) in [(3, 4, 5), (20, 20, 20), (40, 2, 31)]:
        assert oracle.field(m16, [i + 0.5, j + 0.5, k + 0.5]) == dec[k, j, i]


def test_query_with_subvoxel_keeps_hits_and_changes_distances(plane):
    m, _, _ = plane
    from paper_2301_08068_amd import workloads as W
    p = dict(W.params("static", max_range=5.0))
    q0 = oracle.query(m, [0.6, 0.7, 0.5], [0.2, 0.3, 0.4], 1024, p)
    q1 = oracle.query(m, [0.6, 0.7, 0.5], [0.2, 0.3, 0.4], 1024, dict(p, subvoxel=1.0))
    assert q0["n_hit"] == q1["n_hit"] and q0["visits"] == q1["visits"]
    assert not np.array_equal(q0["S"], q1["S"])
