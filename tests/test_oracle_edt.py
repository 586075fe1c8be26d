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
