"""Pins of the oracle's voxel traversal (Sec. III-E: d_i = R(x, r_i); readings R6, R7, R9, R14).

Each pin checks the traversal against something it does not compute itself: exact
ray-plane geometry, a ray-sphere bracket, brute force over every voxel box, and exact
symmetries of the grid.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2301_08068_amd import workloads as W


def _map_from_prims(dims, h, prims, trunc=0.3):
    tsdf = W.build_tsdf(dims, h, (0.0, 0.0, 0.0), prims, trunc)
    return W.VoxelMap("t", tsdf, h, np.zeros(3), prims, trunc)


def _rand_dirs(rng, n):
    d = rng.normal(size=(n, 3))
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("plane", ["floor", "ceiling"])
def test_plane_on_voxel_face_is_exact(plane, rng):
    """A half-space whose plane is a voxel face voxelises exactly; d is the plane distance."""
    h = 0.1
    if plane == "floor":
        prims = [("halfspace_below", 2, 0.3)]        # plane z = 3 h, occupied layers k <= 2
    else:
        prims = [("slab", 2, 5.0, 7.0)]              # plane z = 50 h, occupied layers k >= 50
    vm = _map_from_prims((64, 64, 64), h, prims)
    om = oracle.OracleMap.from_voxelmap(vm)
    dirs = oracle.directions(4096)
    checked = 0
    for s in range(20):
        g = np.array([rng.uniform(5, 59), rng.uniform(5, 59), rng.uniform(8, 45)], dtype=np.float32)
        tr = oracle.trace(om, g, dirs, 1e9)
        gz = float(g[2])
        for i in range(len(dirs)):
            r = dirs[i].astype(np.float64)
            toward = r[2] < 0 if plane == "floor" else r[2] > 0
            if not toward:
                assert tr["hit"][i] == -1
                continue
            zp = 3.0 if plane == "floor" else 50.0
            t = (zp - gz) / r[2]
            p = g.astype(np.float64) + t * r
            if tr["flags"][i] & oracle.TIE:
                continue
            near_edge = min(abs(p[0]), abs(p[1]), abs(p[0] - 64), abs(p[1] - 64)) < 1e-6
            if near_edge:
                continue
            if not (0.0 < p[0] < 64.0 and 0.0 < p[1] < 64.0):
                assert tr["hit"][i] == -1           # leaves through a side before the plane
                continue
            layer = 2 if plane == "floor" else 50
            exp_lin = int(math.floor(p[0])) + 64 * (int(math.floor(p[1])) + 64 * layer)
            assert tr["hit"][i] == exp_lin
            assert abs(tr["d"][i] - t * h) <= 1e-12 * t * h
            checked += 1
    assert checked > 10000


def test_sphere_bracket(rng):
    """Hits lie within (sqrt(3)/2) h of the sphere; lines missing the inflated sphere miss;
    rays entering the deflated sphere hit no later than that entry."""
    h, R, c = 0.1, 1.3, np.array([3.2, 3.3, 3.1])
    vm = _map_from_prims((64, 64, 64), h, [("sphere", *c.tolist(), R)])
    om = oracle.OracleMap.from_voxelmap(vm)
    dirs = oracle.directions(8192)
    half_diag = math.sqrt(3) / 2 * h
    n_hit = n_in = 0
    for s in range(12):
        while True:
            x = rng.uniform(0.3, 6.1, size=3)
            if np.linalg.norm(x - c) > R + 0.3:
                break
        g = oracle.grid_start(om, x)
        xe = g.astype(np.float64) * h                   # the start the traversal really uses
        tr = oracle.trace(om, g, dirs, 1e9)
        r = dirs.astype(np.float64)
        oc = xe - c
        b = r @ oc
        for Rk, kind in ((R + half_diag, "outer"), (R - half_diag, "inner")):
            disc = b * b - (oc @ oc - Rk * Rk)
            if kind == "outer":
                misses = disc < 0
                assert np.all(tr["hit"][misses] == -1)
            else:
                ent = -b - np.sqrt(np.maximum(disc, 0))
                enters = (disc > 0) & (ent > 0)
                assert np.all(tr["hit"][enters] >= 0)
                assert np.all(tr["d"][enters] <= ent[enters] + 1e-9)
                n_in += int(enters.sum())
        hits = tr["hit"] >= 0
        p = xe + r[hits] * tr["d"][hits, None]
        dist = np.linalg.norm(p - c, axis=1)
        assert np.all(dist >= R - half_diag - 1e-9) and np.all(dist <= R + half_diag + 1e-9)
        n_hit += int(hits.sum())
    assert n_hit > 5000 and n_in > 2000


def _brute_force_first_hit(occ, g, r, max_t):
    """First occupied voxel box that the ray crosses with positive length (slab method)."""
    nz, ny, nx = occ.shape
    kk, jj, ii = np.nonzero(occ)
    lo = np.stack([ii, jj, kk], 1).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - g) / r
        t2 = (lo + 1 - g) / r
    tn = np.minimum(t1, t2)
    tf = np.maximum(t1, t2)
    zero = r == 0
    if zero.any():
        inside = (g >= lo) & (g <= lo + 1)
        tn = np.where(zero, np.where(inside, -np.inf, np.inf), tn)
        tf = np.where(zero, np.where(inside, np.inf, -np.inf), tf)
    ent = tn.max(1)
    ex = tf.min(1)
    ok = (ex > np.maximum(ent, 0) + 1e-9) & (ent <= max_t)
    if not ok.any():
        return -1, math.inf, ent, ok
    j = np.argmin(np.where(ok, ent, np.inf))
    lin = int(ii[j] + nx * (jj[j] + ny * kk[j]))
    return lin, float(ent[j]), ent, ok


@pytest.mark.parametrize("dims,p_occ,seed", [((8, 8, 8), 0.05, 0), ((12, 9, 14), 0.3, 1),
                                            ((16, 11, 7), 0.05, 2), ((10, 16, 13), 0.3, 3)])
def test_brute_force_tiny_grids(dims, p_occ, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    occ = rng.uniform(size=(nz, ny, nx)) < p_occ
    tsdf = np.where(occ, -0.05, 0.05).astype(np.float32)
    om = oracle.OracleMap(tsdf, 1.0, (0, 0, 0))
    n_ok = n_flag = 0
    for s in range(10):
        while True:
            g = (rng.uniform(0, 1, size=3) * np.array(dims)).astype(np.float32)
            v0 = np.floor(g).astype(int)
            if not occ[v0[2], v0[1], v0[0]]:
                break
        dirs = _rand_dirs(rng, 1000)
        max_t = rng.uniform(2, 2 * max(dims))
        tr = oracle.trace(om, g, dirs, max_t)
        for i in range(len(dirs)):
            lin, t, _, _ = _brute_force_first_hit(occ, g.astype(np.float64), dirs[i].astype(np.float64), max_t)
            if tr["flags"][i] & (oracle.TIE | oracle.RANGE_TIE):
                alts = set(int(a) for a in tr["alt_hit"][i, :tr["alt_n"][i]])
                assert lin in alts
                n_flag += 1
                continue
            assert tr["hit"][i] == lin, (s, i)
            if lin >= 0:
                assert abs(tr["d"][i] - t) <= 1e-9 * max(1.0, t)
            n_ok += 1
    assert n_ok > 9000


def test_translation_invariance_exact(rng, tiny_map):
    """Embedding the grid at an integer offset re-indexes hits and leaves d bit-identical."""
    occ = tiny_map.tsdf
    off = (5, 9, 3)
    big = np.full((64 + 8, 64 + 12, 64 + 10), 0.3, dtype=np.float32)
    big[off[2]:off[2] + 64, off[1]:off[1] + 64, off[0]:off[0] + 64] = occ
    # the padding is free, so a ray leaving the block still ends as a miss
    om_a = oracle.OracleMap(occ, 1.0, (0, 0, 0))
    om_b = oracle.OracleMap(big, 1.0, (0, 0, 0))
    dirs = oracle.directions(2048)
    for s in range(6):
        while True:
            g = (np.round(rng.uniform(1, 63, size=3) * 1024) / 1024 + 1 / 2048).astype(np.float32)
            v0 = np.floor(g).astype(int)
            if occ[v0[2], v0[1], v0[0]] > 0:
                break
        gb = (g + np.array(off, dtype=np.float32)).astype(np.float32)
        assert np.array_equal(gb.astype(np.float64) - np.array(off), g.astype(np.float64))
        ta = oracle.trace(om_a, g, dirs, 40.0)
        tb = oracle.trace(om_b, gb, dirs, 40.0)
        ha = ta["hit"] >= 0
        # every hit inside the block maps to the shifted voxel, same distance bit for bit
        i = ta["hit"][ha] % 64
        j = (ta["hit"][ha] // 64) % 64
        k = ta["hit"][ha] // (64 * 64)
        lin_b = (i + off[0]) + 74 * ((j + off[1]) + 76 * (k + off[2]))
        assert np.array_equal(tb["hit"][ha], lin_b)
        assert np.array_equal(tb["d"][ha], ta["d"][ha])
        assert np.array_equal(tb["flags"][ha], ta["flags"][ha])


def test_origin_and_voxel_size_enter_only_through_g(tiny_map):
    """Moving origin and position together (exactly representable shifts) and scaling the
    voxel size changes nothing but the metric scale of d."""
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    dirs = oracle.directions(2048)
    x, _ = W.free_state(tiny_map, 31)
    x = np.round(x * 1024) / 1024
    base = oracle.trace(om, oracle.grid_start(om, x), dirs, 5.0)
    o2 = np.array([-3.25, 1.5, 100.0])
    om2 = oracle.OracleMap(tiny_map.tsdf, tiny_map.voxel_m, o2)
    g2 = oracle.grid_start(om2, x + o2)
    assert np.array_equal(g2, oracle.grid_start(om, x))
    t2 = oracle.trace(om2, g2, dirs, 5.0)
    assert np.array_equal(t2["hit"], base["hit"]) and np.array_equal(t2["d"], base["d"])
    # voxel size 0.1 -> 0.4 with the same grid-space start: d scales by 4 exactly (powers of 2
    # aside, d = t h is one rounding of the same t)
    om4 = oracle.OracleMap(tiny_map.tsdf, 0.4, (0, 0, 0))
    t4 = oracle.trace(om4, oracle.grid_start(om, x), dirs, 20.0)
    hit = base["hit"] >= 0
    assert np.array_equal(t4["hit"][hit], base["hit"][hit])
    assert np.allclose(t4["d"][hit], 4 * base["d"][hit], rtol=4e-16)
    assert oracle.grid_start(om2, x) is None                 # now outside the shifted grid


def test_axis_permutation_and_mirror_symmetry(rng, tiny_map):
    """Permuting grid axes (with g and r) or mirroring one axis maps hits exactly."""
    occ = tiny_map.tsdf  # [z, y, x]
    n = 64
    dirs = oracle.directions(2048)
    om = oracle.OracleMap(occ, 1.0, (0, 0, 0))
    # permutation (x, y, z) -> (y, z, x): new axis a holds old axis perm[a]
    perm = [1, 2, 0]
    occ_p = np.ascontiguousarray(np.transpose(occ, (2 - perm[2], 2 - perm[1], 2 - perm[0])))
    om_p = oracle.OracleMap(occ_p, 1.0, (0, 0, 0))
    # mirror x: voxel i -> n-1-i, g_x -> n - g_x, r_x -> -r_x
    occ_m = np.ascontiguousarray(occ[:, :, ::-1])
    om_m = oracle.OracleMap(occ_m, 1.0, (0, 0, 0))
    for s in range(4):
        while True:
            g = (np.round(rng.uniform(1, 63, size=3) * 256) / 256 + 1 / 512).astype(np.float32)
            v0 = np.floor(g).astype(int)
            if occ[v0[2], v0[1], v0[0]] > 0:
                break
        t0 = oracle.trace(om, g, dirs, 40.0)
        unflagged = (t0["flags"] & oracle.TIE) == 0
        ijk = np.stack([t0["hit"] % n, (t0["hit"] // n) % n, t0["hit"] // (n * n)], 1)
        # permuted
        tp = oracle.trace(om_p, g[perm], np.ascontiguousarray(dirs[:, perm]), 40.0)
        hp = ijk[:, perm]
        lin_p = hp[:, 0] + n * (hp[:, 1] + n * hp[:, 2])
        sel = unflagged & (t0["hit"] >= 0)
        assert np.array_equal(tp["hit"][sel], lin_p[sel])
        assert np.array_equal(tp["d"][sel], t0["d"][sel])
        assert np.array_equal(tp["hit"][unflagged] < 0, t0["hit"][unflagged] < 0)
        # mirrored
        gm = g.copy(); gm[0] = np.float32(n - g[0])
        dm = dirs.copy(); dm[:, 0] = -dm[:, 0]
        tm = oracle.trace(om_m, gm, dm, 40.0)
        lin_m = (n - 1 - ijk[:, 0]) + n * (ijk[:, 1] + n * ijk[:, 2])
        assert np.array_equal(tm["hit"][sel], lin_m[sel])
        assert np.array_equal(tm["d"][sel], t0["d"][sel])


def test_visits_equal_l1_voxel_distance(tiny_map, rng):
    """A 6-connected walk visits 1 + |dv|_1 voxels between start and hit voxel."""
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    dirs = oracle.directions(1024)
    x, v = W.free_state(tiny_map, 7)
    g = oracle.grid_start(om, x)
    tr = oracle.trace(om, g, dirs, 5.0)
    v0 = np.floor(g).astype(np.int64)
    hit = tr["hit"] >= 0
    ijk = np.stack([tr["hit"] % 64, (tr["hit"] // 64) % 64, tr["hit"] // 4096], 1)
    l1 = np.abs(ijk - v0).sum(1)
    assert np.array_equal(tr["visits"][hit], 1 + l1[hit])


def test_encodings_give_identical_hits(tiny_map, paper_map):
    """Float32 TSDF, sign-preserving float16 TSDF and uint8 occupancy: same hits, same d."""
    for vm, n, rmax, seed in ((tiny_map, 1024, 5.0, 100), (paper_map, 2048, 10.0, 200)):
        x, _ = W.free_state(vm, seed)
        enc = {"f32": vm.tsdf, "f16": W.encode_f16(vm.tsdf), "u8": W.encode_u8(vm.tsdf)}
        assert np.array_equal((enc["f16"].view(np.float16) <= 0), vm.tsdf <= 0)
        dirs = oracle.directions(n)
        outs = []
        for k, data in enc.items():
            om = oracle.OracleMap(data, vm.voxel_m, vm.origin_m, k)
            outs.append(oracle.trace(om, oracle.grid_start(om, x), dirs, rmax))
        for o in outs[1:]:
            assert np.array_equal(o["hit"], outs[0]["hit"])
            assert np.array_equal(o["d"], outs[0]["d"])


def test_start_in_collision_and_out_of_grid(tiny_map):
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    dirs = oracle.directions(64)
    g = np.array([10.5, 10.5, 1.5], dtype=np.float32)      # inside the floor
    tr = oracle.trace(om, g, dirs, 5.0)
    assert np.all(tr["hit"] == 10 + 64 * (10 + 64 * 1)) and np.all(tr["d"] == 0.0)
    assert np.all(tr["flags"] & oracle.IN_COLLISION)
    with pytest.raises(ValueError):
        oracle.trace(om, np.array([64.0, 3, 3], np.float32), dirs, 5.0)
    assert oracle.grid_start(om, [-0.01, 1, 1]) is None


def test_range_is_closed_and_misses(tiny_map):
    """A voxel entered exactly at max range counts; anything beyond is a miss."""
    tsdf = np.full((16, 16, 16), 0.05, np.float32)
    tsdf[:, :, 12] = -0.05                                 # wall at x = 12
    om = oracle.OracleMap(tsdf, 0.5, (0, 0, 0))
    g = np.array([2.0, 8.25, 8.25], np.float32)            # wall face 10 voxels = 5 m away
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    assert oracle.trace(om, g, d, 5.0)["hit"][0] == 12 + 16 * (8 + 16 * 8)
    assert oracle.trace(om, g, d, 5.0)["d"][0] == 5.0
    assert oracle.trace(om, g, d, 4.999)["hit"][0] == -1
    assert oracle.trace(om, g, np.array([[-1.0, 0, 0]], np.float32), 100.0)["hit"][0] == -1


def test_exact_tie_steps_lowest_axis_and_lists_both_orders():
    """A ray through a voxel edge crosses x and y faces at the same t: the primary walk
    steps x first (lowest axis, reading R14); the y-first walk is in the admissible set."""
    n = 8
    g = np.array([2.5, 2.5, 2.5], np.float32)
    r = np.array([[1.0, 1.0, 0.0]], np.float32)
    r /= np.float32(np.sqrt(2.0))
    assert r[0, 0] == r[0, 1]
    lin = lambda i, j, k: i + n * (j + n * k)
    for occ_at, expect_primary in (((3, 2, 2), lin(3, 2, 2)), ((2, 3, 2), -1)):
        tsdf = np.full((n, n, n), 0.5, np.float32)
        tsdf[occ_at[2], occ_at[1], occ_at[0]] = -0.5
        om = oracle.OracleMap(tsdf, 1.0, (0, 0, 0))
        tr = oracle.trace(om, g, r, 100.0)
        assert tr["hit"][0] == expect_primary
        assert tr["flags"][0] & oracle.TIE
        alts = set(tr["alt_hit"][0, :tr["alt_n"][0]].tolist())
        assert lin(*occ_at) in alts


def test_f16_occupancy_of_special_values():
    """Occupancy from binary16 bits: +-0 and negatives occupied; positives, +inf, NaN free."""
    pats = {0x0000: True, 0x8000: True, 0x0001: False, 0x8001: True, 0x7C00: False,
            0x3C00: False, 0xBC00: True, 0x7E00: False, 0x03FF: False, 0x83FF: True}
    for bits, occ in pats.items():
        data = np.full((1, 1, 4), 0x3C00, np.uint16)
        data[0, 0, 2] = bits
        om = oracle.OracleMap(data, 1.0, (0, 0, 0), "f16")
        tr = oracle.trace(om, np.array([0.5, 0.5, 0.5], np.float32),
                          np.array([[1.0, 0.0, 0.0]], np.float32), 100.0)
        assert (tr["hit"][0] == 2) == occ, hex(bits)
