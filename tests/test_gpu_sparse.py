"""Sparse block maps on the GPU (rmpc_sparse_map_upload): the exact walk through the block hash
against the float64 oracle walking the same voxels expanded into a dense grid large enough
that no ray leaves it (hits and float64 distances bit for bit, flags and visits exact, TIE a
subset), query sums, negative block coordinates, collision starts, error handling, and an
outdoor-sized world at the bench's size checked on a dense crop around the robot."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2301_08068_amd import workloads as W  # noqa: E402
from gpu_common import compare_query  # noqa: E402

P_TINY = W.params("static", max_range=5.0)
P_PAPER = W.params("static", max_range=10.0)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08068_amd import binding
    c = binding.Context(0, arena_bytes=3 << 30)
    yield c
    c.close()


def _sparse_hits_as_lin(gpu, sm, lo_vox, dims):
    """Hit (slot * 512 + x + 8 y + 64 z) -> linear index in the dense crop starting at lo_vox."""
    nx, ny, _ = dims
    h = gpu["hit"].astype(np.int64)
    out = np.full(h.shape, -1, np.int64)
    ok = h >= 0
    slot, loc = h[ok] // 512, h[ok] % 512
    b = sm.coords[slot].astype(np.int64) * 8 - np.asarray(lo_vox, np.int64)
    vx, vy, vz = b[:, 0] + loc % 8, b[:, 1] + (loc // 8) % 8, b[:, 2] + loc // 64
    out[ok] = vx + nx * (vy + ny * vz)
    return out


def _dyadic_state(m, sm, shift, seed):
    """A free start of dense map m, moved so that its sparse grid coordinates are multiples of
    1/1024 (exact in float32, and after any whole-voxel shift), and a velocity."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = m.tsdf.shape
    while True:
        k = rng.integers(0, np.array([nx, ny, nz]) * 1024)
        v0 = k // 1024
        if m.tsdf[v0[2], v0[1], v0[0]] > 0:
            break
    g = k / 1024.0 + 8.0 * np.asarray(shift)
    x = sm.origin_m + g * sm.voxel_m
    assert np.all(((x - sm.origin_m) / sm.voxel_m).astype(np.float32) == g)
    return x, rng.normal(0.0, 1.0, size=3)


def _dense_start(sm, x, lo_vox):
    """The sparse query's start g = float32((x - origin) / h), moved into the dense crop's
    frame (g - lo, exact in float32, checked)."""
    g = ((np.asarray(x, np.float64) - sm.origin_m) / sm.voxel_m).astype(np.float32)
    gd = g.astype(np.float64) - np.asarray(lo_vox, np.float64)
    assert np.all(gd.astype(np.float32).astype(np.float64) == gd)
    return gd.astype(np.float32)


def _compare(gpu, orc, sm, lo_vox, dims, label):
    hit_g = _sparse_hits_as_lin(gpu, sm, lo_vox, dims)
    hit_o = orc["hit"].astype(np.int64)
    flagged = (orc["flags"] & (oracle.TIE | oracle.RANGE_TIE)) != 0
    same = hit_g == hit_o
    bad = ~same & ~flagged
    assert not bad.any(), f"{label}: {bad.sum()} unflagged rays differ, e.g. ray {np.argmax(bad)}"
    for i in np.nonzero(~same)[0]:
        assert hit_g[i] in orc["alt_hit"][i, :orc["alt_n"][i]], f"{label}: ray {i} not admissible"
    hs = same & (hit_o >= 0)
    assert np.array_equal(gpu["d"][hs], orc["d"][hs]), f"{label}: distances differ"
    assert np.all(np.isinf(gpu["d"][same & (hit_o < 0)]))
    gf, of = gpu["flags"][same].astype(np.uint32), orc["flags"][same].astype(np.uint32)
    T = np.uint32(oracle.TIE)
    assert np.array_equal(gf & ~T, of & ~T), f"{label}: flags differ"
    assert not np.any(gf & ~of & T), f"{label}: TIE where the oracle has none"
    assert np.array_equal(gpu["visits"][same], orc["visits"][same]), f"{label}: visits differ"
    return int(same.sum()), int(flagged.sum())


@pytest.mark.parametrize("shift,keep_free", [((7, 7, 7), 0.3), ((-40, -33, -9), 0.0)])
def test_sparse_tiny_parity(ctx, tiny_map, shift, keep_free):
    """The tiny map's blocks (all occupied ones, a seeded share of the free ones) at block
    offset `shift`, against the oracle on a dense grid padded by 7 blocks (56 voxels > the
    50-voxel range) on every side."""
    sm = W.sparse_from_dense(tiny_map, offset_blocks=shift, keep_free=keep_free, seed=5)
    mid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    lo = (np.asarray(shift) - 7) * 8
    hi = (np.asarray(shift) + 8 + 7) * 8
    dense, o_dense = sm.dense_crop(lo, hi)
    om = oracle.OracleMap(dense, sm.voxel_m, o_dense, "f32")
    dirs = oracle.directions(1024)
    n_same = n_flag = 0
    try:
        for seed in range(100, 160):
            x, v = _dyadic_state(tiny_map, sm, shift, seed)
            g = ctx.trace(mid, x, 1024, P_TINY)
            gd = _dense_start(sm, x, lo)
            o = oracle.trace(om, gd, dirs, P_TINY["max_range"])
            s, f = _compare(g, o, sm, lo, dense.shape[::-1], f"shift {shift} seed {seed}")
            n_same += s
            n_flag += f
            if seed % 4 == 0:
                q = ctx.query(mid, x, v, 1024, P_TINY)
                oq = oracle.combine(P_TINY, dirs, o["d"], o["hit"], v)
                oq["visits"] = int(o["visits"].sum())
                oq["n_tie"] = int(np.count_nonzero(o["flags"] & oracle.TIE))
                compare_query(q, oq, f"query seed {seed}")
    finally:
        ctx.release(mid)
    print(f"sparse tiny {shift}: {n_same} rays identical, {n_flag} flagged, {sm.n_blocks} blocks")


def test_sparse_collision_start(ctx, tiny_map):
    """A start in an occupied voxel: every ray hits it at distance 0 (IN_COLLISION)."""
    sm = W.sparse_from_dense(tiny_map, offset_blocks=(3, -2, 1), keep_free=0.0, seed=6)
    mid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    try:
        k = int(np.argmax(np.any(sm.values <= 0, axis=(1, 2, 3))))
        z, y, x = np.argwhere(sm.values[k] <= 0)[0]
        vox = sm.coords[k].astype(np.int64) * 8 + np.array([x, y, z])
        pos = sm.origin_m + (vox + 0.5) * sm.voxel_m
        q = ctx.query(mid, pos, np.array([0.3, -0.2, 0.1]), 512, P_TINY)
        assert q["flags"] & oracle.Q_IN_COLLISION and q["n_hit"] == 512
        t = ctx.trace(mid, pos, 512, P_TINY)
        assert np.all(t["hit"] == k * 512 + x + 8 * y + 64 * z) and np.all(t["d"] == 0.0)
        assert np.all(t["visits"] == 1) and np.all(t["flags"] & oracle.IN_COLLISION)
    finally:
        ctx.release(mid)


def test_sparse_errors(ctx, tiny_map):
    from paper_2301_08068_amd import binding
    sm = W.sparse_from_dense(tiny_map, offset_blocks=(0, 0, 0), keep_free=0.0, seed=7)
    with pytest.raises(binding.RmpcError, match="twice"):
        ctx.upload_sparse(np.concatenate([sm.coords, sm.coords[:1]]), np.concatenate([sm.values, sm.values[:1]]),
                          sm.voxel_m, sm.origin_m)
    bad = sm.coords.copy()
    bad[0, 1] = 1 << 20
    with pytest.raises(binding.RmpcError, match="coordinate"):
        ctx.upload_sparse(bad, sm.values, sm.voxel_m, sm.origin_m)
    for fv in (0.0, -0.3, float("nan"), 1e6):                 # 1e6 is inf in binary16
        with pytest.raises(binding.RmpcError, match="free_value"):
            ctx.upload_sparse(sm.coords, W.encode_f16(sm.values), sm.voxel_m, sm.origin_m, "f16", fv)
    occ = ctx.upload_sparse(sm.coords, W.encode_u8(sm.values), sm.voxel_m, sm.origin_m, "u8", 0.0)
    try:
        x, v = W.free_state(tiny_map, 100)
        with pytest.raises(binding.RmpcError, match="TSDF"):
            ctx.query(occ, x, v, 256, dict(P_TINY, subvoxel=1.0))
    finally:
        ctx.release(occ)
    mid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    try:
        x, v = W.free_state(tiny_map, 100)
        with pytest.raises(binding.RmpcError, match="one at a time"):
            ctx.query_batch([dict(kind="map", map_id=mid, n=256, x=x, v=v)], map_params=dict(P_TINY, subvoxel=1.0))
        with pytest.raises(binding.RmpcError, match="dense"):
            ctx.edt(mid, (8, 8, 8))
        with pytest.raises(binding.RmpcError, match="far"):
            ctx.query(mid, np.array([1e6, 0.0, 0.0]), v, 256, P_TINY)
        # the ray policy itself is unchanged: zero velocity gives zero sums exactly
        q = ctx.query(mid, x, np.zeros(3), 1024, P_TINY)
        assert not np.any(q["S"]) and not np.any(q["f"]) and q["n_hit"] > 0
    finally:
        ctx.release(mid)


@pytest.fixture(scope="module")
def world():
    return W.sparse_world(20)


@pytest.mark.parametrize("lane_target", [10, 17, 19, 20])
def test_sparse_world_segments(ctx, world, lane_target):
    """The world at other segment counts per ray (1, 2, 8 and 16 lanes per ray at 65,536 rays;
    the default is 4): every ray and the query sums against the oracle."""
    from paper_2301_08068_amd import binding
    sm = world
    mid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    old = ctx.config(binding.CONFIG_SPARSE)
    dirs = oracle.directions(65536)
    try:
        ctx.config(binding.CONFIG_SPARSE, lane_target_log2=lane_target)
        x, v = W.sparse_free_state(sm, 702)
        x = sm.origin_m + np.round((x - sm.origin_m) / sm.voxel_m * 1024.0) / 1024.0 * sm.voxel_m
        g = ((x - sm.origin_m) / sm.voxel_m).astype(np.float32)
        reach = int(np.ceil(P_PAPER["max_range"] / sm.voxel_m)) + 16
        lo = (np.floor((g.astype(np.float64) - reach) / 8) * 8).astype(np.int64)
        hi = (np.ceil((g.astype(np.float64) + reach) / 8) * 8).astype(np.int64)
        dense, o_dense = sm.dense_crop(lo, hi)
        om = oracle.OracleMap(dense, sm.voxel_m, o_dense, "f32")
        t = ctx.trace(mid, x, 65536, P_PAPER)
        o = oracle.trace(om, _dense_start(sm, x, lo), dirs, P_PAPER["max_range"], nthreads=8)
        _compare(t, o, sm, lo, dense.shape[::-1], f"world lane target {lane_target}")
        q = ctx.query(mid, x, v, 65536, P_PAPER)
        oq = oracle.combine(P_PAPER, dirs, o["d"], o["hit"], v)
        oq["visits"] = int(o["visits"].sum())
        oq["n_tie"] = int(np.count_nonzero(o["flags"] & oracle.TIE))
        compare_query(q, oq, f"world query lane target {lane_target}")
    finally:
        ctx.config(binding.CONFIG_SPARSE, **old)
        ctx.release(mid)


def test_sparse_world_65536(ctx, world):
    """The outdoor-sized world of the sparse bench line (negative block coordinates, ~0.5 M
    blocks), 65,536 rays from two states with a 10 m range: every ray against the oracle on a
    dense crop that holds every voxel the rays can reach, and the query sums."""
    sm = world
    mid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    dirs = oracle.directions(65536)
    try:
        for seed in (700, 701):
            x, v = W.sparse_free_state(sm, seed)
            # moved by under 1e-3 voxel so that g is a multiple of 1/1024 (exact in both frames)
            x = sm.origin_m + np.round((x - sm.origin_m) / sm.voxel_m * 1024.0) / 1024.0 * sm.voxel_m
            g = ((x - sm.origin_m) / sm.voxel_m).astype(np.float32)
            reach = int(np.ceil(P_PAPER["max_range"] / sm.voxel_m)) + 16
            lo = (np.floor((g.astype(np.float64) - reach) / 8) * 8).astype(np.int64)
            hi = (np.ceil((g.astype(np.float64) + reach) / 8) * 8).astype(np.int64)
            dense, o_dense = sm.dense_crop(lo, hi)
            om = oracle.OracleMap(dense, sm.voxel_m, o_dense, "f32")
            t = ctx.trace(mid, x, 65536, P_PAPER)
            o = oracle.trace(om, _dense_start(sm, x, lo), dirs, P_PAPER["max_range"], nthreads=8)
            s, f = _compare(t, o, sm, lo, dense.shape[::-1], f"world state {seed}")
            q = ctx.query(mid, x, v, 65536, P_PAPER)
            oq = oracle.combine(P_PAPER, dirs, o["d"], o["hit"], v)
            oq["visits"] = int(o["visits"].sum())
            oq["n_tie"] = int(np.count_nonzero(o["flags"] & oracle.TIE))
            compare_query(q, oq, f"world query {seed}")
            print(f"world state {seed}: {s} rays identical, {f} flagged, {int((o['hit'] >= 0).sum())} hits")
    finally:
        ctx.release(mid)


def test_sparse_in_batches_serving_and_rollouts(ctx, tiny_map):
    """Sparse map queries inside batches (mixed with dense map queries and a scan), through the
    serving loop, and in batched rollouts: each result equals the same query or flight made
    alone with the same launch configuration, bit for bit (single sparse queries are checked
    against the oracle above)."""
    import time
    from paper_2301_08068_amd import binding as B
    shift = (-5, 3, 2)
    sm = W.sparse_from_dense(tiny_map, offset_blocks=shift, keep_free=0.2, seed=8)
    sid = ctx.upload_sparse(sm.coords, sm.values, sm.voxel_m, sm.origin_m, "f32", sm.trunc_m)
    did = ctx.upload(tiny_map.tsdf, tiny_map.voxel_m, tiny_map.origin_m, "f32")
    old_b, old_s = ctx.config(B.CONFIG_BATCH), ctx.config(B.CONFIG_SPARSE)
    lidar = W.params("lidar")
    try:
        bcfg = ctx.config(B.CONFIG_BATCH, use_graph=0)
        # a batch walks sparse maps with block rounds of 4 steps and the batch's segmentation
        ctx.config(B.CONFIG_SPARSE, lookahead=4, lane_target_log2=bcfg["lane_target_log2"])
        qs = []
        for k, seed in enumerate(range(300, 306)):
            x, v = _dyadic_state(tiny_map, sm, shift, seed)
            qs.append(dict(kind="map", map_id=sid, n=[256, 1024, 4096][k % 3], x=x, v=v))
            xd, vd = W.free_state(tiny_map, seed)
            qs.append(dict(kind="map", map_id=did, n=1024, x=xd, v=vd))
        xd, vd = W.free_state(tiny_map, 399)
        pts = torch.from_numpy(W.synth_scan(tiny_map, xd, 399, n_elev=16, n_azim=256)).cuda()
        qs.append(dict(kind="scan", points=pts, v=vd))
        res = ctx.query_batch(qs, map_params=P_TINY, scan_params=lidar)
        for q, r in zip(qs, res):
            alone = ctx.query_batch([q], map_params=P_TINY, scan_params=lidar)[0]
            assert np.array_equal(r["f"], alone["f"]) and np.array_equal(r["S"], alone["S"]), q
            if q["kind"] == "map" and q["map_id"] == sid:
                single = ctx.query(sid, q["x"], q["v"], q["n"], P_TINY)
                assert np.array_equal(r["f"], single["f"]) and np.array_equal(r["S"], single["S"])
                assert r["n_hit"] == single["n_hit"] and r["visits"] == single["visits"]
        # the serving loop: sparse requests among dense ones
        reqs = [B.request(dict(q)) for q in qs[:-1]]
        B.rmpc_server_start(ctx.ptr, n_slots=2, max_batch=4, map_params=P_TINY, scan_params=lidar, launch=bcfg,
                            staging_bytes=0)
        try:
            tks = [B.rmpc_submit(ctx.ptr, r) for r in reqs]
            got, t0 = {}, time.time()
            while len(got) < len(tks):
                for t, r, _ in B.rmpc_poll_completed(ctx.ptr, 64):
                    got[t] = r
                assert time.time() - t0 < 60.0
        finally:
            B.rmpc_server_stop(ctx.ptr)
        for t, r in zip(tks, res[:-1]):
            assert np.array_equal(got[t]["f"], r["f"]) and np.array_equal(got[t]["S"], r["S"])
        # batched flights on the sparse map equal single flights
        flights = []
        for k, seed in enumerate(range(310, 314)):
            x0, v0 = _dyadic_state(tiny_map, sm, shift, seed)
            goal, _ = _dyadic_state(tiny_map, sm, shift, seed + 50)
            flights.append(dict(map_id=sid, n_rays=[256, 1024][k % 2], x0=x0, v0=0.3 * v0, goal=goal, alpha=10.0,
                                beta=15.0, dt=0.001, max_steps=[150, 60][k % 2], goal_tol=0.1))
        out = ctx.rollout_batch(flights, P_TINY)
        for f, r in zip(flights, out):
            a = ctx.rollout(f["map_id"], f["x0"], f["v0"], f["n_rays"], P_TINY, f["goal"], f["alpha"], f["beta"],
                            f["dt"], f["max_steps"], f["goal_tol"])
            assert r["status"] == a["status"] and r["n_steps"] == a["n_steps"], (r, a)
            assert np.array_equal(r["x_final"], a["x_final"]) and np.array_equal(r["v_final"], a["v_final"])
    finally:
        ctx.config(B.CONFIG_BATCH, **old_b)
        ctx.config(B.CONFIG_SPARSE, **old_s)
        ctx.release(sid)
        ctx.release(did)


@pytest.mark.parametrize("enc", ["f32", "f16"])
def test_sparse_subvoxel_distances(ctx, tiny_map, enc):
    """Sub-voxel hit distances on a sparse map: per ray, the oracle's refinement (on the dense
    crop, whose voxels outside the stored blocks hold the same free value) of the oracle's walk
    distance for the same hit, to 1e-12 m; float32 and float16 values.  (Not bit for bit: the
    sample points g + t r are rounded in float64 in the sparse map's frame and in the crop's,
    whose coordinates differ by a whole number of blocks, so the samples can differ in their
    last bits; the walk's distances, computed from integer faces, stay bit-equal.)"""
    shift = (6, -4, 3)
    sm = W.sparse_from_dense(tiny_map, offset_blocks=shift, keep_free=0.3, seed=9)
    vals = sm.values if enc == "f32" else W.encode_f16(sm.values)
    # the free value as the storage type reads it back (exact in binary16 for the f16 map)
    fv = float(np.float32(sm.trunc_m)) if enc == "f32" else float(W.encode_f16(np.float32(sm.trunc_m)).view(np.float16))
    mid = ctx.upload_sparse(sm.coords, vals, sm.voxel_m, sm.origin_m, enc, fv)
    lo = (np.asarray(shift) - 7) * 8
    hi = (np.asarray(shift) + 8 + 7) * 8
    dense, o_dense = sm.dense_crop(lo, hi)
    dense_enc = dense if enc == "f32" else W.encode_f16(dense)
    om = oracle.OracleMap(dense_enc, sm.voxel_m, o_dense, enc)
    dirs = oracle.directions(1024)
    P_SUB = dict(P_TINY, subvoxel=1.0)
    moved = 0
    try:
        for seed in range(400, 412):
            x, v = _dyadic_state(tiny_map, sm, shift, seed)
            walk = ctx.trace(mid, x, 1024, P_TINY)
            ref = ctx.trace(mid, x, 1024, P_SUB)
            assert np.array_equal(walk["hit"], ref["hit"]) and np.array_equal(walk["flags"], ref["flags"])
            gd = _dense_start(sm, x, lo)
            o = oracle.trace(om, gd, dirs, P_TINY["max_range"])
            hits = _sparse_hits_as_lin(walk, sm, lo, dense.shape[::-1])
            for i in range(len(dirs)):
                if hits[i] < 0:
                    assert np.isinf(ref["d"][i])
                    continue
                if hits[i] == o["hit"][i]:
                    cands = [o["d"][i]]
                else:
                    cands = [o["alt_d"][i, j] for j in range(o["alt_n"][i]) if o["alt_hit"][i, j] == hits[i]]
                want = [oracle.subvoxel(om, gd, dirs[i], d) for d in cands]
                assert min(abs(ref["d"][i] - w) for w in want) <= 1e-12, (seed, i, ref["d"][i], want)
                moved += ref["d"][i] != walk["d"][i]
            # the query sums use the refined distances: the oracle's query on the dense crop
            q = ctx.query(mid, x, v, 1024, P_SUB)
            assert np.array_equal(oracle.grid_start(om, x), gd)
            compare_query(q, oracle.query(om, x, v, 1024, P_SUB, dirs=dirs), f"sparse subvoxel query {seed}")
    finally:
        ctx.release(mid)
    assert moved > 1000
