"""GPU exact distance transform (rmpc_edt) against the oracle's: every voxel bit for bit on the
tiny map in all three encodings and on ragged random grids; sampled voxels of the 400^3 map
against brute force over all its occupied voxels; empty and full grids."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2301_08068_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08068_amd import binding
    c = binding.Context(0, arena_bytes=1 << 30)
    yield c
    c.close()


def _gpu_edt(ctx, data, h, enc):
    mid = ctx.upload(data, h, np.zeros(3), enc)
    try:
        return ctx.edt(mid, data.shape).cpu().numpy()
    finally:
        ctx.release(mid)


@pytest.mark.parametrize("enc", ["f32", "f16", "u8"])
def test_tiny_map_bitwise(ctx, tiny_map, enc):
    data = {"f32": tiny_map.tsdf, "f16": W.encode_f16(tiny_map.tsdf), "u8": W.encode_u8(tiny_map.tsdf)}[enc]
    g = _gpu_edt(ctx, data, tiny_map.voxel_m, enc)
    o = oracle.edt(oracle.OracleMap(data, tiny_map.voxel_m, tiny_map.origin_m, enc))
    assert np.array_equal(g, o)


# line groups of the y and z passes: 64 lines of 23 (one partial group), 32 of 300, 16 of 1,000
# with a ragged last group (37 = 2 x 16 + 5), and single-element lines
@pytest.mark.parametrize("shape,p", [((37, 23, 51), 0.002), ((5, 300, 7), 0.01), ((64, 1, 130), 0.05),
                                     ((3, 1000, 37), 0.003), ((1000, 2, 70), 0.002)])
def test_ragged_random_grids(ctx, shape, p):
    rng = np.random.default_rng(sum(shape))
    occ = rng.uniform(size=shape) < p
    occ[0, 0, 0] = True
    t = np.where(occ, -0.05, 0.3).astype(np.float32)
    g = _gpu_edt(ctx, t, 0.1, "f32")
    assert np.array_equal(g, oracle.edt(oracle.OracleMap(t, 0.1, np.zeros(3), "f32")))


def test_longest_lines(ctx):
    """y and z lines of 4,096 voxels (the largest extent a map may have): two lines per group of
    the y and z passes; every voxel against the oracle."""
    rng = np.random.default_rng(7)
    for shape in ((1, 4096, 3), (4096, 1, 3)):
        t = np.where(rng.uniform(size=shape) < 0.001, -0.05, 0.3).astype(np.float32)
        t.reshape(-1)[1234] = -0.05
        g = _gpu_edt(ctx, t, 0.1, "f32")
        assert np.array_equal(g, oracle.edt(oracle.OracleMap(t, 0.1, np.zeros(3), "f32"))), shape


def test_empty_and_full(ctx):
    free = np.full((9, 10, 11), 0.3, np.float32)
    assert np.all(_gpu_edt(ctx, free, 0.1, "f32") == -1)
    assert np.all(_gpu_edt(ctx, -free, 0.1, "f32") == 0)


def test_paper_map_sampled(ctx, paper_map):
    g = _gpu_edt(ctx, paper_map.tsdf, paper_map.voxel_m, "f32")
    occ = paper_map.tsdf <= 0
    assert np.all(g[occ] == 0) and np.all(g[~occ] > 0)
    pts = np.argwhere(occ).astype(np.int64)               # (k, j, i)
    rng = np.random.default_rng(12)
    for _ in range(48):
        k, j, i = (int(v) for v in rng.integers(0, 400, size=3))
        best = int(np.min((pts[:, 0] - k) ** 2 + (pts[:, 1] - j) ** 2 + (pts[:, 2] - i) ** 2))
        assert g[k, j, i] == best, (k, j, i)


def test_esdf_policy_matches_oracle(ctx, tiny_map):
    """The single-lookup ESDF policy at many states of the tiny map: counts and flags exact,
    sums and the resolved acceleration to 1e-9 of their size (float64 on both sides; only the
    exp and log1p of the policy round differently)."""
    from paper_2301_08068_amd import binding as B
    mid = ctx.upload(tiny_map.tsdf, tiny_map.voxel_m, tiny_map.origin_m, "f32")
    om = oracle.OracleMap.from_voxelmap(tiny_map)
    p = W.params("static")
    try:
        sq = ctx.edt(mid, tiny_map.tsdf.shape)
        osq = oracle.edt(om)
        n_contrib = 0
        for seed in range(900, 1000):
            x, v = W.free_state(tiny_map, seed)
            g = ctx.esdf_query(mid, sq, x, v, p)
            o = oracle.esdf_query(om, osq, x, v, p)
            for k in ("n_hit", "n_contrib", "flags", "rank"):
                assert g[k] == o[k], (seed, k, g[k], o[k])
            for k in ("S", "b", "f"):
                scale = max(np.abs(o[k]).max(), 1e-300)
                assert np.abs(g[k] - o[k]).max() <= 1e-9 * scale, (seed, k, g[k], o[k])
            n_contrib += o["n_contrib"]
        assert n_contrib > 20
        with pytest.raises(B.RmpcError) as e:
            ctx.esdf_query(mid, sq, [-1.0, 0.5, 0.5], [0, 0, 0], p)
        assert e.value.status == B.RMPC_E_OUT_OF_BOUNDS
    finally:
        ctx.release(mid)
