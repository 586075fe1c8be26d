"""GPU tests of the serving loop: requests of every kind submitted while earlier ones run get
exactly the result rmpc_query_batch gives each alone with the same launch configuration
(results of one request do not depend on which others share its launch), scans staged from
pinned host memory match scans read from device memory, poll and stop follow their contract,
and the counters add up."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2301_08068_amd import workloads as W  # noqa: E402
from gpu_common import compare_query  # noqa: E402
import oracle  # noqa: E402

P = W.params("static", max_range=10.0)
L = W.params("lidar")


@pytest.fixture(scope="module")
def env(paper_map):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08068_amd import binding as B
    ctx = B.Context(0, arena_bytes=1 << 30)
    maps = {
        "f32": ctx.upload(paper_map.tsdf, paper_map.voxel_m, paper_map.origin_m, "f32"),
        "f16": ctx.upload(W.encode_f16(paper_map.tsdf), paper_map.voxel_m, paper_map.origin_m, "f16"),
        "u8": ctx.upload(W.encode_u8(paper_map.tsdf), paper_map.voxel_m, paper_map.origin_m, "u8"),
    }
    yield ctx, maps
    ctx.close()


def _requests(paper_map, maps, n=60, seed=21):
    """Mixed requests: map queries on the three encodings with uneven ray counts, scans from
    device memory and scans from pinned host memory."""
    from paper_2301_08068_amd import binding as B
    rng = np.random.default_rng(seed)
    counts = W.ray_counts(n, seed=seed, lo=64, hi=65536)
    out = []
    for k in range(n):
        x, v = W.free_state(paper_map, 700 + k)
        kind = k % 4
        if kind < 2:
            key = ["f32", "f16", "u8"][int(rng.integers(0, 3))]
            q = dict(kind="map", map_id=maps[key], n=int(counts[k]), x=x, v=v)
            out.append(dict(q=q, req=B.request(q), host=None, dev=None))
        else:
            pts = W.synth_scan(paper_map, x, 700 + k, n_elev=16, n_azim=256)
            dev = torch.from_numpy(pts).cuda()
            q = dict(kind="scan", n=pts.shape[0], v=v, points_ptr=dev.data_ptr())
            if kind == 2:
                out.append(dict(q=q, req=B.request(q), host=None, dev=dev))
            else:
                host = torch.from_numpy(pts).pin_memory()
                out.append(dict(q=q, req=B.request(dict(q, points_ptr=0), host.data_ptr()), host=host, dev=dev))
    torch.cuda.synchronize()
    return out


def _drain(B, ctx, n, timeout_s=60.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for t, r, lat in B.rmpc_poll_completed(ctx.ptr, 64):
            got[t] = (r, lat)
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {n} results"
    return got


def test_served_equals_batch_alone(env, paper_map):
    from paper_2301_08068_amd import binding as B
    ctx, maps = env
    launch = ctx.config(B.CONFIG_BATCH, use_graph=0)
    reqs = _requests(paper_map, maps)
    B.rmpc_server_start(ctx.ptr, n_slots=3, max_batch=8, map_params=P, scan_params=L, launch=launch,
                        staging_bytes=1 << 20)
    try:
        tickets = []
        for i, r in enumerate(reqs):
            tickets.append(B.rmpc_submit(ctx.ptr, r["req"]))
            if i % 7 == 3:
                time.sleep(2e-4)            # let some launches start before the next arrivals
        assert tickets == sorted(tickets) and len(set(tickets)) == len(tickets)
        got = _drain(B, ctx, len(reqs))
        st = B.rmpc_server_stats(ctx.ptr)
    finally:
        B.rmpc_server_stop(ctx.ptr)
    assert st["submitted"] == st["completed"] == len(reqs) and st["pending"] == st["in_flight"] == 0
    assert 1 <= st["batch_max"] <= 8 and st["launches"] >= (len(reqs) + 7) // 8
    assert st["staging_peak"] <= 1 << 20
    for t, r in zip(tickets, reqs):
        res, lat = got[t]
        assert lat > 0
        q = r["q"]
        alone = ctx.query_batch([q], map_params=P if q["kind"] == "map" else None,
                                scan_params=L if q["kind"] == "scan" else None)[0]
        for k in ("S", "b", "f", "lam"):
            assert np.array_equal(res[k], alone[k]), (k, q["kind"], q["n"])
        for k in ("rank", "n_hit", "n_contrib", "n_tie", "flags", "visits", "n_rays"):
            assert res[k] == alone[k], k


def test_served_matches_oracle(env, paper_map):
    from paper_2301_08068_amd import binding as B
    ctx, maps = env
    reqs = _requests(paper_map, maps, n=12, seed=5)
    B.rmpc_server_start(ctx.ptr, n_slots=2, max_batch=4, map_params=P, scan_params=L,
                        launch=ctx.config(B.CONFIG_BATCH), staging_bytes=1 << 20)
    try:
        tickets = [B.rmpc_submit(ctx.ptr, r["req"]) for r in reqs]
        got = _drain(B, ctx, len(reqs))
    finally:
        B.rmpc_server_stop(ctx.ptr)
    enc = {maps["f32"]: paper_map.tsdf, maps["f16"]: W.encode_f16(paper_map.tsdf),
           maps["u8"]: W.encode_u8(paper_map.tsdf)}
    names = {maps["f32"]: "f32", maps["f16"]: "f16", maps["u8"]: "u8"}
    for t, r in zip(tickets, reqs):
        q = r["q"]
        if q["kind"] == "map":
            om = oracle.OracleMap(enc[q["map_id"]], paper_map.voxel_m, paper_map.origin_m, names[q["map_id"]])
            o = oracle.query(om, q["x"], q["v"], q["n"], P, nthreads=8)
        else:
            o = oracle.scan(r["dev"].cpu().numpy(), q["v"], L)
        compare_query(got[t][0], o, "served vs oracle")


def test_poll_contract_and_refusals(env, paper_map):
    from paper_2301_08068_amd import binding as B
    ctx, maps = env
    x, v = W.free_state(paper_map, 1)
    q = dict(kind="map", map_id=maps["u8"], n=4096, x=x, v=v)
    with pytest.raises(B.RmpcError) as e:
        B.rmpc_submit(ctx.ptr, B.request(q))
    assert e.value.status == B.RMPC_E_STOPPED
    B.rmpc_server_start(ctx.ptr, n_slots=1, max_batch=2, map_params=P, scan_params=L,
                        launch=ctx.config(B.CONFIG_BATCH), staging_bytes=0, max_pending=4)
    try:
        # invalid requests are refused at submission and nothing is queued
        for bad, status in ((dict(q, n=0), B.RMPC_E_INVALID), (dict(q, x=[-5.0, 0, 0]), B.RMPC_E_OUT_OF_BOUNDS),
                            (dict(q, map_id=77), B.RMPC_E_NOMAP)):
            with pytest.raises(B.RmpcError) as e:
                B.rmpc_submit(ctx.ptr, B.request(bad))
            assert e.value.status == status
        host = torch.zeros((10, 3), dtype=torch.float32).pin_memory()
        with pytest.raises(B.RmpcError) as e:     # host scan without staging memory
            B.rmpc_submit(ctx.ptr, B.request(dict(kind="scan", n=10, v=v), host.data_ptr()))
        assert e.value.status == B.RMPC_E_NOMEM
        with pytest.raises(B.RmpcError):
            B.rmpc_poll(ctx.ptr, 12345)
        # maps cannot change while the server runs
        with pytest.raises(B.RmpcError):
            ctx.release(maps["u8"])
        # a full queue refuses, and the refusals are counted
        accepted, refused = [], 0
        for _ in range(64):
            try:
                accepted.append(B.rmpc_submit(ctx.ptr, B.request(q)))
            except B.RmpcError as err:
                assert err.status == B.RMPC_E_NOMEM
                refused += 1
        assert B.rmpc_server_stats(ctx.ptr)["refused"] == refused
        # poll by ticket: not ready or ready; a retired ticket is unknown
        results = {}
        t0 = time.time()
        while len(results) < len(accepted):
            for t in accepted:
                if t not in results:
                    r, lat = B.rmpc_poll(ctx.ptr, t)
                    if r is not None:
                        results[t] = r
            assert time.time() - t0 < 60
        with pytest.raises(B.RmpcError) as e:
            B.rmpc_poll(ctx.ptr, accepted[0])
        assert e.value.status == B.RMPC_E_INVALID
        ref = ctx.query_batch([q], map_params=P)[0]
        for r in results.values():
            assert np.array_equal(r["f"], ref["f"]) and np.array_equal(r["S"], ref["S"])
        assert B.rmpc_poll_completed(ctx.ptr, 16) == []          # all retired by rmpc_poll
    finally:
        B.rmpc_server_stop(ctx.ptr)
    with pytest.raises(B.RmpcError) as e:
        B.rmpc_server_stop(ctx.ptr)
    assert e.value.status == B.RMPC_E_STOPPED


def test_stop_finishes_queued_work(env, paper_map):
    from paper_2301_08068_amd import binding as B
    ctx, maps = env
    B.rmpc_server_start(ctx.ptr, n_slots=2, max_batch=16, map_params=P, scan_params=L,
                        launch=ctx.config(B.CONFIG_BATCH))
    xs = [W.free_state(paper_map, 40 + k) for k in range(40)]
    for x, v in xs:
        B.rmpc_submit(ctx.ptr, B.request(dict(kind="map", map_id=maps["f16"], n=65536, x=x, v=v)))
    B.rmpc_server_stop(ctx.ptr)                  # returns after every queued request ran
    # the context is usable afterwards, and a new server starts cleanly
    B.rmpc_server_start(ctx.ptr, n_slots=1, max_batch=1, map_params=P, scan_params=L,
                        launch=ctx.config(B.CONFIG_BATCH))
    t = B.rmpc_submit(ctx.ptr, B.request(dict(kind="map", map_id=maps["f16"], n=100, x=xs[0][0], v=xs[0][1])))
    got = _drain(B, ctx, 1)
    B.rmpc_server_stop(ctx.ptr)
    assert t in got


@pytest.mark.parametrize("use_graph", [0, 1])
def test_one_tile_slots(env, paper_map, use_graph):
    """A server whose launches hold a single 256-lane tile starts (its warm-up stays inside the
    slots' buffers), serves a request that fits one tile bit-equal to the same query alone,
    refuses one that does not, and stops cleanly."""
    from paper_2301_08068_amd import binding as B
    ctx, maps = env
    x, v = W.free_state(paper_map, 3)
    q = dict(kind="map", map_id=maps["f32"], n=16, x=x, v=v)
    launch = dict(ctx.config(B.CONFIG_BATCH), use_graph=use_graph)
    B.rmpc_server_start(ctx.ptr, n_slots=2, max_batch=1, max_tiles=1, map_params=P, scan_params=L,
                        launch=launch, staging_bytes=1 << 16)
    try:
        with pytest.raises(B.RmpcError) as e:
            B.rmpc_submit(ctx.ptr, B.request(dict(q, n=4096)))
        assert e.value.status == B.RMPC_E_INVALID
        t = B.rmpc_submit(ctx.ptr, B.request(q))
        got = _drain(B, ctx, 1)
    finally:
        B.rmpc_server_stop(ctx.ptr)
    alone = ctx.query_batch([q], map_params=P)[0]
    res = got[t][0]
    for k in ("S", "b", "f", "lam"):
        assert np.array_equal(res[k], alone[k]), k
    for k in ("rank", "n_hit", "n_contrib", "n_tie", "flags", "visits", "n_rays"):
        assert res[k] == alone[k], k
