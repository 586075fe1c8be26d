"""The allocation-free scan query (rmpc_scan_query_noalloc) through the C ABI: two calls in a
row, the second on a smaller frame, each bit-equal to rmpc_scan_query on the same points and
within the oracle's tolerance; the first call runs before any context exists."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2301_08068_amd import workloads as W  # noqa: E402


def _noalloc(binding, pts, v, params):
    out = torch.zeros(binding.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream(0)
    binding.rmpc_scan_query_noalloc(0, pts.data_ptr(), pts.shape[0], v, params, out.data_ptr(),
                                    stream=stream.cuda_stream)
    stream.synchronize()
    return binding.result_from_bytes(out.cpu().numpy().tobytes())


def _same(a, b):
    for k in ("f", "S", "b", "lam"):
        assert np.array_equal(a[k], b[k]), (k, a[k], b[k])
    for k in ("rank", "n_hit", "n_contrib", "n_tie", "flags", "n_rays", "visits"):
        assert a[k] == b[k], (k, a[k], b[k])


def test_noalloc_scan_equals_scan_query(tiny_map, paper_map):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08068_amd import binding
    L = W.params("lidar")
    x1, v1 = W.free_state(paper_map, 611)
    big = W.synth_scan(paper_map, x1, 611, n_elev=128, n_azim=2048, fov_deg=90.0)      # 262,144 points
    x2, v2 = W.free_state(tiny_map, 612)
    small = W.synth_scan(tiny_map, x2, 612, n_elev=16, n_azim=250)                      # 4,000 points
    cases = [(big, v1), (small, v2)]
    dev = [torch.from_numpy(p).to("cuda:0") for p, _ in cases]
    print(f"noalloc: {[p.shape[0] for p, _ in cases]} points", flush=True)
    got = [_noalloc(binding, d, v, L) for d, (_, v) in zip(dev, cases)]   # before any context
    ctx = binding.Context(0, arena_bytes=64 << 20)
    try:
        for d, (p, v), g in zip(dev, cases, got):
            ref = ctx.scan_query(d, v, L)
            _same(g, ref)
            o = oracle.scan(p, v, L)
            scale = max(np.abs(o["S"]).max(), 1e-300)
            assert np.max(np.abs(g["S"] - o["S"])) <= 1e-4 * scale
            assert g["n_hit"] == o["n_hit"] and g["n_contrib"] == o["n_contrib"]
        # again, in the other order (the fixed scratch keeps the previous call's contents)
        again = _noalloc(binding, dev[1], cases[1][1], L)
        _same(again, got[1])
        # an empty frame: zero sums, nothing hit
        empty = torch.zeros((0, 3), dtype=torch.float32, device="cuda:0")
        e = _noalloc(binding, empty, v1, L)
        assert e["n_hit"] == 0 and not np.any(e["S"]) and not np.any(e["f"])
    finally:
        ctx.close()


def test_noalloc_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08068_amd import binding
    L = W.params("lidar")
    pts = torch.zeros((4, 3), dtype=torch.float32, device="cuda:0")
    out = torch.zeros(binding.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(binding.RmpcError, match="n_points"):
        binding.rmpc_scan_query_noalloc(0, pts.data_ptr(), (1 << 24) + 1, np.zeros(3), L, out.data_ptr())
    with pytest.raises(binding.RmpcError, match="out_dev"):
        binding.rmpc_scan_query_noalloc(0, pts.data_ptr(), 4, np.zeros(3), L, 0)
    with pytest.raises(binding.RmpcError, match="device"):
        binding.rmpc_scan_query_noalloc(99, pts.data_ptr(), 4, np.zeros(3), L, out.data_ptr())
