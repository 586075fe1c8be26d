"""Precision variants on the 400^3 paper-shaped map: the float32 TSDF, the sign-preserving
float16 TSDF and the uint8 occupancy give the same occupancy voxel for voxel, so the GPU walks,
hits and distances are identical across the three, and each result's error against the
float64 oracle comes from the float32 compensated sums alone.  Prints a per-result error table
(also written to the file named by RMPC_PRECISION_REPORT, when that is set)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2301_08068_amd import workloads as W  # noqa: E402
from gpu_common import compare_query, compare_trace  # noqa: E402

P = W.params("static", max_range=10.0)
SEEDS = (200, 201, 202, 203, 204, 205, 206, 207)


def _rel(a, b):
    s = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / s)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08068_amd import binding
    c = binding.Context(0, arena_bytes=1 << 30)
    yield c
    c.close()


def test_precision_report(ctx, paper_map):
    encs = {"f32": paper_map.tsdf, "f16": W.encode_f16(paper_map.tsdf), "u8": W.encode_u8(paper_map.tsdf)}
    mids = {e: ctx.upload(d, paper_map.voxel_m, paper_map.origin_m, e) for e, d in encs.items()}
    om = oracle.OracleMap.from_voxelmap(paper_map)
    dirs = oracle.directions(65536)
    lines = ["precision report: 400^3 paper-shaped map (seed 2), 65536 rays, max range 10 m",
             "error vs the float64 oracle; d: per-ray hit distance; S = sum A_i, b = sum A_i f_i, "
             "f = pinv(S) b (relative to the largest entry)",
             f"{'state':>6} {'enc':>4} {'hit_mismatch':>12} {'d_max_rel':>10} {'S_rel':>10} {'b_rel':>10} "
             f"{'f_rel':>10} {'rank':>4}"]
    worst, allv, n_ill, d_med = {}, {}, {}, {}
    try:
        for seed in SEEDS:
            x, v = W.free_state(paper_map, seed)
            o_tr = oracle.trace(om, oracle.grid_start(om, x), dirs, P["max_range"], nthreads=8)
            o_q = oracle.query(om, x, v, 65536, P, dirs=dirs, nthreads=8)
            res = {}
            for e, mid in mids.items():
                tr = ctx.trace(mid, x, 65536, P)
                compare_trace(tr, o_tr, f"{e} seed {seed}")
                q = ctx.query(mid, x, v, 65536, P)
                compare_query(q, o_q, f"{e} seed {seed}")
                res[e] = (tr, q)
                hs = (tr["hit"] >= 0) & (o_tr["hit"] >= 0)
                if hs.any():
                    rel = np.abs(tr["d"][hs] - o_tr["d"][hs]) / o_tr["d"][hs].clip(1e-300)
                    d_med[e] = max(d_med.get(e, 0.0), float(np.median(rel)))
                d_rel = float(np.max(np.abs(tr["d"][hs] - o_tr["d"][hs]) / o_tr["d"][hs].clip(1e-300))) \
                    if hs.any() else 0.0
                f_rel = float(np.linalg.norm(q["f"] - o_q["f"]) / max(np.linalg.norm(o_q["f"]), 1e-300))
                row = dict(mis=int(np.sum(tr["hit"] != o_tr["hit"])), d=d_rel, S=_rel(q["S"], o_q["S"]),
                           b=_rel(q["b"], o_q["b"]), f=f_rel)
                for k, val in row.items():
                    worst[(e, k)] = max(worst.get((e, k), 0), val)
                    allv.setdefault((e, k), []).append(val)
                n_ill[e] = n_ill.get(e, 0) + int((q["flags"] & oracle.Q_ILL) != 0)
                lines.append(f"{seed:>6} {e:>4} {row['mis']:>12d} {row['d']:>10.2e} {row['S']:>10.2e} "
                             f"{row['b']:>10.2e} {row['f']:>10.2e} {q['rank']:>4d}")
            # identical occupancy -> identical walks and bitwise identical results
            for e in ("f16", "u8"):
                assert np.array_equal(res[e][0]["hit"], res["f32"][0]["hit"])
                assert np.array_equal(res[e][0]["d"], res["f32"][0]["d"])
                for k in ("S", "b", "f"):
                    assert np.array_equal(res[e][1][k], res["f32"][1][k]), (e, k)
    finally:
        for mid in mids.values():
            ctx.release(mid)
    lines.append("worst: " + ", ".join(f"{e}.{k}={v:.2e}" for (e, k), v in sorted(worst.items())))
    lines.append("median: " + ", ".join(f"{e}.{k}={np.median(v):.2e}" for (e, k), v in sorted(allv.items())))
    lines.append("per-ray distance error, median over hit rays: "
                 + ", ".join(f"{e}={v:.2e}" for e, v in sorted(d_med.items())))
    lines.append("results flagged ILL: " + ", ".join(f"{e}={n}" for e, n in sorted(n_ill.items())))
    text = "\n".join(lines)
    print(text)
    report = os.environ.get("RMPC_PRECISION_REPORT")
    if report:
        with open(report, "w") as f:
            f.write(text + "\n")
    for e in encs:
        assert worst[(e, "mis")] == 0 and worst[(e, "d")] == 0.0


# float16 rounding of a stored value v with |v| <= 0.3 m (positives toward zero, negatives to
# nearest): at most one unit in the last place of [0.25, 0.5), 2^-12 m
F16_MAX_ERR_M = 2.0 ** -12


def _secant_gap(om, g, r, d, h):
    """For the oracle's refinement of walk distance d (metres) along r from grid start g: the
    field samples phi_k at t_k = max(t + k/2 - 3/2, 0) voxels (t = d / h); returns the jump
    phi_k - phi_k+1 at the first sign change and the smallest |phi_j| up to it (None: no sign
    change)."""
    t = d / h
    ts = [max(t + 0.5 * k - 1.5, 0.0) for k in range(8)]
    g64, r64 = np.asarray(g, np.float64), np.asarray(r, np.float64)
    phi = [oracle.field(om, g64 + tk * r64) for tk in ts]
    for k in range(7):
        if phi[k] > 0.0 >= phi[k + 1]:
            return phi[k] - phi[k + 1], min(abs(p) for p in phi[:k + 2])
    return None, min(abs(p) for p in phi)


def test_precision_subvoxel_f16_against_f32_oracle(ctx, paper_map):
    """Sub-voxel distances are where float16 storage changes results: the refined distance
    interpolates the stored values.  GPU results on the float16 map against the float64 oracle
    on the float32 map, per ray and per query.  A sample's float16 error is at most
    F16_MAX_ERR_M = E (trilinear weights are convex), so when no sample up to the sign change
    lies within E of zero the same sample pair is used and the crossing moves by at most
    (h/2) E / (phi_k - phi_k+1 - 2E); a ray with a sample within E of zero may take another
    pair and is bounded by the 3.5-voxel sample window instead."""
    h = paper_map.voxel_m
    Ps = dict(P, subvoxel=1.0)
    d16 = W.encode_f16(paper_map.tsdf)
    mid16 = ctx.upload(d16, h, paper_map.origin_m, "f16")
    mid32 = ctx.upload(paper_map.tsdf, h, paper_map.origin_m, "f32")
    om32 = oracle.OracleMap.from_voxelmap(paper_map)
    om16 = oracle.OracleMap(d16, h, paper_map.origin_m, "f16")
    dirs = oracle.directions(65536)
    E = F16_MAX_ERR_M
    lines = ["precision report, sub-voxel distances: float16 map on the GPU vs the float64 oracle on the "
             "float32 map (400^3 paper-shaped map, 65536 rays, max range 10 m)",
             f"{'state':>6} {'hits':>6} {'d_max_m':>10} {'d_med_m':>10} {'d_max_rel':>10} {'near0':>6} "
             f"{'S_rel':>10} {'b_rel':>10} {'f_rel':>10} {'f32gpu_S':>10}"]
    all_err, worst = [], {"S": 0.0, "b": 0.0, "f": 0.0, "d_rel": 0.0, "d": 0.0}
    n_ill = 0
    try:
        for seed in SEEDS:
            x, v = W.free_state(paper_map, seed)
            g = oracle.grid_start(om32, x)
            o_tr = oracle.trace(om32, g, dirs, P["max_range"], nthreads=8)
            tr16 = ctx.trace(mid16, x, 65536, Ps)
            hits = np.nonzero((o_tr["hit"] >= 0) & (tr16["hit"] == o_tr["hit"]))[0]
            assert np.array_equal(tr16["hit"], o_tr["hit"]) or \
                np.all((o_tr["flags"][tr16["hit"] != o_tr["hit"]] & oracle.TIE) != 0)
            err = np.empty(len(hits))
            n_near = 0
            for j, i in enumerate(hits):
                d32 = oracle.subvoxel(om32, g, dirs[i], o_tr["d"][i])
                err[j] = abs(tr16["d"][i] - d32)
                gap, near = _secant_gap(om32, g, dirs[i], o_tr["d"][i], h)
                if gap is None or near <= E:
                    n_near += 1
                    bound = 3.5 * h
                else:
                    # the same pair changes sign on both maps, and the secant fraction moves by
                    # |e_k+1 phi_k - e_k phi_k+1| / (gap (gap + e_k - e_k+1)) <= E / (gap - 2E)
                    bound = 0.5 * h * E / (gap - 2.0 * E) + 1e-12
                assert err[j] <= bound, (seed, i, err[j], bound, gap, near)
            q16 = ctx.query(mid16, x, v, 65536, Ps)
            q32 = ctx.query(mid32, x, v, 65536, Ps)
            o32 = oracle.query(om32, x, v, 65536, Ps, dirs=dirs, nthreads=8)
            o16 = oracle.query(om16, x, v, 65536, Ps, dirs=dirs, nthreads=8)
            n_ill += int((q16["flags"] & oracle.Q_ILL) != 0)
            row = {"S": _rel(q16["S"], o32["S"]), "b": _rel(q16["b"], o32["b"]),
                   "f": float(np.linalg.norm(q16["f"] - o32["f"]) / max(np.linalg.norm(o32["f"]), 1e-300))}
            # the GPU's own error on top of the storage's is the float32 summation's (<= 1e-4)
            assert row["S"] <= _rel(o16["S"], o32["S"]) + 1e-4
            assert row["b"] <= _rel(o16["b"], o32["b"]) + 1e-4
            drel = err / np.array([o_tr["d"][i] for i in hits]).clip(1e-300)
            for k in ("S", "b", "f"):
                worst[k] = max(worst[k], row[k])
            worst["d"] = max(worst["d"], float(err.max()))
            worst["d_rel"] = max(worst["d_rel"], float(drel.max()))
            all_err.append(err)
            lines.append(f"{seed:>6} {len(hits):>6d} {err.max():>10.2e} {np.median(err):>10.2e} "
                         f"{drel.max():>10.2e} {n_near:>6d} {row['S']:>10.2e} {row['b']:>10.2e} "
                         f"{row['f']:>10.2e} {_rel(q32['S'], o32['S']):>10.2e}")
    finally:
        ctx.release(mid16)
        ctx.release(mid32)
    e = np.concatenate(all_err)
    lines.append(f"all states: per-ray distance error max {e.max():.3e} m, median {np.median(e):.3e} m, "
                 f"99th percentile {np.percentile(e, 99):.3e} m, zero on {np.mean(e == 0):.1%} of hits; "
                 f"worst relative d {worst['d_rel']:.2e}; worst S {worst['S']:.2e}, b {worst['b']:.2e}, "
                 f"f {worst['f']:.2e}; results flagged ILL: {n_ill}")
    lines.append("uint8 occupancy stores no field: sub-voxel distances are refused on it")
    text = "\n".join(lines)
    print(text)
    report = os.environ.get("RMPC_PRECISION_REPORT")
    if report:
        with open(report, "a") as f:
            f.write(text + "\n")
    assert e.max() > 0.0       # float16 storage does change sub-voxel distances
