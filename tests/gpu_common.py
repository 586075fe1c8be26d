"""Helpers shared by the GPU parity tests: comparison of library results with the oracle."""
import numpy as np

import oracle


def compare_trace(gpu, orc, label=""):
    """Per-ray parity: hit voxel bit-exact (flagged rays: inside the admissible set), the
    float64 distance bit-exact for equal hits, visit counts and flags exact except TIE, which
    the GPU may leave off where the oracle sets it."""
    hit_g, hit_o = gpu["hit"].astype(np.int64), orc["hit"].astype(np.int64)
    flagged = (orc["flags"] & (oracle.TIE | oracle.RANGE_TIE)) != 0
    same = hit_g == hit_o
    bad = ~same & ~flagged
    assert not bad.any(), f"{label}: {bad.sum()} unflagged rays hit another voxel, e.g. ray {np.argmax(bad)}"
    for i in np.nonzero(~same)[0]:
        alts = orc["alt_hit"][i, :orc["alt_n"][i]]
        assert hit_g[i] in alts, f"{label}: flagged ray {i} hit {hit_g[i]} not admissible {alts}"
    hs = same & (hit_o >= 0)
    assert np.array_equal(gpu["d"][hs], orc["d"][hs]), f"{label}: distances differ"
    assert np.all(np.isinf(gpu["d"][same & (hit_o < 0)]))
    # every flag but TIE is exact; the walk skips free cells whole and reports the near-ties of
    # the decisions it takes, a subset of the oracle's
    gf, of = gpu["flags"][same].astype(np.uint32), orc["flags"][same].astype(np.uint32)
    assert np.array_equal(gf & ~np.uint32(oracle.TIE), of & ~np.uint32(oracle.TIE)), f"{label}: flags differ"
    assert not np.any(gf & ~of & oracle.TIE), f"{label}: TIE flag on a ray the oracle does not flag"
    assert np.array_equal(gpu["visits"][same], orc["visits"][same]), f"{label}: visits differ"
    return int(same.sum()), int(flagged.sum())


def compare_query(g, o, label="", rtol=1e-4, ties="subset"):
    """Query parity: sums within rtol of their largest entry, f within rtol unless ILL, counts
    exact.  ties="subset": o is the oracle, whose near-ties include the GPU's; "ignore": two
    GPU results whose launches may differ in lookahead (the ties a walk sees depend on it)."""
    sS = max(np.abs(o["S"]).max(), 1e-300)
    sb = max(np.abs(o["b"]).max(), 1e-300)
    assert np.max(np.abs(g["S"] - o["S"])) <= rtol * sS, f"{label}: S {g['S']} vs {o['S']}"
    assert np.max(np.abs(g["b"] - o["b"])) <= rtol * sb, f"{label}: b {g['b']} vs {o['b']}"
    ill = (g["flags"] | o["flags"]) & oracle.Q_ILL
    if not ill and np.linalg.norm(o["f"]) > 0:
        err = np.linalg.norm(g["f"] - o["f"]) / np.linalg.norm(o["f"])
        assert err <= rtol, f"{label}: f {g['f']} vs {o['f']} (rel {err:.2e})"
        assert g["rank"] == o["rank"], label
    else:
        # graded by the invariant only: S f = b within the tolerance
        S = g["S"]
        if np.linalg.norm(g["b"]) > 0:
            assert np.linalg.norm(S @ g["f"] - g["b"]) <= rtol * np.linalg.norm(g["b"]) * 10, label
    for k in ("n_hit", "n_contrib", "visits"):
        assert g[k] == o[k], f"{label}: {k} {g[k]} vs {o[k]}"
    if ties == "subset":
        assert g["n_tie"] <= o["n_tie"], f"{label}: n_tie {g['n_tie']} vs {o['n_tie']}"
