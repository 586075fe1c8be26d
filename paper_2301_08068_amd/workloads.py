"""Seeded synthetic workloads: voxel maps, robot states, trajectories, LiDAR scans, arrivals.

This module produces *inputs* only.  It holds none of the method's arithmetic (no Halton
directions, no voxel traversal, no motion-policy terms, no resolve): both the CPU oracle and
the GPU library consume what it generates.  Everything is driven by numpy's PCG64
``default_rng`` so a seed fully determines an input.

Map recipe (after the random-primitive maps of Sec. IV-A: spheres and boxes merged by a
boolean union, up to 200 obstacles): the stored value at each voxel centre
``origin + (idx + 1/2) h`` is ``clamp(min_k sdf_k(centre), -T, T)`` computed in float64 from
textbook signed distance functions of spheres, axis-aligned boxes, half-spaces and slabs,
then stored as float32.  A voxel is occupied when that value is <= 0.  Each primitive only
updates voxels within ``T`` of its bounding box, which is exact because the clamp commutes
with the min.

Arrays are laid out x-fastest: ``tsdf[k, j, i]`` is voxel ``lin = i + nx*(j + ny*k)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------------------
# primitives and their signed distance functions (inputs geometry only)
# ----------------------------------------------------------------------------------------

Primitive = Tuple  # ("sphere", cx, cy, cz, R) | ("box", cx, cy, cz, ex, ey, ez) (half extents)
#                    | ("halfspace_below", axis, level)  solid where p[axis] < level
#                    | ("slab", axis, lo, hi)            solid where lo < p[axis] < hi


def _sdf(prim: Primitive, p: np.ndarray) -> np.ndarray:
    """Signed distance of points ``p`` (..., 3) to one primitive, negative inside."""
    kind = prim[0]
    if kind == "sphere":
        c = np.asarray(prim[1:4], dtype=np.float64)
        return np.linalg.norm(p - c, axis=-1) - prim[4]
    if kind == "box":
        c = np.asarray(prim[1:4], dtype=np.float64)
        e = np.asarray(prim[4:7], dtype=np.float64)
        q = np.abs(p - c) - e
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        inside = np.minimum(np.max(q, axis=-1), 0.0)
        return outside + inside
    if kind == "halfspace_below":
        axis, level = prim[1], prim[2]
        return p[..., axis] - level
    if kind == "slab":
        axis, lo, hi = prim[1], prim[2], prim[3]
        mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        return np.abs(p[..., axis] - mid) - half
    raise ValueError(kind)


def _bbox(prim: Primitive, extent: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """World-space axis-aligned bounds of the solid part of a primitive (clipped to extent)."""
    kind = prim[0]
    lo = np.zeros(3)
    hi = extent.copy()
    if kind == "sphere":
        c = np.asarray(prim[1:4]); r = prim[4]
        return c - r, c + r
    if kind == "box":
        c = np.asarray(prim[1:4]); e = np.asarray(prim[4:7])
        return c - e, c + e
    if kind == "halfspace_below":
        hi = hi.copy(); hi[prim[1]] = prim[2]
        lo = lo - 1e9 * (np.arange(3) == prim[1])
        return lo, hi
    if kind == "slab":
        lo = lo.copy(); hi = hi.copy()
        lo[prim[1]] = prim[2]; hi[prim[1]] = prim[3]
        return lo, hi
    raise ValueError(kind)


def sdf_union(prims: Sequence[Primitive], p: np.ndarray) -> np.ndarray:
    """Analytic signed distance of the union of primitives at points ``p`` (..., 3)."""
    p = np.asarray(p, dtype=np.float64)
    out = np.full(p.shape[:-1], np.inf)
    for prim in prims:
        out = np.minimum(out, _sdf(prim, p))
    return out


@dataclasses.dataclass
class VoxelMap:
    """A synthetic map: float32 TSDF on a dense grid plus the primitives that built it."""

    name: str
    tsdf: np.ndarray          # float32 [nz, ny, nx], x fastest
    voxel_m: float
    origin_m: np.ndarray      # world coordinate of the grid's min corner
    prims: List[Primitive]
    trunc_m: float

    @property
    def dims(self) -> Tuple[int, int, int]:
        nz, ny, nx = self.tsdf.shape
        return nx, ny, nz

    @property
    def extent_m(self) -> np.ndarray:
        return np.asarray(self.dims, dtype=np.float64) * self.voxel_m

    def occupied_fraction(self) -> float:
        return float(np.count_nonzero(self.tsdf <= 0)) / self.tsdf.size


def build_tsdf(dims: Tuple[int, int, int], voxel_m: float, origin_m, prims: Sequence[Primitive],
               trunc_m: float) -> np.ndarray:
    """Truncated signed distance at voxel centres, float64 math, stored float32 [nz, ny, nx]."""
    nx, ny, nz = dims
    origin = np.asarray(origin_m, dtype=np.float64)
    extent = np.asarray(dims, dtype=np.float64) * voxel_m
    out = np.full((nz, ny, nx), trunc_m, dtype=np.float64)
    n = np.array([nx, ny, nz])
    for prim in prims:
        lo_w, hi_w = _bbox(prim, extent)
        lo_w = np.asarray(lo_w, dtype=np.float64) - trunc_m
        hi_w = np.asarray(hi_w, dtype=np.float64) + trunc_m
        # voxel index range whose centres may lie within trunc of the bbox
        lo_i = np.clip(np.floor((lo_w - origin) / voxel_m - 0.5).astype(np.int64), 0, n)
        hi_i = np.clip(np.ceil((hi_w - origin) / voxel_m - 0.5).astype(np.int64) + 1, 0, n)
        if np.any(hi_i <= lo_i):
            continue
        xs = origin[0] + (np.arange(lo_i[0], hi_i[0]) + 0.5) * voxel_m
        ys = origin[1] + (np.arange(lo_i[1], hi_i[1]) + 0.5) * voxel_m
        zs = origin[2] + (np.arange(lo_i[2], hi_i[2]) + 0.5) * voxel_m
        # process slab by slab along z to bound temporary memory
        for kk in range(0, len(zs), 16):
            zc = zs[kk:kk + 16]
            P = np.stack(np.meshgrid(xs, ys, zc, indexing="ij"), axis=-1)  # [x, y, z, 3]
            d = np.clip(_sdf(prim, P), -trunc_m, trunc_m).transpose(2, 1, 0)  # -> [z, y, x]
            sl = (slice(lo_i[2] + kk, lo_i[2] + kk + len(zc)),
                  slice(lo_i[1], hi_i[1]), slice(lo_i[0], hi_i[0]))
            np.minimum(out[sl], d, out=out[sl])
    return out.astype(np.float32)


# ----------------------------------------------------------------------------------------
# the map configurations
# ----------------------------------------------------------------------------------------

def tiny_map(seed: int = 1) -> VoxelMap:
    """64^3 grid, 0.1 m voxels (6.4 m cube), float32 TSDF truncated at 0.3 m.

    20 spheres (centres uniform in the cube, radius U[0.2, 1.0] m) plus a ground
    half-space z < 0.3 m whose plane lies exactly on a voxel face (z = 3 h).
    """
    rng = np.random.default_rng(seed)
    h, dims = 0.1, (64, 64, 64)
    prims: List[Primitive] = [("halfspace_below", 2, 0.3)]
    for _ in range(20):
        c = rng.uniform(0.0, 6.4, size=3)
        r = rng.uniform(0.2, 1.0)
        prims.append(("sphere", float(c[0]), float(c[1]), float(c[2]), float(r)))
    tsdf = build_tsdf(dims, h, (0.0, 0.0, 0.0), prims, 0.3)
    return VoxelMap("tiny64", tsdf, h, np.zeros(3), prims, 0.3)


def _random_obstacles(rng, n: int, lo: float, hi: float, size_scale: float = 1.0) -> List[Primitive]:
    prims: List[Primitive] = []
    for _ in range(n):
        c = rng.uniform(lo, hi, size=3)
        if rng.uniform() < 0.5:
            r = rng.uniform(0.15, 1.0) * size_scale
            prims.append(("sphere", float(c[0]), float(c[1]), float(c[2]), float(r)))
        else:
            side = rng.uniform(0.3, 2.0, size=3) * size_scale
            prims.append(("box", float(c[0]), float(c[1]), float(c[2]),
                          float(side[0] / 2), float(side[1] / 2), float(side[2] / 2)))
    return prims


def _walls(extent: float, thick: float) -> List[Primitive]:
    return [("slab", a, 0.0, thick) for a in range(3)] + \
           [("slab", a, extent - thick, extent) for a in range(3)]


def paper_map(seed: int = 2, n_cells: int = 400, voxel_m: float = 0.05,
              n_prims: int = 200) -> VoxelMap:
    """Paper-shaped map: 400^3 grid of 0.05 m voxels (20 m cube), float32 TSDF (T = 0.3 m).

    Six 0.25 m walls on the cube faces plus ``n_prims`` obstacles; a fair coin picks a
    sphere (radius U[0.15, 1.0] m) or an axis-aligned box (each side U[0.3, 2] m).
    Centres are uniform in [1, 19]^3 m (scaled with the cube for other sizes).
    """
    rng = np.random.default_rng(seed)
    extent = n_cells * voxel_m
    prims = _walls(extent, 0.25) + _random_obstacles(rng, n_prims, 0.05 * extent, 0.95 * extent)
    tsdf = build_tsdf((n_cells,) * 3, voxel_m, (0.0, 0.0, 0.0), prims, 0.3)
    return VoxelMap(f"paper{n_cells}_s{seed}", tsdf, voxel_m, np.zeros(3), prims, 0.3)


def eval_map(seed: int, n_prims: int, n_cells: int = 200, voxel_m: float = 0.05,
             size_scale: float = 1.3) -> VoxelMap:
    """Map of the closed-loop evaluation (after Sec. IV-A: random spheres and boxes merged in a
    10 m cube, up to 200 obstacles, about 45 % of the voxels occupied at 200).

    200^3 voxels of 0.05 m, no walls; ``n_prims`` obstacles drawn as in ``paper_map`` with
    every size multiplied by ``size_scale`` (1.3 gives about 0.45 occupied at 200 obstacles),
    centres uniform in [0.5, 9.5]^3 m.
    """
    rng = np.random.default_rng(seed)
    extent = n_cells * voxel_m
    prims = _random_obstacles(rng, n_prims, 0.05 * extent, 0.95 * extent, size_scale)
    tsdf = build_tsdf((n_cells,) * 3, voxel_m, (0.0, 0.0, 0.0), prims, 0.3)
    return VoxelMap(f"eval{n_cells}_n{n_prims}_s{seed}", tsdf, voxel_m, np.zeros(3), prims, 0.3)


def eval_pair(m: VoxelMap, seed: int, clearance_m: float = 0.3) -> Tuple[np.ndarray, np.ndarray]:
    """Start and goal of one evaluation flight, on opposite sides of the cube: start x in
    [3 %, 10 %] of the extent, goal x in [90 %, 97 %], y and z in [10 %, 90 %]; each redrawn
    until its voxel is free and the analytic clearance is at least ``clearance_m``."""
    rng = np.random.default_rng(seed)
    ext = m.extent_m

    def draw(lo_x, hi_x):
        while True:
            f = np.array([rng.uniform(lo_x, hi_x), rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9)])
            x = m.origin_m + f * ext
            if _is_free(m, x) and sdf_union(m.prims, x[None, :])[0] >= clearance_m:
                return x

    start = draw(0.03, 0.10)
    return start, draw(0.90, 0.97)


def occ_source_map(seed: int, n_cells: int = 256, voxel_m: float = 0.05,
                   n_prims: int = 120) -> VoxelMap:
    """Source TSDF for the 256^3 occupancy maps of the serving mix (120 primitives)."""
    return paper_map(seed=seed, n_cells=n_cells, voxel_m=voxel_m, n_prims=n_prims)


# ----------------------------------------------------------------------------------------
# storage encodings of a float32 TSDF (inputs for the precision variants)
# ----------------------------------------------------------------------------------------

def encode_f16(tsdf: np.ndarray) -> np.ndarray:
    """Sign-preserving float16 encoding, returned as uint16 bit patterns.

    Values <= 0 round to nearest (a tiny negative may become -0, still <= 0).  Positive
    values round toward zero and never reach +0: what would underflow becomes the smallest
    subnormal 2^-24.  Hence (f16 <= 0) == (f32 <= 0) voxel for voxel.
    """
    x = np.asarray(tsdf, dtype=np.float32)
    h = x.astype(np.float16)
    bits = h.view(np.uint16).copy()
    pos = x > 0
    over = pos & (h.astype(np.float32) > x)
    bits[over] -= 1                       # one ulp toward zero (positive, non-zero bits)
    zero_pos = pos & ((bits & 0x7FFF) == 0)
    bits[zero_pos] = 1                    # smallest positive subnormal
    return bits


def encode_u8(tsdf: np.ndarray) -> np.ndarray:
    """Occupancy bytes: 1 where the TSDF is <= 0, else 0."""
    return (np.asarray(tsdf) <= 0).astype(np.uint8)


# ----------------------------------------------------------------------------------------
# robot states
# ----------------------------------------------------------------------------------------

def _is_free(m: VoxelMap, x: np.ndarray) -> bool:
    g = (x - m.origin_m) / m.voxel_m
    v = np.floor(g).astype(np.int64)
    nx, ny, nz = m.dims
    if np.any(v < 0) or v[0] >= nx or v[1] >= ny or v[2] >= nz:
        return False
    if m.tsdf[v[2], v[1], v[0]] <= 0:
        return False
    return bool(sdf_union(m.prims, x[None, :])[0] >= m.voxel_m)


def free_state(m: VoxelMap, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Position uniform in the grid, redrawn until its voxel is free and the analytic
    clearance is at least one voxel; velocity ~ N(0, I3) m/s."""
    rng = np.random.default_rng(seed)
    ext = m.extent_m
    while True:
        x = m.origin_m + rng.uniform(0.0, 1.0, size=3) * ext
        if _is_free(m, x):
            break
    v = rng.normal(0.0, 1.0, size=3)
    return x, v


def trajectory_states(m: VoxelMap, n_traj: int = 8, per_traj: int = 64, seed0: int = 300
                      ) -> Tuple[np.ndarray, np.ndarray]:
    """States along ``n_traj`` seeded polylines through 6 free waypoints each.

    ``per_traj`` states per polyline, equally spaced by arc length; velocity is the unit
    tangent times a speed U[0.5, 3] m/s.  A sample that is not free is moved to the nearest
    free point found by a seeded outward search.
    """
    xs, vs = [], []
    for j in range(n_traj):
        rng = np.random.default_rng(seed0 + j)
        wps = []
        while len(wps) < 6:
            x = m.origin_m + rng.uniform(0.05, 0.95, size=3) * m.extent_m
            if _is_free(m, x):
                wps.append(x)
        wps = np.asarray(wps)
        seg = np.linalg.norm(np.diff(wps, axis=0), axis=1)
        cum = np.concatenate([[0.0], np.cumsum(seg)])
        s = np.linspace(0.0, cum[-1], per_traj)
        for sk in s:
            i = min(int(np.searchsorted(cum, sk, side="right")) - 1, len(seg) - 1)
            a = (sk - cum[i]) / seg[i]
            x = wps[i] * (1 - a) + wps[i + 1] * a
            tan = (wps[i + 1] - wps[i]) / seg[i]
            rad = m.voxel_m
            while not _is_free(m, x):
                cand = x + rng.normal(0.0, rad, size=3)
                if _is_free(m, cand):
                    x = cand
                    break
                rad *= 1.05
            xs.append(x)
            vs.append(tan * rng.uniform(0.5, 3.0))
    return np.asarray(xs), np.asarray(vs)


def ray_counts(n: int, seed: int = 399, lo: int = 4096, hi: int = 65536) -> np.ndarray:
    """Log-uniform ray counts in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))).astype(np.int32)


def poisson_arrivals(rate_hz: float, n: int, seed: int = 500) -> np.ndarray:
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


# ----------------------------------------------------------------------------------------
# LiDAR scans from the analytic geometry (not from the voxel map)
# ----------------------------------------------------------------------------------------

def _ray_enter(prim: Primitive, p0: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Smallest t > 0 at which the rays p0 + t u (u: [n,3]) enter the primitive's solid."""
    n = u.shape[0]
    kind = prim[0]
    t = np.full(n, np.inf)
    if kind == "sphere":
        c = np.asarray(prim[1:4]); R = prim[4]
        oc = p0 - c
        b = u @ oc
        cc = oc @ oc - R * R
        disc = b * b - cc
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t0 = -b - sq
        t = np.where(ok & (t0 > 0), t0, t)
        return t
    if kind in ("box", "slab"):
        if kind == "box":
            c = np.asarray(prim[1:4]); e = np.asarray(prim[4:7])
            lo, hi = c - e, c + e
        else:
            lo = np.full(3, -np.inf); hi = np.full(3, np.inf)
            lo[prim[1]], hi[prim[1]] = prim[2], prim[3]
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (lo - p0) / u
            t2 = (hi - p0) / u
        tn = np.where(np.isnan(t1), -np.inf, np.minimum(t1, t2))
        tf = np.where(np.isnan(t2), np.inf, np.maximum(t1, t2))
        # zero direction component: inside the slab for all t or never
        zero = u == 0
        inside = (p0 > lo) & (p0 < hi)
        tn = np.where(zero, np.where(inside, -np.inf, np.inf), tn)
        tf = np.where(zero, np.where(inside, np.inf, -np.inf), tf)
        tenter = tn.max(axis=1)
        texit = tf.min(axis=1)
        ok = (tenter <= texit) & (tenter > 0)
        return np.where(ok, tenter, t)
    if kind == "halfspace_below":
        axis, level = prim[1], prim[2]
        ua = u[:, axis]
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = (level - p0[axis]) / ua
        ok = (ua < 0) & (p0[axis] > level)
        return np.where(ok, tt, t)
    raise ValueError(kind)


def lidar_directions(n_elev: int = 64, n_azim: int = 1024, fov_deg: float = 45.0) -> np.ndarray:
    """Unit beam directions [n_elev * n_azim, 3], elevations evenly over +-fov/2."""
    el = np.deg2rad(np.linspace(-fov_deg / 2, fov_deg / 2, n_elev))
    az = np.arange(n_azim) * (2 * np.pi / n_azim)
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)


def synth_scan(m: VoxelMap, x: np.ndarray, seed: int, n_elev: int = 64, n_azim: int = 1024,
               max_range_m: float = 20.0, noise_m: float = 0.02, dropout: float = 0.1,
               fov_deg: float = 45.0) -> np.ndarray:
    """Robot-relative, world-aligned float32 points [n_elev*n_azim, 3].

    Range = the analytic first entry into the primitives' union plus N(0, noise^2);
    beams with no return within ``max_range_m`` and Bernoulli(dropout) beams are (0, 0, 0).
    """
    rng = np.random.default_rng(seed)
    u = lidar_directions(n_elev, n_azim, fov_deg)
    t = np.full(u.shape[0], np.inf)
    for prim in m.prims:
        t = np.minimum(t, _ray_enter(prim, np.asarray(x, dtype=np.float64), u))
    rng_m = t + rng.normal(0.0, noise_m, size=t.shape)
    keep = np.isfinite(t) & (t <= max_range_m) & (rng.uniform(size=t.shape) >= dropout)
    pts = u * np.where(keep, rng_m, 0.0)[:, None]
    return pts.astype(np.float32)


# ----------------------------------------------------------------------------------------
# policy parameter sets: Table I ("Static Map" and "LiDAR" columns) plus the constants the
# paper leaves open (epsilon, max range, pseudo-inverse cut, minimum LiDAR range) and the
# sub-voxel distance switch (0: the walk's voxel-face distance)
# ----------------------------------------------------------------------------------------

STATIC_MAP_PARAMS = dict(c=0.2, eta_rep=88.0, nu_rep=1.4, eta_damp=140.0, nu_damp=1.2,
                         radius=2.4, eps=1e-3, max_range=10.0, rank_tol=1e-6, min_range=0.1, subvoxel=0.0)
LIDAR_PARAMS = dict(c=1.0, eta_rep=1.2, nu_rep=1.5, eta_damp=3.0, nu_damp=1.0,
                    radius=1.3, eps=1e-3, max_range=20.0, rank_tol=1e-6, min_range=0.1, subvoxel=0.0)


def params(preset: str = "static", **overrides) -> dict:
    """A parameter dict (``preset`` is "static" or "lidar"), with overrides applied."""
    base = {"static": STATIC_MAP_PARAMS, "lidar": LIDAR_PARAMS}[preset]
    out = dict(base)
    for k, v in overrides.items():
        if k not in out:
            raise KeyError(k)
        out[k] = float(v)
    return out


# ----------------------------------------------------------------------------------------
# sparse block maps (8^3-voxel blocks stored where a surface is within reach)
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class SparseMap:
    """A synthetic sparse map: float32 TSDF in 8^3-voxel blocks at integer block coordinates
    (block (bx, by, bz) covers voxels 8 bx .. 8 bx + 7 along x, ...); every voxel outside a
    stored block is free.  Voxel (i, j, k) has its centre at origin + (idx + 1/2) h."""

    name: str
    coords: np.ndarray        # int32 [n, 3]
    values: np.ndarray        # float32 [n, 8, 8, 8], indexed (block, z, y, x)
    voxel_m: float
    origin_m: np.ndarray
    prims: List[Primitive]
    trunc_m: float

    @property
    def n_blocks(self) -> int:
        return int(self.coords.shape[0])

    def occupied_fraction(self) -> float:
        """Occupied share of the stored voxels."""
        return float(np.count_nonzero(self.values <= 0)) / self.values.size

    def dense_crop(self, lo_vox, hi_vox) -> Tuple[np.ndarray, np.ndarray]:
        """The voxels [lo, hi) (x, y, z) as a dense float32 TSDF array [z, y, x] (free voxels
        +trunc) and the world origin of its minimum corner; lo and hi are multiples of 8."""
        lo = np.asarray(lo_vox, dtype=np.int64)
        hi = np.asarray(hi_vox, dtype=np.int64)
        assert np.all(lo % 8 == 0) and np.all(hi % 8 == 0) and np.all(hi > lo)
        n = hi - lo
        out = np.full((n[2], n[1], n[0]), self.trunc_m, np.float32)
        b = self.coords.astype(np.int64) * 8
        sel = np.nonzero(np.all((b >= lo) & (b < hi), axis=1))[0]
        for k in sel:
            o = b[k] - lo
            out[o[2]:o[2] + 8, o[1]:o[1] + 8, o[0]:o[0] + 8] = self.values[k]
        return out, np.asarray(self.origin_m, dtype=np.float64) + lo * self.voxel_m


def sparse_from_dense(m: VoxelMap, offset_blocks=(0, 0, 0), keep_free: float = 0.3, seed: int = 0,
                      origin_m=None) -> SparseMap:
    """The whole 8^3 blocks of a dense map as a sparse map: every block holding an occupied
    voxel, and each free block with probability keep_free (seeded), stored in a seeded random
    order at block coordinates shifted by offset_blocks.  The sparse frame's voxel (0, 0, 0)
    sits at origin_m (default: where the shifted blocks line up with the dense grid)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = m.tsdf.shape
    coords, vals = [], []
    for bz in range(nz // 8):
        for by in range(ny // 8):
            for bx in range(nx // 8):
                blk = m.tsdf[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
                if np.any(blk <= 0) or rng.uniform() < keep_free:
                    coords.append((bx + offset_blocks[0], by + offset_blocks[1], bz + offset_blocks[2]))
                    vals.append(blk)
    order = rng.permutation(len(coords))
    off = np.asarray(offset_blocks, dtype=np.float64)
    origin = np.asarray(m.origin_m, dtype=np.float64) - 8 * off * m.voxel_m if origin_m is None else \
        np.asarray(origin_m, dtype=np.float64)
    return SparseMap(f"sparse({m.name})", np.asarray(coords, np.int32)[order],
                     np.asarray(vals, np.float32)[order], m.voxel_m, origin, list(m.prims), m.trunc_m)


def _block_voxel_centres(coords: np.ndarray, origin: np.ndarray, h: float) -> np.ndarray:
    """World centres [n, 8, 8, 8, 3] (block, z, y, x) of the voxels of blocks `coords`."""
    i = np.arange(8)
    zz, yy, xx = np.meshgrid(i, i, i, indexing="ij")
    local = np.stack([xx, yy, zz], axis=-1).astype(np.float64)          # [z, y, x, 3]
    base = coords.astype(np.float64)[:, None, None, None, :] * 8.0
    return origin + (base + local + 0.5) * h


def sparse_world(seed: int = 20, side_m: float = 160.0, height_m: float = 12.8, voxel_m: float = 0.05,
                 n_prims: int = 1500, ground_m: float = 0.5, trunc_m: float = 0.3) -> SparseMap:
    """An outdoor-sized world stored sparsely: a side x side area (centred on the origin in x
    and y) with a ground half-space below ground_m and n_prims random spheres and boxes (sizes
    as in the paper-shaped map) resting on or above it.  Blocks are stored where a surface is
    within trunc of the block (the ground's layers and the primitives' bounding boxes), as a
    mapping system allocates blocks near observed surfaces; block coordinates are negative on
    the lower half of each horizontal axis.  At 0.05 m the dense grid would be 3200 x 3200 x
    256 voxels (2.6e9, 10.5 GB as float32)."""
    rng = np.random.default_rng(seed)
    h = voxel_m
    nb_xy = int(round(side_m / (8 * h)))
    origin = np.zeros(3)
    prims: List[Primitive] = [("halfspace_below", 2, ground_m)]
    for _ in range(n_prims):
        c = np.array([rng.uniform(-side_m / 2 + 2, side_m / 2 - 2), rng.uniform(-side_m / 2 + 2, side_m / 2 - 2),
                      rng.uniform(ground_m, 4.0)])
        if rng.uniform() < 0.5:
            prims.append(("sphere", *c, rng.uniform(0.15, 1.0)))
        else:
            prims.append(("box", *c, *(0.5 * rng.uniform(0.3, 2.0, size=3))))
    # blocks within trunc of a surface
    keys = set()
    zlo = int(np.floor((ground_m - trunc_m) / (8 * h)))
    zhi = int(np.floor((ground_m + trunc_m) / (8 * h)))
    bxs = np.arange(-nb_xy // 2, nb_xy // 2)
    for bz in range(zlo, zhi + 1):
        for bx in bxs:
            keys.update((int(bx), int(by), bz) for by in bxs)
    for p in prims[1:]:
        lo, hi = _bbox(p, np.zeros(3))
        lo_b = np.floor((np.asarray(lo) - trunc_m - origin) / (8 * h)).astype(int)
        hi_b = np.floor((np.asarray(hi) + trunc_m - origin) / (8 * h)).astype(int)
        lo_b[:2] = np.maximum(lo_b[:2], -nb_xy // 2)
        hi_b[:2] = np.minimum(hi_b[:2], nb_xy // 2 - 1)
        for bz in range(lo_b[2], hi_b[2] + 1):
            for by in range(lo_b[1], hi_b[1] + 1):
                for bx in range(lo_b[0], hi_b[0] + 1):
                    keys.add((bx, by, bz))
    coords = np.array(sorted(keys), np.int32)
    coords = coords[rng.permutation(len(coords))]
    index = {tuple(c): k for k, c in enumerate(coords.tolist())}
    # values: the ground (a function of z only), then each primitive over its blocks
    n = len(coords)
    zc = origin[2] + (coords[:, 2].astype(np.float64)[:, None] * 8 + np.arange(8) + 0.5) * h     # [n, 8]
    vals = np.clip(zc - ground_m, -trunc_m, trunc_m)[:, :, None, None] * np.ones((1, 1, 8, 8))
    vals = vals.astype(np.float64)
    for p in prims[1:]:
        lo, hi = _bbox(p, np.zeros(3))
        lo_b = np.floor((np.asarray(lo) - trunc_m - origin) / (8 * h)).astype(int)
        hi_b = np.floor((np.asarray(hi) + trunc_m - origin) / (8 * h)).astype(int)
        ks = [index[(bx, by, bz)] for bz in range(lo_b[2], hi_b[2] + 1) for by in range(lo_b[1], hi_b[1] + 1)
              for bx in range(lo_b[0], hi_b[0] + 1) if (bx, by, bz) in index]
        if not ks:
            continue
        ks = np.asarray(ks)
        P = _block_voxel_centres(coords[ks], origin, h)
        vals[ks] = np.minimum(vals[ks], np.clip(_sdf(p, P), -trunc_m, trunc_m))
    # blocks with no voxel within trunc of a surface are free throughout: not stored
    keep = np.any(vals < trunc_m, axis=(1, 2, 3))
    return SparseMap(f"sparse_world({seed})", coords[keep], vals[keep].astype(np.float32), h, origin, prims,
                     trunc_m)


def sparse_free_state(m: SparseMap, seed: int, height_m=(1.0, 3.0)) -> Tuple[np.ndarray, np.ndarray]:
    """A position over the world's area at a height in height_m, redrawn until the analytic
    clearance is at least one voxel and its voxel is free; velocity ~ N(0, I3) m/s."""
    rng = np.random.default_rng(seed)
    lo = m.coords.min(axis=0).astype(np.float64) * 8 * m.voxel_m + m.origin_m
    hi = (m.coords.max(axis=0).astype(np.float64) + 1) * 8 * m.voxel_m + m.origin_m
    while True:
        x = np.array([rng.uniform(lo[0] + 12, hi[0] - 12), rng.uniform(lo[1] + 12, hi[1] - 12),
                      rng.uniform(*height_m)])
        if sdf_union(m.prims, x[None, :])[0] >= m.voxel_m:
            break
    return x, rng.normal(0.0, 1.0, size=3)
