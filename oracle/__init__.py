"""ctypes front-end of the float64 CPU oracle (``rmp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product library.  It shares no code with the GPU path; the
two only receive the same seeded inputs.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from . import build as _build

MAX_ALT = 16
TIE, RANGE_TIE, START_FACE, IN_COLLISION = 1, 2, 4, 8
Q_ILL, Q_IN_COLLISION, Q_TIE = 1, 2, 4
DTYPES = {"f32": 0, "f16": 1, "u8": 2}


class _Map(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dtype", C.c_int32),
                ("h", C.c_double), ("origin", C.c_double * 3), ("data", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("c", "eta_rep", "nu_rep", "eta_damp", "nu_damp", "radius",
                 "eps", "max_range", "rank_tol", "min_range", "subvoxel")]


class _Result(C.Structure):
    _fields_ = [("S", C.c_double * 9), ("b", C.c_double * 3), ("f", C.c_double * 3),
                ("lam", C.c_double * 3), ("rank", C.c_int32), ("n_hit", C.c_int32),
                ("n_contrib", C.c_int32), ("n_tie", C.c_int32), ("flags", C.c_uint32),
                ("pad", C.c_int32), ("visits", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or \
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER
        L.orc_radical_inverse.restype = C.c_double
        L.orc_radical_inverse.argtypes = [C.c_uint64, C.c_uint32]
        L.orc_directions.argtypes = [C.c_int32, P(C.c_float)]
        L.orc_grid_start.restype = C.c_int
        L.orc_grid_start.argtypes = [P(_Map), P(C.c_double), P(C.c_float)]
        L.orc_trace.restype = C.c_int32
        L.orc_trace.argtypes = [P(_Map), P(C.c_float), P(C.c_float), C.c_int32, C.c_double,
                                P(C.c_int32), P(C.c_double), P(C.c_uint32), P(C.c_int32),
                                P(C.c_int32), P(C.c_int32), P(C.c_double), C.c_int32]
        L.orc_soft_normalize.argtypes = [P(C.c_double), C.c_double, P(C.c_double)]
        L.orc_weight.restype = C.c_double
        L.orc_weight.argtypes = [C.c_double, C.c_double]
        L.orc_rmp_ray.argtypes = [P(_Params), P(C.c_double), C.c_double, P(C.c_double),
                                  P(C.c_double), P(C.c_double)]
        L.orc_sym3_eig.argtypes = [P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_resolve.argtypes = [P(C.c_double), P(C.c_double), C.c_double, P(C.c_double),
                                  P(C.c_double), P(C.c_int32), P(C.c_uint32)]
        L.orc_combine.argtypes = [P(_Params), P(C.c_double), P(C.c_double), P(C.c_int32),
                                  C.c_int32, P(C.c_double), P(_Result)]
        L.orc_query.restype = C.c_int32
        L.orc_query.argtypes = [P(_Map), P(C.c_double), P(C.c_double), C.c_int32,
                                P(C.c_float), P(_Params), C.c_int32, P(_Result)]
        L.orc_field.restype = C.c_double
        L.orc_field.argtypes = [P(_Map), P(C.c_double)]
        L.orc_subvoxel.restype = C.c_double
        L.orc_subvoxel.argtypes = [P(_Map), P(C.c_float), P(C.c_float), C.c_double]
        L.orc_edt.restype = C.c_int32
        L.orc_edt.argtypes = [P(_Map), P(C.c_int32)]
        L.orc_esdf_query.restype = C.c_int32
        L.orc_esdf_query.argtypes = [P(_Map), P(C.c_int32), P(C.c_double), P(C.c_double), P(_Params), P(_Result)]
        L.orc_scan.restype = C.c_int32
        L.orc_scan.argtypes = [P(C.c_float), C.c_int32, P(C.c_double), P(_Params), P(_Result)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _d3(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))


class OracleMap:
    """A dense voxel map as the oracle sees it (the array is kept alive here)."""

    def __init__(self, data: np.ndarray, voxel_m: float, origin_m, dtype: str = "f32"):
        want = {"f32": np.float32, "f16": np.uint16, "u8": np.uint8}[dtype]
        self.data = np.ascontiguousarray(data, dtype=want)
        nz, ny, nx = self.data.shape
        self.s = _Map(nx, ny, nz, DTYPES[dtype], float(voxel_m),
                      (C.c_double * 3)(*[float(o) for o in origin_m]),
                      self.data.ctypes.data_as(C.c_void_p))

    @classmethod
    def from_voxelmap(cls, vm, dtype: str = "f32", data: Optional[np.ndarray] = None):
        return cls(vm.tsdf if data is None else data, vm.voxel_m, vm.origin_m, dtype)


def params_struct(p: Dict[str, float]) -> _Params:
    return _Params(*[float(p.get(k, 0.0)) if k == "subvoxel" else float(p[k]) for k, _ in _Params._fields_])


def radical_inverse(i: int, base: int) -> float:
    return lib().orc_radical_inverse(i, base)


def directions(n: int) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float32)
    lib().orc_directions(n, _ptr(out, C.c_float))
    return out


def grid_start(m: OracleMap, x) -> Optional[np.ndarray]:
    g = np.empty(3, dtype=np.float32)
    ok = lib().orc_grid_start(C.byref(m.s), _ptr(_d3(x), C.c_double), _ptr(g, C.c_float))
    return g if ok else None


def trace(m: OracleMap, g, dirs: np.ndarray, max_range: float, nthreads: int = 1) -> Dict:
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float32).reshape(3))
    dirs = np.ascontiguousarray(dirs, dtype=np.float32)
    n = dirs.shape[0]
    out = dict(hit=np.empty(n, np.int32), d=np.empty(n, np.float64), flags=np.empty(n, np.uint32),
               visits=np.empty(n, np.int32), alt_n=np.empty(n, np.int32),
               alt_hit=np.empty((n, MAX_ALT), np.int32), alt_d=np.empty((n, MAX_ALT), np.float64))
    rc = lib().orc_trace(C.byref(m.s), _ptr(g, C.c_float), _ptr(dirs, C.c_float), n, max_range,
                         _ptr(out["hit"], C.c_int32), _ptr(out["d"], C.c_double),
                         _ptr(out["flags"], C.c_uint32), _ptr(out["visits"], C.c_int32),
                         _ptr(out["alt_n"], C.c_int32), _ptr(out["alt_hit"], C.c_int32),
                         _ptr(out["alt_d"], C.c_double), nthreads)
    if rc < 0:
        raise ValueError("start outside the grid")
    return out


def field(m: OracleMap, p) -> float:
    """Trilinear interpolation of the stored TSDF values (at voxel centres) at grid point p."""
    return lib().orc_field(C.byref(m.s), _ptr(_d3(p), C.c_double))


def subvoxel(m: OracleMap, g, r, d: float) -> float:
    """Refined hit distance (reading R20): one secant step on the field across the entry
    point of the hit voxel at walk distance d (metres) from grid start g along r."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float32).reshape(3))
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float32).reshape(3))
    return lib().orc_subvoxel(C.byref(m.s), _ptr(g, C.c_float), _ptr(r, C.c_float), float(d))


def edt(m: OracleMap) -> np.ndarray:
    """Squared centre-to-centre distance (voxels^2) from every voxel to the nearest occupied
    voxel, shaped like the map's array (z, y, x); -1 everywhere when nothing is occupied."""
    nz, ny, nx = m.data.shape[:3]
    out = np.empty((nz, ny, nx), np.int32)
    if lib().orc_edt(C.byref(m.s), _ptr(out, C.c_int32)) != 0:
        raise MemoryError("orc_edt")
    return out


def esdf_query(m: OracleMap, sq: np.ndarray, x, v, p: Dict[str, float]) -> Dict:
    """Single-lookup ESDF policy (reading R22) on the squared distance transform sq."""
    sq = np.ascontiguousarray(sq, dtype=np.int32)
    r = _Result()
    ps = params_struct(p)
    if lib().orc_esdf_query(C.byref(m.s), _ptr(sq, C.c_int32), _ptr(_d3(x), C.c_double), _ptr(_d3(v), C.c_double),
                            C.byref(ps), C.byref(r)) < 0:
        raise ValueError("start outside the grid")
    return _result_dict(r)


def soft_normalize(v, c: float) -> np.ndarray:
    out = np.empty(3)
    lib().orc_soft_normalize(_ptr(_d3(v), C.c_double), c, _ptr(out, C.c_double))
    return out


def weight(d: float, r: float) -> float:
    return lib().orc_weight(d, r)


def rmp_ray(p: Dict[str, float], rhat, d: float, v):
    A = np.empty(9)
    b = np.empty(3)
    ps = params_struct(p)
    lib().orc_rmp_ray(C.byref(ps), _ptr(_d3(rhat), C.c_double), float(d),
                      _ptr(_d3(v), C.c_double), _ptr(A, C.c_double), _ptr(b, C.c_double))
    return A.reshape(3, 3), b


def sym3_eig(S):
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(9))
    lam = np.empty(3)
    Q = np.empty(9)
    lib().orc_sym3_eig(_ptr(S, C.c_double), _ptr(lam, C.c_double), _ptr(Q, C.c_double))
    return lam, Q.reshape(3, 3)


def resolve(S, b, rank_tol: float):
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(9))
    f = np.empty(3)
    lam = np.empty(3)
    rank = C.c_int32(0)
    fl = C.c_uint32(0)
    lib().orc_resolve(_ptr(S, C.c_double), _ptr(_d3(b), C.c_double), rank_tol, _ptr(f, C.c_double),
                      _ptr(lam, C.c_double), C.byref(rank), C.byref(fl))
    return f, lam, rank.value, fl.value


def _result_dict(r: _Result) -> Dict:
    return dict(S=np.array(r.S[:]).reshape(3, 3), b=np.array(r.b[:]), f=np.array(r.f[:]),
                lam=np.array(r.lam[:]), rank=r.rank, n_hit=r.n_hit, n_contrib=r.n_contrib,
                n_tie=r.n_tie, flags=r.flags, visits=r.visits)


def combine(p: Dict[str, float], rhat: np.ndarray, d: np.ndarray, hit: np.ndarray, v) -> Dict:
    rhat = np.ascontiguousarray(rhat, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64)
    hit = np.ascontiguousarray(hit, dtype=np.int32)
    r = _Result()
    ps = params_struct(p)
    lib().orc_combine(C.byref(ps), _ptr(rhat, C.c_double), _ptr(d, C.c_double),
                      _ptr(hit, C.c_int32), rhat.shape[0], _ptr(_d3(v), C.c_double), C.byref(r))
    return _result_dict(r)


def query(m: OracleMap, x, v, n: int, p: Dict[str, float], nthreads: int = 1,
          dirs: Optional[np.ndarray] = None) -> Dict:
    dirs = directions(n) if dirs is None else np.ascontiguousarray(dirs[:n], dtype=np.float32)
    r = _Result()
    ps = params_struct(p)
    rc = lib().orc_query(C.byref(m.s), _ptr(_d3(x), C.c_double), _ptr(_d3(v), C.c_double), n,
                         _ptr(dirs, C.c_float), C.byref(ps), nthreads, C.byref(r))
    if rc < 0:
        raise ValueError("start outside the grid")
    return _result_dict(r)


def scan(points: np.ndarray, v, p: Dict[str, float]) -> Dict:
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    r = _Result()
    ps = params_struct(p)
    lib().orc_scan(_ptr(pts, C.c_float), pts.shape[0], _ptr(_d3(v), C.c_double), C.byref(ps),
                   C.byref(r))
    return _result_dict(r)


# ------------------------------------------------------------------------------------------
# closed-loop rollout (Sec. III-A Eq. 1 with the goal attractor of Sec. III-C): the ray policy
# summed with the attractor (metric I), resolved and integrated step by step
# ------------------------------------------------------------------------------------------

ROLLOUT_GOAL, ROLLOUT_COLLISION, ROLLOUT_LEFT_GRID, ROLLOUT_TIMEOUT = 1, 2, 3, 4


def attractor(goal, x, v, alpha: float, beta: float, c: float) -> np.ndarray:
    """Goal attractor force (Sec. III-C Eq. 3): alpha s(goal - x) - beta v, s of Eq. 4."""
    return alpha * soft_normalize(np.asarray(goal, np.float64) - np.asarray(x, np.float64), c) \
        - beta * np.asarray(v, np.float64)


def smoothness(xs: np.ndarray, every: int = 1) -> float:
    """Mean angular similarity 1 - acos(cos angle)/pi between consecutive non-zero displacement
    segments of a path sampled at every ``every``-th point xs[0], xs[every], ... (1.0: straight;
    the path measure of Sec. IV-B); 1.0 with fewer than two segments."""
    seg = np.diff(np.asarray(xs, np.float64)[::every], axis=0)
    seg = seg[np.linalg.norm(seg, axis=1) > 0.0]
    if len(seg) < 2:
        return 1.0
    a, b = seg[:-1], seg[1:]
    cosang = np.sum(a * b, axis=1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
    return float(np.mean(1.0 - np.arccos(np.clip(cosang, -1.0, 1.0)) / np.pi))


def rollout(m: OracleMap, x0, v0, n_rays: int, p: Dict[str, float], goal, alpha: float, beta: float,
            dt: float, max_steps: int, goal_tol: float, nthreads: int = 1, ray_weight: float = 1.0,
            smooth_every: int = 1) -> Dict:
    """Each step k: stop when within goal_tol of the goal or outside the grid; query the state
    (stop when its voxel is occupied); a_k = (I + w S)^-1 (f_a + w b) with S, b the ray sums,
    w = ray_weight (1: Eq. 1 as written) and f_a the attractor; v_{k+1} = v_k + a_k dt,
    x_{k+1} = x_k + v_{k+1} dt (semi-implicit Euler)."""
    x = np.array(x0, np.float64)
    v = np.array(v0, np.float64)
    xs, vs, acc = [x.copy()], [v.copy()], []
    status = ROLLOUT_TIMEOUT
    for _ in range(max_steps):
        if np.linalg.norm(x - np.asarray(goal, np.float64)) <= goal_tol:
            status = ROLLOUT_GOAL
            break
        try:
            q = query(m, x, v, n_rays, p, nthreads=nthreads)
        except ValueError:
            status = ROLLOUT_LEFT_GRID
            break
        if q["flags"] & Q_IN_COLLISION:
            status = ROLLOUT_COLLISION
            break
        a = np.linalg.solve(np.eye(3) + ray_weight * q["S"],
                            attractor(goal, x, v, alpha, beta, p["c"]) + ray_weight * q["b"])
        v = v + a * dt
        x = x + v * dt
        xs.append(x.copy())
        vs.append(v.copy())
        acc.append(a)
    else:
        if np.linalg.norm(x - np.asarray(goal, np.float64)) <= goal_tol:
            status = ROLLOUT_GOAL
    xs = np.array(xs)
    return dict(status=status, n_steps=len(xs) - 1, x=xs, v=np.array(vs), a=np.array(acc).reshape(-1, 3),
                smoothness=smoothness(xs, smooth_every), path_length=float(np.sum(np.linalg.norm(np.diff(xs, axis=0), axis=1))))
