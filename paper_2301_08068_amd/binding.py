"""ctypes binding of ``librmpcast.so`` (the C ABI in ``include/rmpcast.h``).

The functions named ``rmpc_*`` marshal arguments for the C entry point of the same name and
nothing else; every step of a query runs in the library's HIP kernels.  PyTorch supplies the
device memory (the arena and scan buffers) and streams.  There is no fallback: if the
library is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmpcast.so")

RMPC_OK, RMPC_E_INVALID, RMPC_E_NOMAP, RMPC_E_OUT_OF_BOUNDS = 0, -1, -2, -3
RMPC_E_NOMEM, RMPC_E_HIP, RMPC_E_STOPPED = -4, -5, -6
RMPC_TSDF_F32, RMPC_TSDF_F16, RMPC_OCC_U8 = 0, 1, 2
DTYPES = {"f32": RMPC_TSDF_F32, "f16": RMPC_TSDF_F16, "u8": RMPC_OCC_U8}
Q_ILL, Q_IN_COLLISION, Q_TIE = 1, 2, 4
RAY_TIE, RAY_RANGE_TIE, RAY_START_FACE, RAY_IN_COLLISION = 1, 2, 4, 8
MAX_RAYS = 65536


class RmpcError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class MapDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dtype", C.c_int32),
                ("voxel_m", C.c_double), ("origin_m", C.c_double * 3)]


class SparseDesc(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("dtype", C.c_int32), ("voxel_m", C.c_double),
                ("origin_m", C.c_double * 3), ("free_value", C.c_double)]


class Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("c", "eta_rep", "nu_rep", "eta_damp", "nu_damp", "radius",
                                          "eps", "max_range_m", "rank_tol", "min_range_m")] + \
               [("subvoxel", C.c_int32), ("reserved", C.c_int32)]


class QueryDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("map_id", C.c_int32), ("n", C.c_int32), ("reserved", C.c_int32),
                ("x", C.c_double * 3), ("v", C.c_double * 3), ("points_dev", C.c_void_p)]


class LaunchConfig(C.Structure):
    _fields_ = [("lookahead", C.c_int32), ("lane_target_log2", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("use_graph", C.c_int32)]


KIND_MAP, KIND_SCAN = 0, 1
CONFIG_QUERY, CONFIG_BATCH, CONFIG_SPARSE = 0, 1, 2


class Request(C.Structure):
    _fields_ = [("q", QueryDesc), ("points_host", C.c_void_p)]


class ServerConfig(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("max_batch", C.c_int32), ("max_tiles", C.c_int32),
                ("max_pending", C.c_int32), ("staging_bytes", C.c_size_t), ("map_params", Params),
                ("scan_params", Params), ("launch", LaunchConfig)]


class ServerCounters(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("submitted", "completed", "launches", "pending", "in_flight",
                                          "refused", "staging_waits", "staging_peak", "batch_max")]


class Result(C.Structure):
    _fields_ = [("f", C.c_double * 3), ("A", C.c_double * 9), ("b", C.c_double * 3),
                ("lam", C.c_double * 3), ("rank", C.c_int32), ("n_hit", C.c_int32),
                ("n_contrib", C.c_int32), ("n_tie", C.c_int32), ("flags", C.c_uint32),
                ("n_rays", C.c_int32), ("visits", C.c_int64)]


RESULT_BYTES = C.sizeof(Result)

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2301_08068_amd/build.py")
# The library finds the HIP runtime by soname (libamdhip64.so.7), which torch also ships: torch
# must load first so that one runtime, torch's, serves both the arena/streams and the library.
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)
_P = C.POINTER
_lib.rmpc_last_error.restype = C.c_char_p
_lib.rmpc_last_error.argtypes = []
class RolloutParams(C.Structure):
    _fields_ = [("goal", C.c_double * 3), ("alpha", C.c_double), ("beta", C.c_double), ("dt", C.c_double),
                ("max_steps", C.c_int32), ("goal_tol", C.c_double), ("ray_weight", C.c_double),
                ("smooth_every", C.c_int32)]


class Flight(C.Structure):
    _fields_ = [("map_id", C.c_int32), ("n_rays", C.c_int32), ("x0", C.c_double * 3), ("v0", C.c_double * 3),
                ("rp", RolloutParams)]


class RolloutResult(C.Structure):
    _fields_ = [("status", C.c_uint32), ("n_steps", C.c_int32), ("smoothness", C.c_double),
                ("path_length_m", C.c_double), ("x", C.c_double * 3), ("v", C.c_double * 3)]


ROLLOUT_GOAL, ROLLOUT_COLLISION, ROLLOUT_LEFT_GRID, ROLLOUT_TIMEOUT = 1, 2, 3, 4

_SIGS = {
    "rmpc_create": [C.c_int, C.c_void_p, C.c_size_t, _P(C.c_void_p)],
    "rmpc_destroy": [C.c_void_p],
    "rmpc_map_upload": [C.c_void_p, _P(MapDesc), C.c_void_p, C.c_int, C.c_void_p, _P(C.c_int32)],
    "rmpc_map_release": [C.c_void_p, C.c_int32],
    "rmpc_sparse_map_upload": [C.c_void_p, _P(SparseDesc), C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                               _P(C.c_int32)],
    "rmpc_map_footprint": [_P(MapDesc), _P(C.c_size_t)],
    "rmpc_query": [C.c_void_p, C.c_int32, _P(C.c_double), _P(C.c_double), C.c_int32, _P(Params),
                   C.c_void_p, _P(Result)],
    "rmpc_scan_query": [C.c_void_p, C.c_void_p, C.c_int32, _P(C.c_double), _P(Params), C.c_void_p,
                        _P(Result)],
    "rmpc_scan_query_noalloc": [C.c_int, C.c_void_p, C.c_int32, _P(C.c_double), _P(Params), C.c_void_p,
                                C.c_void_p],
    "rmpc_trace_debug": [C.c_void_p, C.c_int32, _P(C.c_double), C.c_int32, _P(Params), C.c_void_p,
                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "rmpc_directions": [C.c_void_p, C.c_int32, _P(C.c_float)],
    "rmpc_query_batch": [C.c_void_p, _P(QueryDesc), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                         _P(Result)],
    "rmpc_config_set": [C.c_void_p, C.c_int32, _P(LaunchConfig)],
    "rmpc_config_get": [C.c_void_p, C.c_int32, _P(LaunchConfig)],
    "rmpc_tune_batch": [C.c_void_p, _P(QueryDesc), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_char_p, _P(LaunchConfig)],
    "rmpc_set_profiling": [C.c_void_p, C.c_int],
    "rmpc_get_profile": [C.c_void_p, _P(C.c_double), _P(C.c_int64)],
    "rmpc_server_start": [C.c_void_p, _P(ServerConfig)],
    "rmpc_submit": [C.c_void_p, _P(Request), _P(C.c_uint64)],
    "rmpc_poll": [C.c_void_p, C.c_uint64, _P(Result), _P(C.c_int32), _P(C.c_double)],
    "rmpc_poll_completed": [C.c_void_p, C.c_int32, _P(C.c_uint64), _P(Result), _P(C.c_double),
                            _P(C.c_int32)],
    "rmpc_server_stats": [C.c_void_p, _P(ServerCounters)],
    "rmpc_server_stop": [C.c_void_p],
    "rmpc_rollout": [C.c_void_p, C.c_int32, _P(C.c_double), _P(C.c_double), C.c_int32, _P(Params),
                     _P(RolloutParams), C.c_void_p, _P(C.c_double), _P(RolloutResult)],
    "rmpc_rollout_batch": [C.c_void_p, _P(Flight), C.c_int32, _P(Params), C.c_void_p, _P(RolloutResult)],
    "rmpc_edt": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "rmpc_esdf_query": [C.c_void_p, C.c_int32, C.c_void_p, _P(C.c_double), _P(C.c_double), _P(Params), C.c_void_p,
                        _P(Result)],
}
for _name, _args in _SIGS.items():
    getattr(_lib, _name).argtypes = _args
    getattr(_lib, _name).restype = C.c_int


def exported_symbols():
    """Names of the C entry points this binding resolves."""
    return sorted(list(_SIGS) + ["rmpc_last_error"])


def _check(st: int, where: str):
    if st != RMPC_OK:
        raise RmpcError(st, where, _lib.rmpc_last_error().decode())


def _d3(x):
    a = (C.c_double * 3)(*[float(v) for v in np.asarray(x, dtype=np.float64).reshape(3)])
    return a


_PARAM_KEYS = ("c", "eta_rep", "nu_rep", "eta_damp", "nu_damp", "radius", "eps", "max_range",
               "rank_tol", "min_range")
_param_cache: Dict[tuple, Params] = {}


def params_struct(p: Dict[str, float]) -> Params:
    """A Params struct from a dict of _PARAM_KEYS (plus an optional "subvoxel" switch)."""
    key = tuple(float(p[k]) for k in _PARAM_KEYS) + (int(bool(p.get("subvoxel", 0))),)
    ps = _param_cache.get(key)
    if ps is None:
        if len(_param_cache) > 256:
            _param_cache.clear()
        ps = _param_cache[key] = Params(*key, 0)
    return ps


def result_dict(r: Result) -> Dict:
    return dict(f=np.array(r.f[:]), S=np.array(r.A[:]).reshape(3, 3), b=np.array(r.b[:]),
                lam=np.array(r.lam[:]), rank=r.rank, n_hit=r.n_hit, n_contrib=r.n_contrib,
                n_tie=r.n_tie, flags=r.flags, n_rays=r.n_rays, visits=r.visits)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


# ----------------------------------------------------------------------------- C entry points

def rmpc_create(device: int, arena_ptr: int, arena_bytes: int) -> int:
    out = C.c_void_p()
    _check(_lib.rmpc_create(device, C.c_void_p(arena_ptr), arena_bytes, C.byref(out)), "rmpc_create")
    return out.value


def rmpc_destroy(ctx: int) -> None:
    _check(_lib.rmpc_destroy(C.c_void_p(ctx)), "rmpc_destroy")


def rmpc_map_upload(ctx: int, nx: int, ny: int, nz: int, dtype: str, voxel_m: float, origin_m,
                    voxels_ptr: int, on_device: bool, stream=None) -> int:
    desc = MapDesc(nx, ny, nz, DTYPES[dtype], float(voxel_m), _d3(origin_m))
    mid = C.c_int32(-1)
    _check(_lib.rmpc_map_upload(C.c_void_p(ctx), C.byref(desc), C.c_void_p(voxels_ptr),
                                int(bool(on_device)), C.c_void_p(_stream_ptr(stream)), C.byref(mid)),
           "rmpc_map_upload")
    return mid.value


def rmpc_sparse_map_upload(ctx: int, coords: np.ndarray, values_ptr: int, n_blocks: int, dtype: str,
                           voxel_m: float, origin_m, on_device: bool, free_value: float = 0.0,
                           stream=None) -> int:
    """coords: int32 [n_blocks, 3] block coordinates (host); values_ptr: n_blocks * 512
    elements of the dtype, block after block, x fastest within a block; free_value: the TSDF
    field outside the stored blocks (TSDF maps)."""
    c = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
    assert c.shape[0] == n_blocks
    d = SparseDesc(int(n_blocks), DTYPES[dtype], float(voxel_m), _d3(origin_m), float(free_value))
    mid = C.c_int32(-1)
    _check(_lib.rmpc_sparse_map_upload(C.c_void_p(ctx), C.byref(d), c.ctypes.data_as(C.c_void_p),
                                       C.c_void_p(values_ptr), int(bool(on_device)),
                                       C.c_void_p(_stream_ptr(stream)), C.byref(mid)), "rmpc_sparse_map_upload")
    return mid.value


def rmpc_map_footprint(nx: int, ny: int, nz: int, dtype: str, voxel_m: float, origin_m) -> int:
    d = MapDesc(nx, ny, nz, DTYPES[dtype], voxel_m, _d3(origin_m))
    out = C.c_size_t()
    _check(_lib.rmpc_map_footprint(C.byref(d), C.byref(out)), "rmpc_map_footprint")
    return out.value


def rmpc_map_release(ctx: int, map_id: int) -> None:
    _check(_lib.rmpc_map_release(C.c_void_p(ctx), map_id), "rmpc_map_release")


def rmpc_query(ctx: int, map_id: int, x, v, n_rays: int, params: Dict[str, float], stream=None) -> Dict:
    r = Result()
    ps = params_struct(params)
    _check(_lib.rmpc_query(C.c_void_p(ctx), map_id, _d3(x), _d3(v), int(n_rays), C.byref(ps),
                           C.c_void_p(_stream_ptr(stream)), C.byref(r)), "rmpc_query")
    return result_dict(r)


def rollout_params(goal, alpha: float, beta: float, dt: float, max_steps: int, goal_tol: float,
                   ray_weight: float = 1.0, smooth_every: int = 1) -> RolloutParams:
    return RolloutParams((C.c_double * 3)(*[float(g) for g in np.asarray(goal, np.float64).reshape(3)]),
                         float(alpha), float(beta), float(dt), int(max_steps), float(goal_tol), float(ray_weight),
                         int(smooth_every))


def _rollout_dict(r: RolloutResult) -> Dict:
    return dict(status=r.status, n_steps=r.n_steps, smoothness=r.smoothness, path_length=r.path_length_m,
                x_final=np.array(r.x[:]), v_final=np.array(r.v[:]))


def rmpc_rollout(ctx: int, map_id: int, x0, v0, n_rays: int, params: Dict[str, float], goal, alpha: float,
                 beta: float, dt: float, max_steps: int, goal_tol: float, trajectory: bool = False,
                 stream=None, ray_weight: float = 1.0, smooth_every: int = 1) -> Dict:
    """Closed-loop rollout; with trajectory=True also returns the visited states x, v."""
    rp = rollout_params(goal, alpha, beta, dt, max_steps, goal_tol, ray_weight, smooth_every)
    traj = np.zeros((int(max_steps) + 1, 6), np.float64) if trajectory else None
    tp = traj.ctypes.data_as(_P(C.c_double)) if traj is not None else None
    r = RolloutResult()
    ps = params_struct(params)
    _check(_lib.rmpc_rollout(C.c_void_p(ctx), int(map_id), _d3(x0), _d3(v0), int(n_rays), C.byref(ps),
                             C.byref(rp), C.c_void_p(_stream_ptr(stream)), tp, C.byref(r)), "rmpc_rollout")
    out = _rollout_dict(r)
    if traj is not None:
        out["x"] = traj[:r.n_steps + 1, :3].copy()
        out["v"] = traj[:r.n_steps + 1, 3:].copy()
    return out


def rmpc_rollout_batch(ctx: int, flights, params: Dict[str, float], stream=None) -> list:
    """Batched rollout.  flights: dicts with map_id, n_rays, x0, v0, goal, alpha, beta, dt,
    max_steps, goal_tol and optionally ray_weight, smooth_every."""
    fs = (Flight * len(flights))()
    for k, f in enumerate(flights):
        fs[k].map_id = int(f["map_id"])
        fs[k].n_rays = int(f["n_rays"])
        fs[k].x0 = (C.c_double * 3)(*np.asarray(f["x0"], np.float64).reshape(3).tolist())
        fs[k].v0 = (C.c_double * 3)(*np.asarray(f["v0"], np.float64).reshape(3).tolist())
        fs[k].rp = rollout_params(f["goal"], f["alpha"], f["beta"], f["dt"], f["max_steps"], f["goal_tol"],
                                  f.get("ray_weight", 1.0), f.get("smooth_every", 1))
    out = (RolloutResult * len(flights))()
    ps = params_struct(params)
    _check(_lib.rmpc_rollout_batch(C.c_void_p(ctx), fs, len(flights), C.byref(ps), C.c_void_p(_stream_ptr(stream)),
                                   out), "rmpc_rollout_batch")
    return [_rollout_dict(r) for r in out]


class PreparedQuery:
    """rmpc_query with its arguments marshalled once: each call passes the same C arguments
    and returns the Result struct it filled (for loops that repeat one query)."""

    def __init__(self, ctx: int, map_id: int, x, v, n_rays: int, params: Dict[str, float], stream=None):
        self._args = (C.c_void_p(ctx), int(map_id), _d3(x), _d3(v), int(n_rays), C.byref(params_struct(params)),
                      C.c_void_p(_stream_ptr(stream)))
        self.result = Result()
        self._out = C.byref(self.result)
        self._fn = _lib.rmpc_query

    def __call__(self) -> Result:
        st = self._fn(*self._args, self._out)
        if st != RMPC_OK:
            _check(st, "rmpc_query")
        return self.result


class PreparedScan:
    """rmpc_scan_query with its arguments marshalled once (for loops that repeat one frame)."""

    def __init__(self, ctx: int, points_ptr: int, n_points: int, v, params: Dict[str, float], stream=None):
        self._args = (C.c_void_p(ctx), C.c_void_p(points_ptr), int(n_points), _d3(v),
                      C.byref(params_struct(params)), C.c_void_p(_stream_ptr(stream)))
        self.result = Result()
        self._out = C.byref(self.result)
        self._fn = _lib.rmpc_scan_query

    def __call__(self) -> Result:
        st = self._fn(*self._args, self._out)
        if st != RMPC_OK:
            _check(st, "rmpc_scan_query")
        return self.result


def rmpc_scan_query(ctx: int, points_ptr: int, n_points: int, v, params: Dict[str, float],
                    stream=None) -> Dict:
    r = Result()
    ps = params_struct(params)
    _check(_lib.rmpc_scan_query(C.c_void_p(ctx), C.c_void_p(points_ptr), int(n_points), _d3(v),
                                C.byref(ps), C.c_void_p(_stream_ptr(stream)), C.byref(r)),
           "rmpc_scan_query")
    return result_dict(r)


def rmpc_scan_query_noalloc(device: int, points_ptr: int, n_points: int, v, params: Dict[str, float],
                            out_ptr: int, stream=None) -> None:
    """Enqueue the context-free scan query; the result lands in the device buffer at out_ptr
    (RESULT_BYTES bytes) in stream order."""
    _check(_lib.rmpc_scan_query_noalloc(int(device), C.c_void_p(points_ptr), int(n_points), _d3(v),
                                        C.byref(params_struct(params)), C.c_void_p(_stream_ptr(stream)),
                                        C.c_void_p(out_ptr)), "rmpc_scan_query_noalloc")


def result_from_bytes(buf: bytes) -> Dict:
    """A result dict from the RESULT_BYTES bytes of an rmpc_result copied from the device."""
    return result_dict(Result.from_buffer_copy(buf))


def rmpc_trace_debug(ctx: int, map_id: int, x, n_rays: int, params: Dict[str, float], hit_ptr: int,
                     dist_ptr: int, flags_ptr: int, visits_ptr: int = 0, stream=None) -> None:
    ps = params_struct(params)
    _check(_lib.rmpc_trace_debug(C.c_void_p(ctx), map_id, _d3(x), int(n_rays), C.byref(ps),
                                 C.c_void_p(_stream_ptr(stream)), C.c_void_p(hit_ptr),
                                 C.c_void_p(dist_ptr), C.c_void_p(flags_ptr),
                                 C.c_void_p(visits_ptr or None)), "rmpc_trace_debug")


def rmpc_directions(ctx: int, n: int) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float32)
    _check(_lib.rmpc_directions(C.c_void_p(ctx), int(n), out.ctypes.data_as(_P(C.c_float))),
           "rmpc_directions")
    return out


def query_descs(queries) -> "C.Array":
    """Build a QueryDesc array from dicts: {"kind": "map", "map_id", "n", "x", "v"} or
    {"kind": "scan", "points_ptr", "n", "v"}."""
    arr = (QueryDesc * len(queries))()
    for k, q in enumerate(queries):
        d = arr[k]
        d.kind = KIND_MAP if q["kind"] == "map" else KIND_SCAN
        d.map_id = int(q.get("map_id", -1))
        d.n = int(q["n"])
        d.x = _d3(q.get("x", (0.0, 0.0, 0.0)))
        d.v = _d3(q["v"])
        d.points_dev = C.c_void_p(int(q.get("points_ptr", 0)) or None)
    return arr


def rmpc_query_batch(ctx: int, descs, map_params: Optional[Dict[str, float]],
                     scan_params: Optional[Dict[str, float]], stream=None) -> list:
    n = len(descs)
    out = (Result * n)()
    mp = C.byref(params_struct(map_params)) if map_params else None
    sp = C.byref(params_struct(scan_params)) if scan_params else None
    _check(_lib.rmpc_query_batch(C.c_void_p(ctx), descs, n, mp, sp, C.c_void_p(_stream_ptr(stream)), out),
           "rmpc_query_batch")
    return [result_dict(r) for r in out]


def rmpc_config_set(ctx: int, which: int, lookahead: int, lane_target_log2: int,
                    blocks_per_cu: int = 0, use_graph: int = 0) -> None:
    cfg = LaunchConfig(lookahead, lane_target_log2, blocks_per_cu, use_graph)
    _check(_lib.rmpc_config_set(C.c_void_p(ctx), which, C.byref(cfg)), "rmpc_config_set")


def rmpc_config_get(ctx: int, which: int) -> Dict[str, int]:
    cfg = LaunchConfig()
    _check(_lib.rmpc_config_get(C.c_void_p(ctx), which, C.byref(cfg)), "rmpc_config_get")
    return {k: getattr(cfg, k) for k, _ in LaunchConfig._fields_}


def rmpc_tune_batch(ctx: int, descs, map_params, scan_params, cache_path: Optional[str] = None,
                    stream=None) -> Dict[str, int]:
    cfg = LaunchConfig()
    mp = C.byref(params_struct(map_params)) if map_params else None
    sp = C.byref(params_struct(scan_params)) if scan_params else None
    _check(_lib.rmpc_tune_batch(C.c_void_p(ctx), descs, len(descs), mp, sp, C.c_void_p(_stream_ptr(stream)),
                                cache_path.encode() if cache_path else None, C.byref(cfg)), "rmpc_tune_batch")
    return {k: getattr(cfg, k) for k, _ in LaunchConfig._fields_}


def rmpc_set_profiling(ctx: int, enable: bool) -> None:
    _check(_lib.rmpc_set_profiling(C.c_void_p(ctx), int(bool(enable))), "rmpc_set_profiling")


def rmpc_get_profile(ctx: int) -> Tuple[float, int]:
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(_lib.rmpc_get_profile(C.c_void_p(ctx), C.byref(ms), C.byref(n)), "rmpc_get_profile")
    return ms.value, n.value


def request(q: Dict, points_host_ptr: Optional[int] = None) -> Request:
    """A serving request from a query dict (see query_descs); scan points either on the device
    ("points_ptr") or in host memory (points_host_ptr, pinned for asynchronous copies)."""
    r = Request()
    r.q = query_descs([q])[0]
    r.points_host = C.c_void_p(int(points_host_ptr) if points_host_ptr else None)
    return r


def rmpc_server_start(ctx: int, n_slots: int, max_batch: int, map_params: Dict[str, float],
                      scan_params: Dict[str, float], launch: Dict[str, int], staging_bytes: int = 0,
                      max_tiles: int = 0, max_pending: int = 0) -> None:
    cfg = ServerConfig(int(n_slots), int(max_batch), int(max_tiles), int(max_pending), int(staging_bytes),
                       params_struct(map_params), params_struct(scan_params),
                       LaunchConfig(launch["lookahead"], launch["lane_target_log2"], launch["blocks_per_cu"],
                                    launch["use_graph"]))
    _check(_lib.rmpc_server_start(C.c_void_p(ctx), C.byref(cfg)), "rmpc_server_start")


def rmpc_submit(ctx: int, req: Request) -> int:
    t = C.c_uint64(0)
    _check(_lib.rmpc_submit(C.c_void_p(ctx), C.byref(req), C.byref(t)), "rmpc_submit")
    return t.value


def rmpc_poll(ctx: int, ticket: int) -> Tuple[Optional[Dict], float]:
    r = Result()
    done = C.c_int32(0)
    lat = C.c_double(0.0)
    _check(_lib.rmpc_poll(C.c_void_p(ctx), C.c_uint64(ticket), C.byref(r), C.byref(done), C.byref(lat)),
           "rmpc_poll")
    return (result_dict(r), lat.value) if done.value else (None, 0.0)


def rmpc_poll_completed(ctx: int, max_n: int = 256, raw: bool = False):
    """Ready results in completion order: a list of (ticket, result dict, latency_s); with
    raw=True the tuple (tickets, latencies, Result array, count) without conversion."""
    tickets = (C.c_uint64 * max_n)()
    out = (Result * max_n)()
    lat = (C.c_double * max_n)()
    n = C.c_int32(0)
    _check(_lib.rmpc_poll_completed(C.c_void_p(ctx), int(max_n), tickets, out, lat, C.byref(n)),
           "rmpc_poll_completed")
    if raw:
        return tickets[:n.value], lat[:n.value], out, n.value
    return [(tickets[i], result_dict(out[i]), lat[i]) for i in range(n.value)]


def rmpc_server_stats(ctx: int) -> Dict[str, int]:
    c = ServerCounters()
    _check(_lib.rmpc_server_stats(C.c_void_p(ctx), C.byref(c)), "rmpc_server_stats")
    return {k: getattr(c, k) for k, _ in ServerCounters._fields_}


def rmpc_server_stop(ctx: int) -> None:
    _check(_lib.rmpc_server_stop(C.c_void_p(ctx)), "rmpc_server_stop")


# ----------------------------------------------------------------------------- convenience

class Context:
    """A library context on ``cuda:device`` whose arena is a torch uint8 tensor."""

    def __init__(self, device: int = 0, arena_bytes: int = 1 << 30, stream=None):
        import torch
        self.device = device
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        self.ptr = rmpc_create(device, self.arena.data_ptr(), arena_bytes)
        # queries go to this stream (default: the torch stream current at creation)
        self.stream = int(stream) if stream is not None else \
            torch.cuda.current_stream(device).cuda_stream

    def close(self):
        if self.ptr:
            rmpc_destroy(self.ptr)
            self.ptr = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self, data: np.ndarray, voxel_m: float, origin_m, dtype: str = "f32",
               on_device: bool = True) -> int:
        """Upload a [nz, ny, nx] array (float32 TSDF, uint16 binary16 bits or uint8)."""
        import torch
        want = {"f32": np.float32, "f16": np.uint16, "u8": np.uint8}[dtype]
        arr = np.ascontiguousarray(data, dtype=want)
        nz, ny, nx = arr.shape
        if on_device:
            t = torch.from_numpy(arr.view(np.uint8).reshape(-1)).to(f"cuda:{self.device}")
            mid = rmpc_map_upload(self.ptr, nx, ny, nz, dtype, voxel_m, origin_m, t.data_ptr(), True)
            del t
        else:
            mid = rmpc_map_upload(self.ptr, nx, ny, nz, dtype, voxel_m, origin_m, arr.ctypes.data, False)
        return mid

    def upload_sparse(self, coords: np.ndarray, values: np.ndarray, voxel_m: float, origin_m,
                      dtype: str = "f32", free_value: float = 0.3) -> int:
        """Upload a sparse block map: coords int32 [n, 3], values [n, 8, 8, 8] indexed
        (block, z, y, x) (float32 TSDF, uint16 binary16 bits or uint8); free_value: the TSDF
        field outside the stored blocks (the truncation distance)."""
        import torch
        want = {"f32": np.float32, "f16": np.uint16, "u8": np.uint8}[dtype]
        arr = np.ascontiguousarray(values, dtype=want).reshape(-1, 8, 8, 8)
        t = torch.from_numpy(arr.view(np.uint8).reshape(-1)).to(f"cuda:{self.device}")
        mid = rmpc_sparse_map_upload(self.ptr, coords, t.data_ptr(), arr.shape[0], dtype, voxel_m, origin_m,
                                     True, free_value=free_value, stream=self.stream)
        del t
        return mid

    def release(self, map_id: int) -> None:
        rmpc_map_release(self.ptr, map_id)

    def query(self, map_id: int, x, v, n_rays: int, params: Dict[str, float]) -> Dict:
        return rmpc_query(self.ptr, map_id, x, v, n_rays, params, stream=self.stream)

    def scan_query(self, points, v, params: Dict[str, float]) -> Dict:
        """points: a cuda float32 tensor [n, 3] (or a numpy array, uploaded here)."""
        import torch
        if isinstance(points, np.ndarray):
            points = torch.from_numpy(np.ascontiguousarray(points, np.float32)).to(f"cuda:{self.device}")
        assert points.dtype == torch.float32 and points.is_cuda and points.is_contiguous()
        return rmpc_scan_query(self.ptr, points.data_ptr(), points.shape[0], v, params, stream=self.stream)

    def trace(self, map_id: int, x, n_rays: int, params: Dict[str, float]) -> Dict[str, np.ndarray]:
        import torch
        dev = f"cuda:{self.device}"
        hit = torch.empty(n_rays, dtype=torch.int32, device=dev)
        dist = torch.empty(n_rays, dtype=torch.float64, device=dev)
        flags = torch.empty(n_rays, dtype=torch.uint8, device=dev)
        visits = torch.empty(n_rays, dtype=torch.int32, device=dev)
        rmpc_trace_debug(self.ptr, map_id, x, n_rays, params, hit.data_ptr(), dist.data_ptr(),
                         flags.data_ptr(), visits.data_ptr(), stream=self.stream)
        return dict(hit=hit.cpu().numpy(), d=dist.cpu().numpy(), flags=flags.cpu().numpy(),
                    visits=visits.cpu().numpy())

    def directions(self, n: int) -> np.ndarray:
        return rmpc_directions(self.ptr, n)

    def rollout(self, map_id: int, x0, v0, n_rays: int, params: Dict[str, float], goal, alpha: float,
                beta: float, dt: float, max_steps: int, goal_tol: float, trajectory: bool = False,
                ray_weight: float = 1.0, smooth_every: int = 1) -> Dict:
        return rmpc_rollout(self.ptr, map_id, x0, v0, n_rays, params, goal, alpha, beta, dt, max_steps,
                            goal_tol, trajectory, stream=self.stream, ray_weight=ray_weight,
                            smooth_every=smooth_every)

    def edt(self, map_id: int, shape) -> "torch.Tensor":
        """Squared distance transform of a resident map (rmpc_edt) as a cuda int32 tensor of
        the map's array shape (z, y, x)."""
        import torch
        out = torch.empty(tuple(shape), dtype=torch.int32, device=f"cuda:{self.device}")
        _check(_lib.rmpc_edt(C.c_void_p(self.ptr), int(map_id), C.c_void_p(out.data_ptr()),
                             C.c_void_p(_stream_ptr(self.stream))), "rmpc_edt")
        return out

    def esdf_query(self, map_id: int, sqdist, x, v, params: Dict[str, float]) -> Dict:
        """Single-lookup ESDF policy (rmpc_esdf_query) on a distance transform from edt()."""
        r = Result()
        _check(_lib.rmpc_esdf_query(C.c_void_p(self.ptr), int(map_id), C.c_void_p(sqdist.data_ptr()), _d3(x), _d3(v),
                                    C.byref(params_struct(params)), C.c_void_p(_stream_ptr(self.stream)),
                                    C.byref(r)), "rmpc_esdf_query")
        return result_dict(r)

    def rollout_batch(self, flights, params: Dict[str, float]) -> list:
        return rmpc_rollout_batch(self.ptr, flights, params, stream=self.stream)

    def query_batch(self, queries, map_params=None, scan_params=None) -> list:
        """queries: list of dicts (see query_descs); scan points as cuda float32 tensors under
        "points" are kept alive here for the call."""
        keep = []
        qs = []
        for q in queries:
            q = dict(q)
            if q["kind"] == "scan" and "points" in q:
                pts = q.pop("points")
                keep.append(pts)
                q["points_ptr"] = pts.data_ptr()
                q["n"] = pts.shape[0]
            qs.append(q)
        return rmpc_query_batch(self.ptr, query_descs(qs), map_params, scan_params, stream=self.stream)

    def config(self, which: int, **kw) -> Dict[str, int]:
        cur = rmpc_config_get(self.ptr, which)
        if kw:
            cur.update(kw)
            rmpc_config_set(self.ptr, which, cur["lookahead"], cur["lane_target_log2"],
                            cur["blocks_per_cu"], cur["use_graph"])
        return cur
