"""ctypes binding of libwos (include/wos.h): the same entry points, argument marshalling only.

Device buffers are torch tensors on the HIP device (their data_ptr() is passed); streams are torch
streams (their HIP handle is passed).  Every compute step runs in libwos's HIP kernels; there is no
fallback: if libwos.so is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwos.so")

WOS_SVD_HESTENES, WOS_SVD_GRAM = 0, 1
WOS_OK, WOS_EINVAL, WOS_ENOMEM, WOS_EDEVICE, WOS_EBUSY, WOS_ETIMEOUT, WOS_ENOTSUP, WOS_ECANCELLED = range(8)
STATUS_NAMES = ["WOS_OK", "WOS_EINVAL", "WOS_ENOMEM", "WOS_EDEVICE", "WOS_EBUSY", "WOS_ETIMEOUT",
                "WOS_ENOTSUP", "WOS_ECANCELLED"]
WOS_FP64, WOS_FP32_GEOM_FP64_EXIT = 0, 1
WOS_RADIUS_WOE_BOUND, WOS_RADIUS_MAPPED_EXACT, WOS_RADIUS_MAPPED_BOUND = 0, 1, 2
WOS_TSVD_RANK, WOS_TSVD_DISCREPANCY, WOS_TIKHONOV = 0, 1, 2
WOS_STATS_WORDS = 8
STAT_NAMES = ["walks", "steps", "max_steps", "cap_hits", "escapes", "fp64_evals", "lane_slots", "reserved"]
WOS_DISK, WOS_ANNULUS, WOS_ELLIPSE, WOS_POLYGON, WOS_BALL, WOS_BOX, WOS_PERFORATED, WOS_PERFBOX, WOS_TRIMESH = range(9)
WOS_MAX_POLY_VERTS = 64
WOS_MAX_HOLES = 32
WOS_MAX_ELEMENTS = 16384


class WosError(RuntimeError):
    def __init__(self, status: int, message: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")
        self.status = status


class WosGeometry(C.Structure):
    _fields_ = [("dim", C.c_int32), ("kind", C.c_int32), ("params", C.c_double * 8),
                ("layout", C.c_int32 * 4), ("verts", C.POINTER(C.c_double)), ("n_verts", C.c_int32)]


class WosWalkParams(C.Structure):
    _fields_ = [("K", C.c_double * 9), ("eps", C.c_double), ("walk_begin", C.c_uint64),
                ("walk_end", C.c_uint64), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("precision", C.c_int32), ("radius_mode", C.c_int32), ("max_steps", C.c_uint32)]


class WosMeasureJob(C.Structure):
    _fields_ = [("geom", WosGeometry), ("walk", WosWalkParams), ("x_obs_dev", C.c_void_p),
                ("n_obs", C.c_int32), ("counts_dev", C.c_void_p), ("stats_dev", C.c_void_p),
                ("trace_dev", C.c_void_p)]


class WosTuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("walks_per_lane", C.c_int32), ("items", C.c_int32)]


WOS_ITEMS_AUTO, WOS_ITEMS_BLOCK, WOS_ITEMS_WAVE, WOS_ITEMS_POINT = 0, 1, 2, 3


class WosRegParams(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rank", C.c_int32), ("alpha", C.c_double),
                ("noise_delta", C.c_double), ("tau", C.c_double)]


class WosRequest(C.Structure):
    _fields_ = [("geom", WosGeometry), ("walk", WosWalkParams), ("x_obs_host", C.POINTER(C.c_double)),
                ("n_obs", C.c_int32), ("gamma1_mask_host", C.POINTER(C.c_uint8)),
                ("uD_host", C.POINTER(C.c_double)), ("u0_host", C.POINTER(C.c_double)),
                ("reg", WosRegParams), ("arrival_s", C.c_double)]


class WosResult(C.Structure):
    _fields_ = [("u1_host", C.POINTER(C.c_double)), ("pred_host", C.POINTER(C.c_double)),
                ("s_host", C.POINTER(C.c_double)), ("rank_used", C.c_int32), ("alpha_used", C.c_double),
                ("status", C.c_int32), ("t_arrive", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("walks", C.c_uint64), ("steps", C.c_uint64), ("svd_fallback", C.c_int32)]


class WosServeOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_inflight", C.c_int32), ("timeout_s", C.c_double),
                ("svd_mode", C.c_int32)]


# exported entry points: name -> (restype, argtypes)
_VP = C.c_void_p
_SIGS = {
    "wos_create": (C.c_int, [C.POINTER(_VP), C.c_int, C.c_size_t]),
    "wos_streams_create": (C.c_int, [_VP, C.c_int32, C.POINTER(_VP), C.POINTER(_VP)]),
    "wos_streams_destroy": (C.c_int, [_VP, _VP, _VP]),
    "wos_destroy": (C.c_int, [_VP]),
    "wos_last_error": (C.c_char_p, []),
    "wos_element_count": (C.c_int, [C.POINTER(WosGeometry), C.POINTER(C.c_int32)]),
    "wos_element_measures": (C.c_int, [C.POINTER(WosGeometry), C.POINTER(C.c_double)]),
    "wos_build_measure": (C.c_int, [_VP, C.POINTER(WosGeometry), C.POINTER(WosWalkParams), _VP, C.c_int32,
                                    _VP, _VP, _VP, _VP]),
    "wos_build_measure_noalloc": (C.c_int, [_VP, C.POINTER(WosGeometry), C.POINTER(WosWalkParams), _VP, C.c_int32,
                                            _VP, _VP, _VP, _VP]),
    "wos_build_measure_batch": (C.c_int, [_VP, C.POINTER(WosMeasureJob), C.c_int32, _VP]),
    "wos_set_tuning": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, C.POINTER(WosTuning)]),
    "wos_autotune": (C.c_int, [_VP, C.POINTER(WosMeasureJob), C.c_uint64, C.POINTER(WosTuning), _VP]),
    "wos_svd_create": (C.c_int, [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_uint8), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(_VP)]),
    "wos_svd_destroy": (C.c_int, [_VP, _VP]),
    "wos_svd": (C.c_int, [_VP, _VP, _VP, C.c_uint64, _VP]),
    "wos_svd_factors": (C.c_int, [_VP, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "wos_svd_info": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32), _VP]),
    "wos_svd_gram_check": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), _VP]),
    "wos_svd_timing": (C.c_int, [_VP, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_uint64)]),
    "wos_reconstruct": (C.c_int, [_VP, _VP, _VP, C.c_uint64, _VP, _VP, C.POINTER(WosRegParams), _VP, _VP, _VP,
                                  _VP, _VP]),
    "wos_reconstruct_sweep": (C.c_int, [_VP, _VP, _VP, C.c_uint64, _VP, _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "wos_eigenfunctions": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP]),
    "wos_density": (C.c_int, [_VP, _VP, C.c_int32, C.c_int32, C.c_uint64, _VP, _VP, _VP, _VP]),
    "wos_plan_create": (C.c_int, [_VP, C.POINTER(WosMeasureJob), _VP, _VP, _VP, C.POINTER(WosRegParams), _VP, _VP,
                                  _VP, _VP, C.POINTER(_VP)]),
    "wos_plan_create_batch": (C.c_int, [_VP, C.POINTER(WosMeasureJob), C.c_int32, C.POINTER(C.c_void_p)]),
    "wos_plan_launch": (C.c_int, [_VP, _VP]),
    "wos_diag_trig32": (C.c_int, [C.c_float, C.c_uint32, _VP, _VP, _VP]),
    "wos_plan_destroy": (C.c_int, [_VP]),
    "wos_serve": (C.c_int, [_VP, C.POINTER(WosRequest), C.c_int32, C.POINTER(WosResult), C.POINTER(WosServeOpts)]),
    "wos_serve_start": (C.c_int, [_VP, C.POINTER(WosServeOpts)]),
    "wos_serve_submit": (C.c_int, [_VP, C.POINTER(WosRequest), C.POINTER(C.c_uint64)]),
    "wos_serve_poll": (C.c_int, [_VP, C.c_uint64, C.POINTER(WosResult), C.c_int32]),
    "wos_serve_stop": (C.c_int, [_VP]),
}

_lib = None


def lib():
    """Loads libwos.so (raises if it was not built: there is no other implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2409_03686_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != WOS_OK:
        raise WosError(status, lib().wos_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device or host address of a torch tensor / numpy array (None passes NULL)."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ------------------------------------------------------------------------------- marshalling

def geometry(g) -> WosGeometry:
    """wos_geometry from an object with dim, kind, params, layout, verts (e.g. wos_inputs.Geometry)."""
    s = WosGeometry()
    s.dim, s.kind = int(g.dim), int(g.kind)
    for k, v in enumerate(g.params):
        s.params[k] = float(v)
    for k, v in enumerate(g.layout):
        s.layout[k] = int(v)
    if getattr(g, "verts", None) is not None:
        v = np.ascontiguousarray(np.asarray(g.verts, np.float64).ravel())
        s._keep = v
        s.verts = v.ctypes.data_as(C.POINTER(C.c_double))
        s.n_verts = (len(v) // (int(g.dim) + 1) if int(g.kind) in (WOS_PERFORATED, WOS_PERFBOX) else
                     len(v) // 9 if int(g.kind) == WOS_TRIMESH else len(v) // 2)
    return s


def walk_params(K, eps, walk_begin, walk_end, seed=0, instance=0, precision=WOS_FP64,
                radius_mode=WOS_RADIUS_WOE_BOUND, max_steps=0) -> WosWalkParams:
    w = WosWalkParams()
    K = np.asarray(K, np.float64)
    d = K.shape[0]
    for i in range(d):
        for j in range(d):
            w.K[i * 3 + j] = float(K[i, j])
    w.eps = float(eps)
    w.walk_begin, w.walk_end = int(walk_begin), int(walk_end)
    w.seed, w.instance = int(seed), int(instance)
    w.precision, w.radius_mode, w.max_steps = int(precision), int(radius_mode), int(max_steps)
    return w


def reg_params(kind=WOS_TSVD_RANK, rank=1, alpha=0.0, noise_delta=0.0, tau=1.1) -> WosRegParams:
    return WosRegParams(int(kind), int(rank), float(alpha), float(noise_delta), float(tau))


# ------------------------------------------------------------------------------- entry points

def wos_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = C.c_void_p()
    _check(lib().wos_create(C.byref(h), int(device), int(hbm_budget_bytes)))
    return h.value


def wos_destroy(ctx: int):
    _check(lib().wos_destroy(ctx))


def wos_streams_create(ctx, spectral_cus: int):
    """(walk_stream, spectral_stream) raw hipStream_t handles on disjoint CU sets."""
    a, b = C.c_void_p(), C.c_void_p()
    _check(lib().wos_streams_create(ctx, int(spectral_cus), C.byref(a), C.byref(b)))
    return a.value, b.value


def wos_streams_destroy(ctx, walk_stream, spectral_stream):
    _check(lib().wos_streams_destroy(ctx, walk_stream, spectral_stream))


def wos_last_error() -> str:
    return lib().wos_last_error().decode()


def wos_element_count(geom) -> int:
    n = C.c_int32()
    _check(lib().wos_element_count(C.byref(geometry(geom)), C.byref(n)))
    return n.value


def wos_element_measures(geom) -> np.ndarray:
    g = geometry(geom)
    n = C.c_int32()
    _check(lib().wos_element_count(C.byref(g), C.byref(n)))
    out = np.zeros(n.value)
    _check(lib().wos_element_measures(C.byref(g), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def wos_build_measure(ctx, geom, walk: WosWalkParams, x_obs_dev, n_obs, counts_dev, stats_dev=None,
                      trace_dev=None, stream=None):
    _check(lib().wos_build_measure(ctx, C.byref(geometry(geom)), C.byref(walk), _ptr(x_obs_dev), int(n_obs),
                                   _ptr(counts_dev), _ptr(stats_dev), _ptr(trace_dev), _stream(stream)))


def wos_build_measure_noalloc(ctx, geom, walk: WosWalkParams, x_obs_dev, n_obs, counts_dev, stats_dev=None,
                              trace_dev=None, stream=None):
    _check(lib().wos_build_measure_noalloc(ctx, C.byref(geometry(geom)), C.byref(walk), _ptr(x_obs_dev), int(n_obs),
                                           _ptr(counts_dev), _ptr(stats_dev), _ptr(trace_dev), _stream(stream)))


def measure_job(geom, walk: WosWalkParams, x_obs_dev, n_obs, counts_dev, stats_dev=None, trace_dev=None):
    J = WosMeasureJob()
    g = geometry(geom)
    J.geom = g
    J._keep = g  # keeps the polygon vertex array alive
    J.walk = walk
    J.x_obs_dev, J.n_obs = _ptr(x_obs_dev), int(n_obs)
    J.counts_dev, J.stats_dev, J.trace_dev = _ptr(counts_dev), _ptr(stats_dev), _ptr(trace_dev)
    return J


def wos_build_measure_batch(ctx, jobs: Sequence[WosMeasureJob], stream=None):
    arr = (WosMeasureJob * len(jobs))(*jobs)
    _check(lib().wos_build_measure_batch(ctx, arr, len(jobs), _stream(stream)))


def wos_set_tuning(ctx, dim, kind, precision, block, walks_per_lane, items=WOS_ITEMS_AUTO):
    t = WosTuning(int(block), int(walks_per_lane), int(items))
    _check(lib().wos_set_tuning(ctx, int(dim), int(kind), int(precision), C.byref(t)))


def wos_autotune(ctx, job: WosMeasureJob, sample_walks: int, stream=None):
    """(block, walks_per_lane, item mode) of the fastest candidate."""
    t = WosTuning()
    _check(lib().wos_autotune(ctx, C.byref(job), int(sample_walks), C.byref(t), _stream(stream)))
    return t.block, t.walks_per_lane, t.items


def wos_svd_create(ctx, n_obs, n_elem, gamma1_mask, sigma, nu=None) -> int:
    m = np.ascontiguousarray(np.asarray(gamma1_mask, np.uint8))
    s = np.ascontiguousarray(np.asarray(sigma, np.float64))
    nu_a = None if nu is None else np.ascontiguousarray(np.asarray(nu, np.float64))
    h = C.c_void_p()
    _check(lib().wos_svd_create(ctx, int(n_obs), int(n_elem), m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                s.ctypes.data_as(C.POINTER(C.c_double)),
                                None if nu_a is None else nu_a.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
    return h.value


def wos_svd_destroy(ctx, h):
    _check(lib().wos_svd_destroy(ctx, h))


def wos_svd(ctx, h, counts_dev, n_walks, stream=None):
    _check(lib().wos_svd(ctx, h, _ptr(counts_dev), int(n_walks), _stream(stream)))


def wos_svd_factors(h):
    U, s, V = C.c_void_p(), C.c_void_p(), C.c_void_p()
    m, n, k = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().wos_svd_factors(h, C.byref(U), C.byref(s), C.byref(V), C.byref(m), C.byref(n), C.byref(k)))
    return U.value, s.value, V.value, m.value, n.value, k.value


def wos_svd_info(h, stream=None):
    """(sweeps, error flags, method) of the last SVD; method is WOS_SVD_HESTENES or WOS_SVD_GRAM."""
    sw, er, me = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().wos_svd_info(h, C.byref(sw), C.byref(er), C.byref(me), _stream(stream)))
    return sw.value, er.value, me.value


def wos_svd_gram_check(h, stream=None):
    """(Gram-path Jacobi sweeps, its error flags, orthogonality statistic, residual certificate) of the
    last wos_svd."""
    sw, er, ck, rs = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
    _check(lib().wos_svd_gram_check(h, C.byref(sw), C.byref(er), C.byref(ck), C.byref(rs), _stream(stream)))
    return sw.value, er.value, ck.value, rs.value


def wos_svd_timing(h):
    """(Jacobi ms, whole SVD ms, plane rotations) of the last wos_svd outside stream capture."""
    jm, tm, nr = C.c_float(), C.c_float(), C.c_uint64()
    _check(lib().wos_svd_timing(h, C.byref(jm), C.byref(tm), C.byref(nr)))
    return jm.value, tm.value, nr.value


def wos_reconstruct(ctx, h, counts_dev, n_walks, uD_dev, u0_dev, reg: WosRegParams, u1_dev, pred_dev=None,
                    rank_used_dev=None, alpha_used_dev=None, stream=None):
    _check(lib().wos_reconstruct(ctx, h, _ptr(counts_dev), int(n_walks), _ptr(uD_dev), _ptr(u0_dev), C.byref(reg),
                                 _ptr(u1_dev), _ptr(pred_dev), _ptr(rank_used_dev), _ptr(alpha_used_dev),
                                 _stream(stream)))


def wos_reconstruct_sweep(ctx, h, counts_dev, n_walks, uD_dev, u0_dev, r_max, u1_dev, pred_dev=None,
                          resid_dev=None, stream=None):
    _check(lib().wos_reconstruct_sweep(ctx, h, _ptr(counts_dev), int(n_walks), _ptr(uD_dev), _ptr(u0_dev),
                                       int(r_max), _ptr(u1_dev), _ptr(pred_dev), _ptr(resid_dev),
                                       _stream(stream)))


def wos_eigenfunctions(ctx, h, n_fun, lambda_dev=None, ef_dev=None, stream=None):
    _check(lib().wos_eigenfunctions(ctx, h, int(n_fun), _ptr(lambda_dev), _ptr(ef_dev), _stream(stream)))


def wos_density(ctx, counts_dev, n_obs, n_elem, n_walks, sigma_dev, rho_dev=None, mean_dev=None, stream=None):
    _check(lib().wos_density(ctx, _ptr(counts_dev), int(n_obs), int(n_elem), int(n_walks), _ptr(sigma_dev),
                             _ptr(rho_dev), _ptr(mean_dev), _stream(stream)))


def wos_plan_create(ctx, job: WosMeasureJob, svd=None, uD_dev=None, u0_dev=None, reg: Optional[WosRegParams] = None,
                    u1_dev=None, pred_dev=None, rank_used_dev=None, alpha_used_dev=None) -> int:
    p = C.c_void_p()
    _check(lib().wos_plan_create(ctx, C.byref(job), svd, _ptr(uD_dev), _ptr(u0_dev),
                                 None if reg is None else C.byref(reg), _ptr(u1_dev), _ptr(pred_dev),
                                 _ptr(rank_used_dev), _ptr(alpha_used_dev), C.byref(p)))
    return p.value


def wos_plan_create_batch(ctx, jobs: Sequence[WosMeasureJob]) -> int:
    arr = (WosMeasureJob * len(jobs))(*jobs)
    p = C.c_void_p()
    _check(lib().wos_plan_create_batch(ctx, arr, len(jobs), C.byref(p)))
    return p.value


def wos_diag_trig32(offset, n, cos_dev, sin_dev, stream=None):
    _check(lib().wos_diag_trig32(float(offset), int(n), _ptr(cos_dev), _ptr(sin_dev), _stream(stream)))


def wos_plan_launch(plan, stream=None):
    _check(lib().wos_plan_launch(plan, _stream(stream)))


def wos_plan_destroy(plan):
    _check(lib().wos_plan_destroy(plan))


def wos_serve(ctx, requests: Sequence[WosRequest], results: Sequence[WosResult], hbm_budget_bytes=0,
              max_inflight=4, timeout_s=0.0, svd_mode=0):
    req = (WosRequest * len(requests))(*requests)
    res = (WosResult * len(results))(*results)
    opts = WosServeOpts(int(hbm_budget_bytes), int(max_inflight), float(timeout_s), int(svd_mode))
    _check(lib().wos_serve(ctx, req, len(requests), res, C.byref(opts)))
    return list(res)


def wos_serve_start(ctx, hbm_budget_bytes=0, max_inflight=4, timeout_s=0.0, svd_mode=0):
    opts = WosServeOpts(int(hbm_budget_bytes), int(max_inflight), float(timeout_s), int(svd_mode))
    _check(lib().wos_serve_start(ctx, C.byref(opts)))


def wos_serve_submit(ctx, request: WosRequest) -> int:
    t = C.c_uint64()
    _check(lib().wos_serve_submit(ctx, C.byref(request), C.byref(t)))
    return t.value


def wos_serve_poll(ctx, ticket: int, result: WosResult, wait_ms: int = -1) -> bool:
    """True when the request finished (result filled, ticket released), False if still running."""
    st = lib().wos_serve_poll(ctx, int(ticket), C.byref(result), int(wait_ms))
    if st == WOS_EBUSY:
        return False
    _check(st)
    return True


def wos_serve_stop(ctx):
    _check(lib().wos_serve_stop(ctx))


# ------------------------------------------------------------------------------- torch helpers

def walk_params_of(inst, walk_begin=0, walk_end=None, precision=None, radius_mode=None) -> WosWalkParams:
    """wos_walk_params of a wos_inputs.Instance."""
    return walk_params(inst.K, inst.eps, walk_begin, inst.n_walks if walk_end is None else walk_end,
                       seed=inst.seed, instance=inst.instance_id,
                       precision=inst.precision if precision is None else precision,
                       radius_mode=inst.radius_mode if radius_mode is None else radius_mode,
                       max_steps=inst.max_steps)


def device_inputs(inst, device="cuda"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(inst.x_obs, np.float64), device=device)


def run_measure(ctx, inst, walk_begin=0, walk_end=None, precision=None, trace=False, stream=None,
                counts=None, stats=None, x_dev=None):
    """Allocates (or accumulates into) counts / stats tensors and enqueues wos_build_measure."""
    import torch
    M = wos_element_count(inst.geom)
    n = inst.x_obs.shape[0]
    we = inst.n_walks if walk_end is None else walk_end
    x = device_inputs(inst) if x_dev is None else x_dev
    if counts is None:
        counts = torch.zeros((n, M), dtype=torch.int32, device=x.device)
    if stats is None:
        stats = torch.zeros(WOS_STATS_WORDS, dtype=torch.int64, device=x.device)
    tr = torch.zeros((n, we - walk_begin, 2), dtype=torch.int32, device=x.device) if trace else None
    w = walk_params_of(inst, walk_begin, we, precision)
    wos_build_measure(ctx, inst.geom, w, x, n, counts, stats, tr, stream)
    return counts, stats, tr, x


def stats_dict(stats) -> dict:
    v = [int(t) for t in stats.cpu().tolist()]
    return dict(zip(STAT_NAMES, v))


_hip = None


def device_to_numpy(ptr: int, count: int, dtype) -> np.ndarray:
    """Copies `count` elements at device address `ptr` (e.g. an SVD factor) to a numpy array."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the HIP runtime torch was built with)
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipDeviceSynchronize.restype = C.c_int
    out = np.empty(int(count), dtype)
    if count:
        if _hip.hipDeviceSynchronize() != 0 or _hip.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) != 0:
            raise WosError(WOS_EDEVICE, "hipMemcpy from device failed")
    return out


def svd_factors_numpy(h):
    """(U m x k, s k, V n x k) of an SVD handle as numpy arrays."""
    U, s, V, m, n, k = wos_svd_factors(h)
    Uh = device_to_numpy(U, m * k, np.float64).reshape(k, m).T
    sh = device_to_numpy(s, k, np.float64)
    Vh = device_to_numpy(V, n * k, np.float64).reshape(k, n).T
    return Uh, sh, Vh
