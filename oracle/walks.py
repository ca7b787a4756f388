"""Oracle walk estimator: Python side (instance set-up, element measures, ctypes to the C core).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


class OgGeom(C.Structure):
    _fields_ = [("dim", C.c_int32), ("kind", C.c_int32), ("p", C.c_double * 8),
                ("layout", C.c_int32 * 4), ("verts", C.POINTER(C.c_double)),
                ("n_verts", C.c_int32), ("nodes", C.c_void_p * 2)]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        L.oracle_build_measure.restype = C.c_int
        L.oracle_build_measure.argtypes = [
            C.POINTER(OgGeom), C.c_int32, C.POINTER(C.c_double), C.c_double, C.c_int,
            C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_double), C.c_int32,
            C.c_uint64, C.c_uint64, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
            C.POINTER(C.c_int32), C.POINTER(C.c_uint32), C.c_int]
        L.oracle_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.oracle_u53.restype = C.c_double
        L.oracle_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_geom_eval.argtypes = [C.POINTER(OgGeom), C.POINTER(C.c_double), C.c_int32,
                                       C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.oracle_directions.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_uint32, C.POINTER(C.c_double)]
        _LIB = L
    return _LIB


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def make_geom(g):
    """og_geom from a wos_inputs.Geometry (keeps the vertex array alive on the struct)."""
    s = OgGeom()
    s.dim, s.kind = int(g.dim), int(g.kind)
    for k, v in enumerate(g.params):
        s.p[k] = float(v)
    for k, v in enumerate(g.layout):
        s.layout[k] = int(v)
    if g.verts is not None:
        import wos_inputs as wi
        v = np.ascontiguousarray(np.asarray(g.verts, np.float64).ravel())
        s._verts = v
        s.verts = _ptr(v, C.c_double)
        s.n_verts = (len(v) // (g.dim + 1) if g.kind in (wi.PERFORATED, wi.PERFBOX) else
                     len(v) // 9 if g.kind == wi.TRIMESH else len(v) // 2)
    return s


def instance_setup(K, dim):
    """lambda_max(K), Khat = K / lambda_max and S = Khat^{1/2} (symmetric principal root).

    Section 4.2 takes the largest eigenvalue of K to be 1 without loss of generality; the walk
    X + dist * Khat^{1/2} U stays in the Euclidean ball of radius dist only under that scaling."""
    K = np.asarray(K, np.float64)[:dim, :dim]
    w, Q = np.linalg.eigh(K)
    lam = w[-1]
    S = (Q * np.sqrt(w / lam)) @ Q.T
    S3 = np.zeros((3, 3))
    S3[:dim, :dim] = S
    return lam, K / lam, S3


def sphere_cell_measures(nz, nphi, R) -> np.ndarray:
    """Areas of the cells of a sphere of radius R: nz x nphi equal-area (z band, azimuth) cells, or,
    for the layout (n, 0), the Voronoi cells of n Bauer nodes (scipy's spherical Voronoi diagram;
    on the sphere the extrinsic Voronoi cells of nodes on it are the spherical ones)."""
    if nphi:
        return np.full(nz * nphi, 4 * np.pi * R * R / (nz * nphi))
    from scipy.spatial import SphericalVoronoi
    import wos_inputs as wi
    sv = SphericalVoronoi(wi.bauer_spiral(nz), radius=1.0)
    return sv.calculate_areas() * R * R


def element_measures(g) -> np.ndarray:
    """sigma(omega_j): surface measure of each boundary element (eq. boundary_weights)."""
    import wos_inputs as wi
    M = g.n_elem
    if g.kind == wi.DISK:
        return np.full(M, 2 * np.pi * g.params[2] / M)
    if g.kind == wi.ANNULUS:
        mo, mi = g.layout
        return np.concatenate([np.full(mo, 2 * np.pi * g.params[3] / mo),
                               np.full(mi, 2 * np.pi * g.params[2] / mi)])
    if g.kind == wi.ELLIPSE:
        a, b = g.params[2], g.params[3]
        xg, wg = np.polynomial.legendre.leggauss(64)
        out = np.empty(M)
        for j in range(M):
            t0, t1 = 2 * np.pi * j / M, 2 * np.pi * (j + 1) / M
            t = 0.5 * (t1 - t0) * xg + 0.5 * (t1 + t0)
            out[j] = 0.5 * (t1 - t0) * np.sum(wg * np.sqrt(a * a * np.sin(t) ** 2 + b * b * np.cos(t) ** 2))
        return out
    if g.kind == wi.POLYGON:
        v = np.asarray(g.verts, float)
        L = np.sqrt(((np.roll(v, -1, 0) - v) ** 2).sum(1)).sum()
        return np.full(M, L / M)
    if g.kind == wi.BALL:
        return sphere_cell_measures(g.layout[0], g.layout[1], g.params[3])
    if g.kind == wi.TRIMESH:  # the areas |(b - a) x (c - a)| / 2 of each element's triangles
        T = np.asarray(g.verts, float).reshape(-1, 3, 3)
        area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
        return area.reshape(M, int(g.layout[0])).sum(1)
    if g.kind in (wi.PERFORATED, wi.PERFBOX):
        # the outer boundary's cells, then each hole's: arcs 2 pi r / m, or sphere cells 4 pi r^2 / (nz nphi)
        d = g.dim
        holes = np.asarray(g.verts, float).reshape(-1, d + 1)
        if g.kind == wi.PERFORATED:
            R = g.params[d]
            outer = (np.full(g.layout[0], 2 * np.pi * R / g.layout[0]) if d == 2 else
                     sphere_cell_measures(g.layout[0], g.layout[1], R))
            hc = (g.layout[1],) if d == 2 else (g.layout[2], g.layout[3])
        else:
            outer = element_measures(wi.Geometry(d, wi.BOX, g.params, (g.layout[0],)))
            hc = tuple(g.layout[1:d])
        if d == 2:
            return np.concatenate([outer] + [np.full(hc[0], 2 * np.pi * r / hc[0]) for r in holes[:, d]])
        return np.concatenate([outer] + [sphere_cell_measures(hc[0], hc[1], r) for r in holes[:, d]])
    if g.kind == wi.BOX:
        d, n = g.dim, g.layout[0]
        lo, hi = np.array(g.params[:d]), np.array(g.params[d:2 * d])
        h = (hi - lo) / n
        out = []
        for f in range(2 * d):
            a = f // 2
            others = [b for b in range(d) if b != a]
            out.append(np.full(n ** (d - 1), float(np.prod(h[others]))))
        return np.concatenate(out)
    raise ValueError(g.kind)


def build_measure(geom, K, x_obs, eps, seed=0, instance_id=0, radius_mode=0, max_steps=10000,
                  walk_begin=0, walk_end=1000, threads=None, trace=False, counts=None, point_ids=None):
    """counts[i, j] = #{k in [walk_begin, walk_end): walk (i, k) stops in element j}.

    Returns (counts uint32 [n_obs, M], stats dict, trace or None)."""
    L = lib()
    g = make_geom(geom)
    M = geom.n_elem
    x = np.ascontiguousarray(np.asarray(x_obs, np.float64).reshape(-1, geom.dim))
    n_obs = x.shape[0]
    _, _, S = instance_setup(K, geom.dim)
    S = np.ascontiguousarray(S)
    if counts is None:
        counts = np.zeros((n_obs, M), np.uint32)
    st = np.zeros(5, np.uint64)
    tr = np.zeros((n_obs, walk_end - walk_begin, 2), np.int32) if trace else None
    nthr = threads or len(os.sched_getaffinity(0))
    pid = None
    if point_ids is not None:
        pid = np.ascontiguousarray(np.asarray(point_ids, np.uint32))
        assert pid.shape == (n_obs,)
    rc = L.oracle_build_measure(C.byref(g), M, _ptr(S, C.c_double), float(eps), int(radius_mode),
                                seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF, int(instance_id),
                                int(max_steps), _ptr(x, C.c_double), n_obs, int(walk_begin),
                                int(walk_end), _ptr(counts, C.c_uint32), _ptr(st, C.c_uint64),
                                _ptr(tr, C.c_int32) if trace else None,
                                _ptr(pid, C.c_uint32) if pid is not None else None, int(nthr))
    if rc != 0:
        raise ValueError("oracle_build_measure rejected its arguments")
    stats = dict(walks=int(st[0]), steps=int(st[1]), max_steps=int(st[2]), cap_hits=int(st[3]),
                 escapes=int(st[4]))
    return counts, stats, tr


def build_instance(inst, walk_begin=0, walk_end=None, **kw):
    we = inst.n_walks if walk_end is None else walk_end
    return build_measure(inst.geom, inst.K, inst.x_obs, inst.eps, seed=inst.seed,
                         instance_id=inst.instance_id, radius_mode=inst.radius_mode,
                         max_steps=inst.max_steps, walk_begin=walk_begin, walk_end=we, **kw)


def philox(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    L.oracle_philox(c, k, o)
    return tuple(int(v) for v in o)


def u53(hi, lo):
    return lib().oracle_u53(hi, lo)


def directions(dim, n, k=0, i=0, inst=0, seed=0):
    out = np.zeros((n, dim))
    lib().oracle_directions(dim, n, k, i, inst, seed & 0xFFFFFFFF, seed >> 32, _ptr(out, C.c_double))
    return out


def geom_eval(geom, pts):
    g = make_geom(geom)
    p = np.ascontiguousarray(np.asarray(pts, np.float64).reshape(-1, geom.dim))
    d = np.zeros(p.shape[0])
    e = np.zeros(p.shape[0], np.int32)
    lib().oracle_geom_eval(C.byref(g), _ptr(p, C.c_double), p.shape[0], _ptr(d, C.c_double),
                           _ptr(e, C.c_int32))
    return d, e


def step_radii(geom, S, pts, radius_mode):
    """Step radius of the given mode at each point (NaN where the mode does not apply)."""
    g = make_geom(geom)
    S = np.ascontiguousarray(np.asarray(S, np.float64))
    p = np.ascontiguousarray(np.asarray(pts, np.float64).reshape(-1, geom.dim))
    r = np.zeros(p.shape[0])
    lib().oracle_step_radii(C.byref(g), _ptr(S, C.c_double), C.c_int(radius_mode), _ptr(p, C.c_double),
                            C.c_int32(p.shape[0]), _ptr(r, C.c_double))
    return r


def walk_exits(geom, S, x0, eps, n, i=0, seed=0, instance_id=0, radius_mode=0, max_steps=10000):
    """Stop positions of n walks from x0 with the given step matrix S (3x3, row-major)."""
    L = lib()
    L.oracle_walk_exits.restype = C.c_int
    g = make_geom(geom)
    S = np.ascontiguousarray(np.asarray(S, np.float64))
    x = np.ascontiguousarray(np.asarray(x0, np.float64))
    out = np.zeros((n, geom.dim))
    rc = L.oracle_walk_exits(C.byref(g), _ptr(S, C.c_double), C.c_double(eps), C.c_int(radius_mode),
                             C.c_uint32(seed & 0xFFFFFFFF), C.c_uint32(seed >> 32),
                             C.c_uint32(instance_id), C.c_uint32(max_steps), _ptr(x, C.c_double),
                             C.c_uint32(i), C.c_uint64(0), C.c_uint64(n), _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("oracle_walk_exits rejected its arguments")
    return out
