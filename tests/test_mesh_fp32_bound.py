"""The FP32 error bounds of the triangle-mesh distance and mapped-exact radius: a CPU replay of the device's FP32 operation
sequence (the record's corner, edges, inverse squared lengths, unit normal and in-plane edge normals
rounded to FP32, fused multiply-adds rounded once) against the oracle's FP64 distance.  The library
subtracts 2 delta = 2 * 2^-18 L (L the largest coordinate magnitude) from every FP32 radius and
decides the exit band in FP64 within delta of eps, so the replayed error must stay well below
delta = 64 units of 2^-24 L."""
import numpy as np

import wos_inputs as wi
from oracle import walks

f32 = np.float32


def _fma(a, b, c):
    # the product of two FP32 numbers is exact in FP64; the sum is then rounded once to FP32 (a
    # double rounding that can differ from a true fused multiply-add by one unit at most)
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def _records(T):
    a, b, c = T[:, 0], T[:, 1], T[:, 2]
    e = np.stack([b - a, c - b, a - c], 1)
    n = np.cross(e[:, 0], e[:, 1])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    m = np.cross(n[:, None, :], e)
    inv = 1.0 / (e ** 2).sum(2)
    return a.astype(f32), e.astype(f32), inv.astype(f32), n.astype(f32), m.astype(f32)


def _dist32(rec, x):
    a, e, inv, n, m = rec
    x = x.astype(f32)
    ap = (x[:, None, :] - a[None]).astype(f32)
    bp = (ap - e[None, :, 0]).astype(f32)
    cp = (bp - e[None, :, 1]).astype(f32)

    def dot(u, v):  # fmaf(u2, v2, fmaf(u1, v1, u0 * v0))
        return _fma(u[..., 2], v[..., 2], _fma(u[..., 1], v[..., 1], (u[..., 0] * v[..., 0]).astype(f32)))

    s0, s1, s2 = dot(m[None, :, 0], ap), dot(m[None, :, 1], bp), dot(m[None, :, 2], cp)
    dp = dot(n[None], ap)

    def seg(w, k):
        ek = e[None, :, k]
        t = (dot(ek, w) * inv[None, :, k]).astype(f32)
        t = np.clip(t, f32(0), f32(1))
        q = np.stack([_fma(-t, ek[..., j], w[..., j]) for j in range(3)], -1)
        return dot(q, q)

    de = np.minimum(seg(ap, 0), np.minimum(seg(bp, 1), seg(cp, 2)))
    inside = (s0 >= 0) & (s1 >= 0) & (s2 >= 0)
    d2 = np.where(inside, (dp * dp).astype(f32), de).min(1)
    return np.sqrt(d2.astype(np.float64))  # the hardware square root: within 1 unit


def test_fp32_mesh_distance_stays_within_its_bound():
    rng = np.random.default_rng(41)
    worst = 0.0
    for T, shift in ((wi.box_mesh([0, 0, 0], [1, 1, 1], 6), 0.0), (wi.sphere_mesh([0, 0, 0], 1.0, 2), 0.0),
                     (wi.l_prism_mesh(4), 0.0), (wi.l_prism_mesh(4), 7.3)):
        T = T + shift
        g = wi.Geometry(3, wi.TRIMESH, (), (1,), verts=T)
        L = np.abs(T).max()
        x = wi.sample_points(g, 1500, rng)
        # and points close to the surface (near faces, edges and corners), where the walks stop
        k = rng.integers(0, len(T), 1500)
        bc = rng.dirichlet([0.3, 0.3, 0.3], 1500)
        y = (bc[:, :, None] * T[k]).sum(1)
        y += rng.standard_normal((1500, 3)) * 1e-3
        y = y[walks.geom_eval(g, y)[0] > 0]
        P = np.concatenate([x, y])
        d64, _ = walks.geom_eval(g, P)
        d32 = _dist32(_records(T), P)
        err = np.abs(d32 - d64).max() / (L * 2.0 ** -24)
        worst = max(worst, err)
    print(f"largest FP32 mesh-distance error: {worst:.2f} units of 2^-24 L")
    assert worst <= 8.0, worst


def test_fp32_mapped_mesh_radius_stays_within_its_bound():
    """The FP32 mapped-exact radius of a mesh: S^{-1} x formed in FP32 (fused multiply-adds on the
    rounded S^{-1}) and the FP32 distance to the FP32 records of the mapped triangles, against the
    oracle's FP64 mapped radius.  The library subtracts 2^-17 L_m (L_m the largest mapped coordinate
    magnitude, 128 units of 2^-24 L_m); the replayed error must stay far below it."""
    rng = np.random.default_rng(42)
    K = np.array([[1.0, 0.3, 0.1], [0.3, 0.5, -0.2], [0.1, -0.2, 0.25]])
    _, _, S = walks.instance_setup(K, 3)
    Si = np.linalg.inv(S[:3, :3])
    Sif = Si.astype(f32)
    worst = 0.0
    for T in (wi.l_prism_mesh(4), wi.box_mesh([0, 0, 0], [1, 1, 1], 6) + 2.5):
        g = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=T)
        MT = T @ Si.T
        Lm = np.abs(MT).max()
        x = wi.sample_points(g, 1200, rng)
        xf = x.astype(f32)
        y = np.stack([_fma(np.full(len(x), Sif[k, 2]), xf[:, 2],
                           _fma(np.full(len(x), Sif[k, 1]), xf[:, 1], (Sif[k, 0] * xf[:, 0]).astype(f32)))
                      for k in range(3)], 1)
        r32 = _dist32(_records(MT), y)
        r64 = walks.step_radii(g, S, x, 1)
        worst = max(worst, np.abs(r32 - r64).max() / (Lm * 2.0 ** -24))
    print(f"largest FP32 mapped mesh radius error: {worst:.2f} units of 2^-24 L_m")
    assert worst <= 16.0, worst
