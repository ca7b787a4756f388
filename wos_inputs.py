"""Seeded synthetic inputs shared by the oracle, the tests, the smoke check and the benchmark.

This module only *describes* problem instances: domain shapes, boundary element layouts, the
Gamma_0 / Gamma_1 split, conductivity matrices, observation points, walk budgets and boundary
data.  It contains none of the estimator's arithmetic (no walks, no distances used by a walk,
no binning, no linear algebra of the reconstruction), so both the HIP path and the CPU oracle
can take the very same instance from here without sharing any of the method.

Geometry kinds (codes shared by the C ABI and the oracle):

  DISK     params (cx, cy, R)                      layout (M,)            M arcs, counter-clockwise from angle 0
  ANNULUS  params (cx, cy, R_in, R_out)            layout (M_out, M_in)   outer arcs first, then inner arcs
  ELLIPSE  params (cx, cy, a, b)                   layout (M,)            equal steps of the eccentric angle
  POLYGON  verts  (n, 2), one counter-clockwise loop  layout (M,)         equal pieces of perimeter
  BALL     params (cx, cy, cz, R)                  layout (n_z, n_phi)    equal-area (z, phi) cells
  BOX      params (lo_0..lo_{d-1}, hi_0..hi_{d-1}) layout (n,)            n^(d-1) patches per face
  PERFORATED a disc / ball with k disjoint round holes.  params (centre, R) of the outer disc or
           ball, verts (k, dim + 1) rows (centre, r) of the holes.  2D layout (M_out, M_hole, k):
           outer arcs first, then M_hole arcs per hole in hole order, all counter-clockwise from
           angle 0 about their own centre.  3D layout (nz_out, nphi_out, nz_hole, nphi_hole), k the
           number of verts rows: equal-area (z, phi) cells of the outer sphere, then of each hole
  PERFBOX  a box with k disjoint round holes.  params (lo, hi) as BOX, verts as PERFORATED.
           2D layout (n, M_hole), 3D layout (n, nz_hole, nphi_hole): the box's face patches
           first, then each hole's cells as above

The paper's problem statement (Section 1.1, the discrete inverse problem with interior data) fixes
what an instance holds: the domain D, its boundary split into an accessible part Gamma_0 and an
inaccessible part Gamma_1, a constant SPD conductivity K, interior points x^D, and data u^D, u^0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

DISK, ANNULUS, ELLIPSE, POLYGON, BALL, BOX, PERFORATED, PERFBOX, TRIMESH = 0, 1, 2, 3, 4, 5, 6, 7, 8
KIND_NAMES = {DISK: "disk", ANNULUS: "annulus", ELLIPSE: "ellipse", POLYGON: "polygon",
              BALL: "ball", BOX: "box", PERFORATED: "perforated", PERFBOX: "perforated box",
              TRIMESH: "triangle mesh"}

FP64 = 0
FP32_GEOM_FP64_EXIT = 1
RADIUS_WOE_BOUND = 0
RADIUS_MAPPED_EXACT = 1
RADIUS_MAPPED_BOUND = 2   # discs, annuli, balls, ellipses: support bound of the inscribed ellipsoid


@dataclasses.dataclass
class Geometry:
    dim: int
    kind: int
    params: tuple = ()
    layout: tuple = ()
    verts: Optional[np.ndarray] = None
    gamma1_mask: Optional[np.ndarray] = None  # uint8, length n_elem, 1 = Gamma_1

    @property
    def n_holes(self) -> int:
        return 0 if self.verts is None else int(np.asarray(self.verts).size // (self.dim + 1))

    @property
    def n_tri(self) -> int:
        """Triangles of a TRIMESH geometry (verts holds them as (n_tri, 3, 3) corner coordinates)."""
        return int(np.asarray(self.verts).size // 9)

    @property
    def n_elem(self) -> int:
        if self.kind == TRIMESH:
            return self.n_tri // int(self.layout[0])
        return element_count(self.dim, self.kind, self.layout, self.n_holes)


@dataclasses.dataclass
class Instance:
    """One measure-building problem: geometry + conductivity + points + walk budget."""
    geom: Geometry
    K: np.ndarray            # (dim, dim) SPD, as given (not normalised)
    x_obs: np.ndarray        # (n_obs, dim) float64
    n_walks: int
    eps: float = 1e-4
    seed: int = 0
    instance_id: int = 0
    precision: int = FP64
    radius_mode: int = RADIUS_WOE_BOUND
    max_steps: int = 10000
    name: str = ""
    uD: Optional[np.ndarray] = None   # interior data at x_obs
    u0: Optional[np.ndarray] = None   # Gamma_0 data, one value per Gamma_0 element (index order)
    u_exact_g1: Optional[np.ndarray] = None  # exact data at Gamma_1 element reference points
    noise_delta: float = 0.0          # expected norm of nu * noise(b), for the discrepancy principle


def _sphere_cells(nz: int, nphi: int) -> int:
    """Cells of a sphere: nz x nphi (z band, azimuth) cells, or, for the layout (n, 0), the Voronoi
    cells of n nodes of Bauer's spiral."""
    return nz if nphi == 0 else nz * nphi


def element_count(dim: int, kind: int, layout, n_holes: int = 0) -> int:
    layout = tuple(int(v) for v in layout)
    if kind in (DISK, ELLIPSE, POLYGON):
        return layout[0]
    if kind == ANNULUS:
        return layout[0] + layout[1]
    if kind == BALL:
        return _sphere_cells(layout[0], layout[1])
    if kind == BOX:
        return 2 * dim * layout[0] ** (dim - 1)
    if kind == PERFORATED:
        if dim == 2:
            return layout[0] + layout[1] * layout[2]
        return _sphere_cells(layout[0], layout[1]) + n_holes * _sphere_cells(layout[2], layout[3])
    if kind == PERFBOX:
        if dim == 2:
            return 4 * layout[0] + n_holes * layout[1]
        return 6 * layout[0] ** 2 + n_holes * _sphere_cells(layout[1], layout[2])
    raise ValueError(f"unknown geometry kind {kind}")


def _sphere_cell_centres(c, R, nz, nphi):
    if nphi == 0:  # Voronoi cells: their nodes
        return np.asarray(c, float) + R * bauer_spiral(nz)
    iz, ip = np.meshgrid(np.arange(nz), np.arange(nphi), indexing="ij")
    z = 1 - 2 * (iz.ravel() + 0.5) / nz
    ph = (ip.ravel() + 0.5) * 2 * np.pi / nphi
    rr = np.sqrt(1 - z * z)
    return np.stack([c[0] + R * rr * np.cos(ph), c[1] + R * rr * np.sin(ph), c[2] + R * z], 1)


def _circle_arc_centres(c, R, m):
    t = (np.arange(m) + 0.5) * 2 * np.pi / m
    return np.stack([c[0] + R * np.cos(t), c[1] + R * np.sin(t)], 1)


def _hole_ref_points(g: "Geometry", cells) -> list:
    d = g.dim
    out = []
    for h in np.asarray(g.verts, float).reshape(-1, d + 1):
        out.append(_circle_arc_centres(h[:2], h[2], cells[0]) if d == 2
                   else _sphere_cell_centres(h[:3], h[3], cells[0], cells[1]))
    return out


# --------------------------------------------------------------------------------------------
# Element reference points (where boundary data is sampled).  These are input definitions: the
# point of each element at which the data u^0 / exact u is given (arc mid-angle, patch centre).
# --------------------------------------------------------------------------------------------

def element_ref_points(g: Geometry) -> np.ndarray:
    M = g.n_elem
    if g.kind == DISK:
        cx, cy, R = g.params
        t = (np.arange(M) + 0.5) * 2 * np.pi / M
        return np.stack([cx + R * np.cos(t), cy + R * np.sin(t)], 1)
    if g.kind == ANNULUS:
        cx, cy, r_in, r_out = g.params
        pts = []
        for R, m in ((r_out, g.layout[0]), (r_in, g.layout[1])):
            t = (np.arange(m) + 0.5) * 2 * np.pi / m
            pts.append(np.stack([cx + R * np.cos(t), cy + R * np.sin(t)], 1))
        return np.concatenate(pts, 0)
    if g.kind == ELLIPSE:
        cx, cy, a, b = g.params
        t = (np.arange(M) + 0.5) * 2 * np.pi / M
        return np.stack([cx + a * np.cos(t), cy + b * np.sin(t)], 1)
    if g.kind == PERFORATED:
        if g.dim == 2:
            outer = _circle_arc_centres(g.params[:2], g.params[2], g.layout[0])
            return np.concatenate([outer] + _hole_ref_points(g, (g.layout[1],)), 0)
        outer = _sphere_cell_centres(g.params[:3], g.params[3], g.layout[0], g.layout[1])
        return np.concatenate([outer] + _hole_ref_points(g, (g.layout[2], g.layout[3])), 0)
    if g.kind == PERFBOX:
        box = element_ref_points(Geometry(g.dim, BOX, g.params, (g.layout[0],)))
        return np.concatenate([box] + _hole_ref_points(g, tuple(g.layout[1:])), 0)
    if g.kind == POLYGON:
        v = np.asarray(g.verts, float)
        seg = np.roll(v, -1, 0) - v
        ln = np.sqrt((seg ** 2).sum(1))
        cum = np.concatenate([[0.0], np.cumsum(ln)])
        L = cum[-1]
        s = (np.arange(M) + 0.5) * L / M
        e = np.searchsorted(cum, s, side="right") - 1
        t = (s - cum[e]) / ln[e]
        return v[e] + t[:, None] * seg[e]
    if g.kind == TRIMESH:  # area-weighted centroid of each element's triangles
        T = np.asarray(g.verts, float).reshape(-1, 3, 3)
        area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
        cen = T.mean(1)
        gsz = int(g.layout[0])
        w = area.reshape(-1, gsz)
        return (cen.reshape(-1, gsz, 3) * w[:, :, None]).sum(1) / w.sum(1)[:, None]
    if g.kind == BALL and g.layout[1] == 0:
        return _sphere_cell_centres(g.params[:3], g.params[3], g.layout[0], 0)
    if g.kind == BALL:
        cx, cy, cz, R = g.params
        nz, nphi = g.layout
        iz, ip = np.meshgrid(np.arange(nz), np.arange(nphi), indexing="ij")
        z = 1 - 2 * (iz.ravel() + 0.5) / nz
        ph = (ip.ravel() + 0.5) * 2 * np.pi / nphi
        rr = np.sqrt(1 - z * z)
        return np.stack([cx + R * rr * np.cos(ph), cy + R * rr * np.sin(ph), cz + R * z], 1)
    if g.kind == BOX:
        d = g.dim
        lo = np.array(g.params[:d], float)
        hi = np.array(g.params[d:2 * d], float)
        n = g.layout[0]
        out = []
        for f in range(2 * d):
            a, side = f // 2, f % 2
            others = [b for b in range(d) if b != a]
            idx = np.stack(np.meshgrid(*[np.arange(n)] * (d - 1), indexing="ij"), -1).reshape(-1, d - 1)
            p = np.zeros((idx.shape[0], d))
            p[:, a] = hi[a] if side else lo[a]
            for c, b in enumerate(others):
                p[:, b] = lo[b] + (idx[:, c] + 0.5) * (hi[b] - lo[b]) / n
            out.append(p)
        return np.concatenate(out, 0)
    raise ValueError(g.kind)


# --------------------------------------------------------------------------------------------
# Conductivity helpers for the *data* (not used by either estimator)
# --------------------------------------------------------------------------------------------

def spd_inv_sqrt(K: np.ndarray) -> np.ndarray:
    w, Q = np.linalg.eigh(np.asarray(K, float))
    return (Q / np.sqrt(w)) @ Q.T


def random_rotation(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random rotation (QR of a Gaussian matrix with sign fix, det = +1)."""
    A = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def harmonic_re_z3(x: np.ndarray, K: np.ndarray) -> np.ndarray:
    """u(x) = Re((y1 + i y2)^3) with y = K^{-1/2} x: harmonic for div(K grad u) = 0 in 2D."""
    y = x @ spd_inv_sqrt(K).T
    z = y[:, 0] + 1j * y[:, 1]
    return np.real(z ** 3)


def random_harmonic_poly(d: int, K: np.ndarray, degree: int, rng: np.random.Generator):
    """u(x) = Re sum_k alpha_k (c_k . y)^k, y = K^{-1/2} x, c_k = a + i b with a ⟂ b, |a| = |b|.

    c_k . c_k = 0 makes every term harmonic in y in any dimension, so u is K-harmonic in x."""
    Kis = spd_inv_sqrt(K)
    terms = []
    for k in range(degree + 1):
        a = rng.standard_normal(d)
        a /= np.linalg.norm(a)
        b = rng.standard_normal(d)
        b -= (b @ a) * a
        b /= np.linalg.norm(b)
        terms.append((rng.standard_normal(), a + 1j * b, k))

    def u(x):
        y = np.asarray(x, float) @ Kis.T
        acc = np.zeros(y.shape[0], complex)
        for alpha, c, k in terms:
            acc += alpha * (y @ c) ** k
        return np.real(acc)
    return u


def add_noise(uD, u0, eta, rng):
    """Additive i.i.d. Gaussian noise of std eta * max|u| over u^D and u^0."""
    scale = eta * max(np.abs(uD).max(initial=0.0), np.abs(u0).max(initial=0.0))
    return (uD + scale * rng.standard_normal(uD.shape),
            u0 + scale * rng.standard_normal(u0.shape), scale)


# --------------------------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------------------------

def cfg1_disk(n_walks: int = 10_000) -> Instance:
    """2D unit disk, K = I, 64 equal arcs (Gamma_0 = upper half), 64 points on radius 0.5."""
    M = 64
    g = Geometry(2, DISK, (0.0, 0.0, 1.0), (M,))
    g.gamma1_mask = (np.arange(M) >= M // 2).astype(np.uint8)
    t = 2 * np.pi * np.arange(64) / 64
    x = 0.5 * np.stack([np.cos(t), np.sin(t)], 1)
    return Instance(g, np.eye(2), x, n_walks, eps=1e-4, seed=0, precision=FP64,
                    name="disk64_K=I_64pts")


def perforated_disk_example(n_walks: int = 10_000, n_obs: int = 100, eps: float = 1e-4,
                            precision: int = FP64, m_out: int = 500, m_hole: int = 100) -> Instance:
    """The paper's Example of a disc perforated by five smaller discs (Section 5.2, Example 4):
    D_0 the unit disc, holes of radius 0.2 centred at 0.5 (cos t_l, sin t_l), t_l = 2 (l - 1) pi / 5;
    Gamma_0 the outer circle (m_out arcs), Gamma_1 the five hole circles (m_hole arcs each); K = I;
    the interior points equally spaced on the circle at distance 0.05 from Gamma_0 (radius 0.95).
    Data: 2D-sol3, u = x_1^2 - x_2^2, without noise.  (The paper uses N = 10^6 and eps = 10^-10.)"""
    t = 2 * np.pi * np.arange(5) / 5
    holes = np.stack([0.5 * np.cos(t), 0.5 * np.sin(t), np.full(5, 0.2)], 1)
    g = Geometry(2, PERFORATED, (0.0, 0.0, 1.0), (m_out, m_hole, 5), verts=holes)
    g.gamma1_mask = (np.arange(g.n_elem) >= m_out).astype(np.uint8)
    s = 2 * np.pi * np.arange(n_obs) / n_obs
    x = 0.95 * np.stack([np.cos(s), np.sin(s)], 1)
    inst = Instance(g, np.eye(2), x, n_walks, eps=eps, seed=4, precision=precision,
                    name="perforated_disc_5holes")
    u = lambda p: p[:, 0] ** 2 - p[:, 1] ** 2
    ref = element_ref_points(g)
    inst.uD = u(x)
    inst.u0 = u(ref[g.gamma1_mask == 0])
    inst.u_exact_g1 = u(ref[g.gamma1_mask == 1])
    return inst


def _with_data(inst: Instance, u) -> Instance:
    ref = element_ref_points(inst.geom)
    m = inst.geom.gamma1_mask
    inst.uD = u(inst.x_obs)
    inst.u0 = u(ref[m == 0])
    inst.u_exact_g1 = u(ref[m == 1])
    return inst


def bauer_spiral(n: int) -> np.ndarray:
    """n nearly uniform unit vectors on Bauer's spiral as Section 5.3 states it: polar angle
    phi_k = arccos(1 - (2k - 1)/n), azimuth theta_k = sqrt(n pi) phi_k, k = 1..n."""
    k = np.arange(1, n + 1)
    phi = np.arccos(1.0 - (2.0 * k - 1.0) / n)
    th = np.sqrt(n * np.pi) * phi
    return np.stack([np.sin(phi) * np.cos(th), np.sin(phi) * np.sin(th), np.cos(phi)], 1)


def annulus_example(example: int = 2, n_walks: int = 10_000, eps: float = 1e-10, precision: int = FP64,
                    m_out: int = 500, m_in: int = 100, n_obs: int = 100) -> Instance:
    """The paper's Examples 2 and 3 (Section 5.2): the concentric annulus between the unit circle and
    the circle of radius 0.5 (Example 2) or 0.2 (Example 3), K = I; Gamma_0 the outer circle (m_out
    arcs), Gamma_1 the inner one (m_in arcs); the points equally spaced from angle 0 on
    Gamma_D = {dist(x, Gamma_0) = 0.05}, the circle of radius 0.95.  The paper: M_0 = 500, M_1 = 100,
    M_D = 100, N = 10^6, eps = 10^-10.  Data: 2D-sol2 (as for Examples 1 and 5), without noise."""
    r_in = {2: 0.5, 3: 0.2}[example]
    g = Geometry(2, ANNULUS, (0.0, 0.0, r_in, 1.0), (m_out, m_in))
    g.gamma1_mask = (np.arange(g.n_elem) >= m_out).astype(np.uint8)
    s = 2 * np.pi * np.arange(n_obs) / n_obs
    x = 0.95 * np.stack([np.cos(s), np.sin(s)], 1)
    inst = Instance(g, np.eye(2), x, n_walks, eps=eps, seed=example, precision=precision,
                    name=f"annulus_example{example}")
    return _with_data(inst, lambda p: (-p[:, 0] ** 3 / 3 - p[:, 0] ** 2 * p[:, 1] + p[:, 0] * p[:, 1] ** 2
                                       + p[:, 1] ** 3 / 3))


def square_hole_example(example: int = 1, n_walks: int = 10_000, eps: Optional[float] = None,
                        precision: int = FP64, m_face: int = 100, m_hole: int = 50,
                        n_obs: int = 40) -> Instance:
    """The paper's Examples 1 and 5 (Section 5.2): D = (-1, 1)^2 minus the disc of radius 0.2 about
    (0.5, 0), K = I, M_0 + M_1 = 4 m_face + m_hole cells (the paper: 400 + 50).
    Example 1: Gamma_0 the square, Gamma_1 the hole circle; the points equally spaced by perimeter
    on Gamma_D = {dist(x, Gamma_0) = 0.05}, the square of half side 0.95, counter-clockwise from
    (0.95, -0.95 + h/2), h the spacing; eps = 1e-7 in the paper.
    Example 5: Gamma_0 empty, Gamma_1 the whole boundary; the points equally spaced on the circle
    of radius 0.3 about (-0.5, 0.5); eps = 1e-10 in the paper.
    Data: 2D-sol2, u = -x1^3/3 - x1^2 x2 + x1 x2^2 + x2^3/3 (harmonic), without noise."""
    g = Geometry(2, PERFBOX, (-1.0, -1.0, 1.0, 1.0), (m_face, m_hole), verts=np.array([[0.5, 0.0, 0.2]]))
    M0 = 4 * m_face
    if example == 1:
        g.gamma1_mask = (np.arange(g.n_elem) >= M0).astype(np.uint8)
        a, L = 0.95, 8 * 0.95
        s = (np.arange(n_obs) + 0.5) * L / n_obs
        side, t = np.floor_divide(s, 2 * a).astype(int), np.mod(s, 2 * a) - a
        x = np.empty((n_obs, 2))
        for k, (cx, cy) in enumerate([(a, None), (None, a), (-a, None), (None, -a)]):
            on = side == k
            if cx is not None:
                x[on] = np.stack([np.full(on.sum(), cx), t[on] if k == 0 else -t[on]], 1)
            else:
                x[on] = np.stack([-t[on] if k == 1 else t[on], np.full(on.sum(), cy)], 1)
    elif example == 5:
        g.gamma1_mask = np.ones(g.n_elem, np.uint8)
        t = 2 * np.pi * np.arange(n_obs) / n_obs
        x = np.stack([-0.5 + 0.3 * np.cos(t), 0.5 + 0.3 * np.sin(t)], 1)
    else:
        raise ValueError(example)
    if eps is None:
        eps = 1e-7 if example == 1 else 1e-10
    inst = Instance(g, np.eye(2), x, n_walks, eps=eps, seed=1, precision=precision,
                    name=f"square_with_hole_example{example}")
    return _with_data(inst, lambda p: (-p[:, 0] ** 3 / 3 - p[:, 0] ** 2 * p[:, 1] + p[:, 0] * p[:, 1] ** 2
                                       + p[:, 1] ** 3 / 3))


def spherical_shell_example(example: int = 6, n_walks: int = 10_000, eps: float = 1e-10,
                            precision: int = FP64, outer=(1000, 0), inner=(100, 0),
                            n_obs: int = 100) -> Instance:
    """The paper's Examples 6 and 7 (Section 5.3): the unit ball minus the ball of radius 0.5 about
    the origin (Example 6) or about (0.3, 0, 0) (Example 7), K = I; Gamma_0 the outer sphere
    (M_0 = 1000 extrinsic Voronoi cells of Bauer nodes), Gamma_1 the inner sphere (M_1 = 100); the
    points on Bauer's spiral on Gamma_D = {dist(x, Gamma_0) = 0.05}, the sphere of radius 0.95.
    Sphere layouts (n_z, n_phi) give equal-area cells instead.
    Data: 3D-sol1, u = x1 x2 + x2^2 - x3^2 (harmonic), without noise."""
    c = {6: (0.0, 0.0, 0.0), 7: (0.3, 0.0, 0.0)}[example]
    g = Geometry(3, PERFORATED, (0.0, 0.0, 0.0, 1.0), tuple(outer) + tuple(inner),
                 verts=np.array([[c[0], c[1], c[2], 0.5]]))
    g.gamma1_mask = (np.arange(g.n_elem) >= _sphere_cells(*outer)).astype(np.uint8)
    x = 0.95 * bauer_spiral(n_obs)
    inst = Instance(g, np.eye(3), x, n_walks, eps=eps, seed=2, precision=precision,
                    name=f"spherical_shell_example{example}")
    return _with_data(inst, lambda p: p[:, 0] * p[:, 1] + p[:, 1] ** 2 - p[:, 2] ** 2)


def cfg2_annulus(n_walks: int = 100_000, n_obs: int = 1024, precision: int = FP32_GEOM_FP64_EXIT,
                 eta: float = 0.01, radius_mode: int = RADIUS_WOE_BOUND) -> Instance:
    """2D annulus r in [0.3, 1], K = [[1, .5], [.5, 2]], 128 + 128 arcs, 1024 points uniform by area.

    Gamma_0 = outer arcs with angle in [0, pi); Gamma_1 = the rest.  Data u = Re(z^3) in mapped
    coordinates y = K^{-1/2} x, with 1 % Gaussian noise."""
    g = Geometry(2, ANNULUS, (0.0, 0.0, 0.3, 1.0), (128, 128))
    mask = np.ones(256, np.uint8)
    mask[:64] = 0
    g.gamma1_mask = mask
    rng = np.random.default_rng(0)
    r = np.sqrt(rng.uniform(0.3 ** 2, 1.0, n_obs))
    th = rng.uniform(0, 2 * np.pi, n_obs)
    x = np.stack([r * np.cos(th), r * np.sin(th)], 1)
    K = np.array([[1.0, 0.5], [0.5, 2.0]])
    inst = Instance(g, K, x, n_walks, eps=1e-4, seed=0, precision=precision, radius_mode=radius_mode,
                    name="annulus256_Kaniso_1024pts")
    ref = element_ref_points(g)
    u_ref = harmonic_re_z3(ref, K)
    uD = harmonic_re_z3(x, K)
    u0 = u_ref[mask == 0]
    nrng = np.random.default_rng(12)
    inst.uD, inst.u0, scale = add_noise(uD, u0, eta, nrng)
    inst.u_exact_g1 = u_ref[mask == 1]
    inst.noise_delta = scale  # ||nu * noise|| ~ scale when nu = 1/sqrt(M_D)
    return inst


def cfg3_cube(n_walks: int = 100_000, precision: int = FP32_GEOM_FP64_EXIT,
              radius_mode: int = RADIUS_MAPPED_EXACT, stride: int = 1, eta: float = 0.01) -> Instance:
    """[0,1]^3, K = Q diag(1,3,10) Q^T (Q Haar-random, seed 1), 24x24 patches per face,
    Gamma_0 = faces {x=0, y=0, z=0}; 4096 points on the 16^3 interior grid.  Data: a random
    K-harmonic polynomial of degree 3 (seed 3) with eta (1 %) Gaussian noise (seed 13)."""
    import scipy.stats as st
    n = 24
    g = Geometry(3, BOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (n,))
    M = 6 * n * n
    face = np.arange(M) // (n * n)
    g.gamma1_mask = (face % 2 == 1).astype(np.uint8)  # faces 0,2,4 are the lo faces -> Gamma_0
    Q = st.special_ortho_group.rvs(3, random_state=1)
    K = Q @ np.diag([1.0, 3.0, 10.0]) @ Q.T
    k = (np.arange(16) + 0.5) / 16
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)[::stride].copy()
    inst = Instance(g, K, x, n_walks, eps=1e-4, seed=0, precision=precision,
                    radius_mode=radius_mode, name="cube3456_Kaniso_4096pts")
    ref = element_ref_points(g)
    rng = np.random.default_rng(3)
    u = random_harmonic_poly(3, K, 3, rng)
    inst.uD, inst.u0, inst.noise_delta = add_noise(u(x), u(ref)[g.gamma1_mask == 0], eta, np.random.default_rng(13))
    inst.u_exact_g1 = u(ref)[g.gamma1_mask == 1]
    return inst


L_SHAPE = np.array([[0, 0], [1, 0], [1, 0.5], [0.5, 0.5], [0.5, 1], [0, 1]], float)


def mesh_winding(tris: np.ndarray, p: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """Winding number of a closed triangle surface about each point: the sum of the solid angles
    of its triangles seen from the point over 4 pi (Van Oosterom and Strackee's formula for the
    solid angle of a triangle); about 1 inside an outward-oriented surface, 0 outside."""
    T = np.asarray(tris, float).reshape(-1, 3, 3)
    p = np.asarray(p, float).reshape(-1, 3)
    out = np.zeros(p.shape[0])
    for s in range(0, T.shape[0], chunk):
        A = T[None, s:s + chunk, 0] - p[:, None]
        B = T[None, s:s + chunk, 1] - p[:, None]
        Cc = T[None, s:s + chunk, 2] - p[:, None]
        la, lb, lc = (np.linalg.norm(v, axis=2) for v in (A, B, Cc))
        det = np.einsum("ptk,ptk->pt", A, np.cross(B, Cc))
        den = la * lb * lc + (A * B).sum(2) * lc + (A * Cc).sum(2) * lb + (B * Cc).sum(2) * la
        out += (2.0 * np.arctan2(det, den)).sum(1)
    return out / (4.0 * np.pi)


def box_mesh(lo, hi, n: int) -> np.ndarray:
    """The surface of the box [lo, hi] (3D) as triangles, outward-oriented, in the cell order of
    the BOX kind: faces (x=lo, x=hi, y=lo, y=hi, z=lo, z=hi), n x n patches each (index along the
    other two axes in increasing axis order), two triangles per patch.  With two triangles per
    element (layout (2,)) the elements are the BOX kind's patches."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    out = []
    for f in range(6):
        a, side = f // 2, f % 2
        b0, b1 = [b for b in range(3) if b != a]
        # e_b0 x e_b1 is +e_a for a = 0, 2 and -e_a for a = 1; outward is +e_a on the hi side
        ccw = (1 if a != 1 else -1) * (1 if side else -1) > 0
        g0 = np.linspace(lo[b0], hi[b0], n + 1)
        g1 = np.linspace(lo[b1], hi[b1], n + 1)
        for i0 in range(n):
            for i1 in range(n):
                q = np.zeros((4, 3))
                q[:, a] = hi[a] if side else lo[a]
                q[:, b0] = [g0[i0], g0[i0 + 1], g0[i0 + 1], g0[i0]]
                q[:, b1] = [g1[i1], g1[i1], g1[i1 + 1], g1[i1 + 1]]
                if ccw:
                    out += [q[[0, 1, 2]], q[[0, 2, 3]]]
                else:
                    out += [q[[0, 2, 1]], q[[0, 3, 2]]]
    return np.array(out)


def sphere_mesh(c, R: float, level: int) -> np.ndarray:
    """An icosahedron subdivided `level` times (each triangle into four) with its vertices on the
    sphere |x - c| = R: 20 * 4^level outward-oriented triangles."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    tris = [np.array([V[i] for i in f], float) for f in F]
    tris = [x / np.linalg.norm(x, axis=1, keepdims=True) for x in tris]
    for _ in range(level):
        nxt = []
        for a, b, cc in tris:
            ab, bc, ca = [(u + v) / np.linalg.norm(u + v) for u, v in ((a, b), (b, cc), (cc, a))]
            nxt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, cc]), np.array([ab, bc, ca])]
        tris = nxt
    T = np.array(tris)
    flip = np.einsum("tk,tk->t", np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), T.mean(1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return np.asarray(c, float) + R * T


def l_prism_mesh(n: int, height: float = 1.0) -> np.ndarray:
    """The L-shaped prism L x [0, height] (L = the L-shape polygon, a non-convex domain): its six
    walls split into patches of side about 1/n, the bottom and top L faces into squares of side
    1/n (n even), two triangles per patch, outward-oriented."""
    L = L_SHAPE
    out = []
    zs = np.linspace(0.0, height, max(1, round(n * height)) + 1)
    for k in range(len(L)):
        p, q = L[k], L[(k + 1) % len(L)]
        m = max(1, round(n * np.linalg.norm(q - p)))
        s = np.linspace(0.0, 1.0, m + 1)
        for i in range(m):
            a, b = p + s[i] * (q - p), p + s[i + 1] * (q - p)
            for j in range(len(zs) - 1):
                P = np.array([[*a, zs[j]], [*b, zs[j]], [*b, zs[j + 1]], [*a, zs[j + 1]]])
                out += [P[[0, 1, 2]], P[[0, 2, 3]]]  # (b - a) x z points out of a CCW loop
    h = 1.0 / n
    for (x0, y0) in ((0.0, 0.0), (0.5, 0.0), (0.0, 0.5)):
        for i in range(n // 2):
            for j in range(n // 2):
                xa, ya = x0 + i * h, y0 + j * h
                sq = np.array([[xa, ya], [xa + h, ya], [xa + h, ya + h], [xa, ya + h]])
                bot = np.column_stack([sq, np.zeros(4)])
                top = np.column_stack([sq, np.full(4, height)])
                out += [bot[[0, 2, 1]], bot[[0, 3, 2]], top[[0, 1, 2]], top[[0, 2, 3]]]
    return np.array(out)


def _inside(g: Geometry, p: np.ndarray) -> np.ndarray:
    """Membership of candidate points in the open domain (used to draw points by rejection)."""
    if g.kind == DISK:
        cx, cy, R = g.params
        return (p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2 < R * R
    if g.kind == ANNULUS:
        cx, cy, ri, ro = g.params
        r2 = (p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2
        return (r2 < ro * ro) & (r2 > ri * ri)
    if g.kind == ELLIPSE:
        cx, cy, a, b = g.params
        return ((p[:, 0] - cx) / a) ** 2 + ((p[:, 1] - cy) / b) ** 2 < 1
    if g.kind == POLYGON:
        v = np.asarray(g.verts)
        ins = np.zeros(p.shape[0], bool)
        for k in range(len(v)):
            a, b = v[k], v[(k + 1) % len(v)]
            cond = (a[1] > p[:, 1]) != (b[1] > p[:, 1])
            xint = a[0] + (p[:, 1] - a[1]) * (b[0] - a[0]) / np.where(b[1] != a[1], b[1] - a[1], 1)
            ins ^= cond & (p[:, 0] < xint)
        return ins
    if g.kind == BALL:
        c = np.array(g.params[:3])
        return ((p - c) ** 2).sum(1) < g.params[3] ** 2
    if g.kind == BOX:
        d = g.dim
        lo, hi = np.array(g.params[:d]), np.array(g.params[d:2 * d])
        return np.all((p > lo) & (p < hi), 1)
    if g.kind == TRIMESH:
        return mesh_winding(g.verts, p) > 0.5
    if g.kind in (PERFORATED, PERFBOX):
        d = g.dim
        if g.kind == PERFORATED:
            ok = ((p - np.array(g.params[:d])) ** 2).sum(1) < g.params[d] ** 2
        else:
            ok = np.all((p > np.array(g.params[:d])) & (p < np.array(g.params[d:2 * d])), 1)
        for h in np.asarray(g.verts, float).reshape(-1, d + 1):
            ok &= ((p - h[:d]) ** 2).sum(1) > h[d] ** 2
        return ok
    raise ValueError(g.kind)


def _bbox(g: Geometry):
    if g.kind == TRIMESH:
        T = np.asarray(g.verts, float).reshape(-1, 3)
        return T.min(0), T.max(0)
    if g.kind == PERFORATED:
        c, R = np.array(g.params[:g.dim]), g.params[g.dim]
        return c - R, c + R
    if g.kind == PERFBOX:
        return np.array(g.params[:g.dim]), np.array(g.params[g.dim:2 * g.dim])
    if g.kind == DISK:
        cx, cy, R = g.params[:3]
        return np.array([cx - R, cy - R]), np.array([cx + R, cy + R])
    if g.kind == ANNULUS:
        cx, cy, _, R = g.params
        return np.array([cx - R, cy - R]), np.array([cx + R, cy + R])
    if g.kind == ELLIPSE:
        cx, cy, a, b = g.params
        return np.array([cx - a, cy - b]), np.array([cx + a, cy + b])
    if g.kind == POLYGON:
        v = np.asarray(g.verts)
        return v.min(0), v.max(0)
    if g.kind == BALL:
        c = np.array(g.params[:3])
        return c - g.params[3], c + g.params[3]
    d = g.dim
    return np.array(g.params[:d]), np.array(g.params[d:2 * d])


def sample_points(g: Geometry, n: int, rng: np.random.Generator, margin: float = 0.0) -> np.ndarray:
    lo, hi = _bbox(g)
    out = []
    while sum(len(o) for o in out) < n:
        p = rng.uniform(lo, hi, (max(2 * n, 64), g.dim))
        ok = _inside(g, p)
        if margin > 0:
            for dlt in np.eye(g.dim) * margin:
                ok &= _inside(g, p + dlt) & _inside(g, p - dlt)
        out.append(p[ok])
    return np.concatenate(out, 0)[:n].copy()


def _layout_for(kind: int, dim: int, M_target: int):
    if kind in (DISK, ELLIPSE, POLYGON):
        return (M_target,)
    if kind == ANNULUS:
        return (M_target - M_target // 2, M_target // 2)
    if kind == BALL:
        nphi = max(4, int(round(math.sqrt(2 * M_target))))
        nz = max(2, M_target // nphi)
        return (nz, nphi)
    if kind == BOX:
        if dim == 2:
            return (max(1, M_target // 4),)
        return (max(1, int(round(math.sqrt(M_target / 6)))),)
    raise ValueError(kind)


def _radius_for(kind: int, mapped_radii: bool) -> int:
    if kind == BOX or (mapped_radii and kind == POLYGON):
        return RADIUS_MAPPED_EXACT
    if mapped_radii and kind in (DISK, ANNULUS, BALL, ELLIPSE):
        return RADIUS_MAPPED_BOUND
    return RADIUS_WOE_BOUND


def random_instance(rng: np.random.Generator, instance_id: int, kind_name: Optional[str] = None,
                    walk_scale: float = 1.0, precision: int = FP32_GEOM_FP64_EXIT,
                    data_degree: int = 6, eta: Optional[float] = None, mapped_radii: bool = True) -> Instance:
    """One instance of the heterogeneous batch: disk, ellipse (1 x 0.4), L-shape, annulus (0.3, 1),
    unit ball or unit cube; random SPD K with condition number in [1, 20] (lambda_max = 1);
    points per instance in [32, 2048]; elements in [64, 2048]; walks log-uniform in [1e3, 1e5];
    Gamma_0 = elements whose reference point's last coordinate is >= the domain centre's.
    Step radius: the kind's mapped radius (exact for the cube and the L-shape, the bound for the
    disk, annulus, ball and ellipse), or with mapped_radii=False the cube's only."""
    kinds = ["disk", "ellipse", "lshape", "annulus", "ball", "cube"]
    kn = kind_name or kinds[int(rng.integers(len(kinds)))]
    if kn == "disk":
        g = Geometry(2, DISK, (0.0, 0.0, 1.0))
    elif kn == "ellipse":
        g = Geometry(2, ELLIPSE, (0.0, 0.0, 1.0, 0.4))
    elif kn == "lshape":
        g = Geometry(2, POLYGON, (), verts=L_SHAPE.copy())
    elif kn == "annulus":
        g = Geometry(2, ANNULUS, (0.0, 0.0, 0.3, 1.0))
    elif kn == "ball":
        g = Geometry(3, BALL, (0.0, 0.0, 0.0, 1.0))
    else:
        g = Geometry(3, BOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0))
    d = g.dim
    M_target = int(rng.integers(64, 2049))
    g.layout = _layout_for(g.kind, d, M_target)
    ref = element_ref_points(g)
    lo, hi = _bbox(g)
    centre = 0.5 * (lo + hi)
    if g.kind == POLYGON:
        centre = np.asarray(g.verts).mean(0)
    g.gamma1_mask = (ref[:, -1] < centre[-1]).astype(np.uint8)
    cond = rng.uniform(1.0, 20.0)
    if d == 2:
        lam = np.array([1.0, 1.0 / cond])
    else:
        mid = math.exp(rng.uniform(math.log(1.0 / cond), 0.0))
        lam = np.array([1.0, mid, 1.0 / cond])
    Q = random_rotation(d, rng)
    K = Q @ np.diag(lam) @ Q.T
    K = 0.5 * (K + K.T)
    n_obs = int(rng.integers(32, 2049))
    x = sample_points(g, n_obs, rng, margin=1e-3)
    N = int(round(10 ** rng.uniform(3, 5) * walk_scale))
    N = max(N, 1)
    inst = Instance(g, K, x, N, eps=1e-4, seed=instance_id + 1000, instance_id=instance_id,
                    precision=precision,
                    radius_mode=_radius_for(g.kind, mapped_radii),
                    name=f"{kn}{g.n_elem}")
    u = random_harmonic_poly(d, K, data_degree, rng)
    uref = u(ref)
    eta_v = rng.uniform(0.01, 0.05) if eta is None else eta
    uD, u0, scale = add_noise(u(x), uref[g.gamma1_mask == 0], eta_v, rng)
    inst.uD, inst.u0 = uD, u0
    inst.u_exact_g1 = uref[g.gamma1_mask == 1]
    inst.noise_delta = scale
    return inst


def cfg4_batch(n_instances: int = 64, seed: int = 4, walk_scale: float = 1.0,
               precision: int = FP32_GEOM_FP64_EXIT, mapped_radii: bool = True) -> list:
    rng = np.random.default_rng(seed)
    return [random_instance(rng, i, walk_scale=walk_scale, precision=precision, mapped_radii=mapped_radii)
            for i in range(n_instances)]


def cfg5_arrivals(rate: float = 200.0, duration_s: float = 60.0, seed: int = 5):
    """Poisson arrival times (seconds) of the serving stream."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            return np.array(out)
        out.append(t)
