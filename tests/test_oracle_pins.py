"""Pins of the CPU oracle against facts fixed outside it: published known answers, closed forms
from the paper's introduction, textbook special cases, brute force and exact invariants.

Every check here would fail for a plausible slip in the oracle (wrong Philox round, wrong uniform
conversion, a non-uniform direction, a wrong square root of K, a wrong distance or element index,
a dropped count, an unnormalised K)."""
import os

import numpy as np
import pytest
from scipy import integrate, stats
from scipy.spatial import cKDTree

import wos_inputs as wi
from oracle import closed_forms as cf
from oracle import walks
from tests import statutil

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Philox and uniforms

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert walks.philox(v[0:4], v[4:6]) == tuple(v[6:10])


def test_u53_range_and_resolution():
    assert walks.u53(0, 0) == 2.0 ** -54
    assert walks.u53(0, 1 << 11) == 2.0 ** -53 + 2.0 ** -54
    # the low 11 bits are dropped
    assert walks.u53(0x12345678, 0x9ABCDEF0) == walks.u53(0x12345678, 0x9ABCD800)
    top = walks.u53(0xFFFFFFFF, 0xFFFFFFFF)
    assert 1 - 2.0 ** -52 < top <= 1.0


def test_philox_uniformity_chi2():
    # 40 000 blocks, 160 000 words, top byte histogram
    words = np.array([walks.philox((b, 7, 3, 1), (11, 22)) for b in range(40000)], np.uint64).ravel()
    hist = np.bincount((words >> np.uint64(24)).astype(np.int64), minlength=256)
    chi = ((hist - hist.mean()) ** 2 / hist.mean()).sum()
    assert stats.chi2.sf(chi, 255) > 1e-4


# ---------------------------------------------------------------- sphere sampler

@pytest.mark.parametrize("dim", [2, 3])
def test_direction_moments(dim):
    n = 200_000
    U = np.concatenate([walks.directions(dim, n // 4, k=k, i=5, inst=2, seed=9) for k in range(4)])
    assert np.allclose(np.linalg.norm(U, axis=1), 1.0, atol=1e-15)
    m = U.mean(0)
    assert np.all(np.abs(m) < 5 * np.sqrt(1.0 / dim / n))
    C = U.T @ U / n
    # Var(U_a^2) <= 1, Var(U_a U_b) <= 1/4 ... use a generous 5-sigma bound
    assert np.all(np.abs(C - np.eye(dim) / dim) < 5 * np.sqrt(0.5 / n))
    if dim == 3:
        assert stats.kstest((U[:, 2] + 1) / 2, "uniform").pvalue > 1e-4
        ph = np.mod(np.arctan2(U[:, 1], U[:, 0]), 2 * np.pi) / (2 * np.pi)
        assert stats.kstest(ph, "uniform").pvalue > 1e-4
    else:
        th = np.mod(np.arctan2(U[:, 1], U[:, 0]), 2 * np.pi) / (2 * np.pi)
        assert stats.kstest(th, "uniform").pvalue > 1e-4


# ---------------------------------------------------------------- geometry vs brute force

def _boundary_samples(g, n):
    """Dense boundary samples with their element index, built from the element definitions."""
    M = g.n_elem
    if g.kind == wi.DISK:
        t = (np.arange(n) + 0.5) * 2 * np.pi / n
        return np.stack([np.cos(t), np.sin(t)], 1) * g.params[2], (t * M / (2 * np.pi)).astype(int)
    if g.kind == wi.ANNULUS:
        mo, mi = g.layout
        t = (np.arange(n) + 0.5) * 2 * np.pi / n
        po = np.stack([np.cos(t), np.sin(t)], 1) * g.params[3]
        pi_ = np.stack([np.cos(t), np.sin(t)], 1) * g.params[2]
        return (np.concatenate([po, pi_]),
                np.concatenate([(t * mo / (2 * np.pi)).astype(int), mo + (t * mi / (2 * np.pi)).astype(int)]))
    if g.kind in (wi.PERFORATED, wi.PERFBOX) and (g.dim == 3 or g.kind == wi.PERFBOX):
        # outer boundary, then each hole (circles: arcs from angle 0; spheres: (z band, azimuth) cells)
        d = g.dim
        holes = np.asarray(g.verts, float).reshape(-1, d + 1)
        if g.kind == wi.PERFORATED:
            pts, el = _sphere_samples(g.params[:3], g.params[3], g.layout[0], g.layout[1], n)
            hc = (g.layout[2], g.layout[3])
        else:
            pts, el = _boundary_samples(wi.Geometry(d, wi.BOX, g.params, (g.layout[0],)), n)
            hc = tuple(g.layout[1:d])
        off, P, E = len(set(el.tolist())), [pts], [el]
        for h in holes:
            if d == 2:
                t = (np.arange(n) + 0.5) * 2 * np.pi / n
                P.append(np.stack([h[0] + h[2] * np.cos(t), h[1] + h[2] * np.sin(t)], 1))
                E.append(off + (t * hc[0] / (2 * np.pi)).astype(int))
            else:
                q, c = _sphere_samples(h[:3], h[3], hc[0], hc[1], n)
                P.append(q)
                E.append(off + c)
            off += int(np.prod(hc))
        return np.concatenate(P), np.concatenate(E)
    if g.kind == wi.PERFORATED:
        mo, mh, k = g.layout[:3]
        t = (np.arange(n) + 0.5) * 2 * np.pi / n
        circles = [(g.params[0], g.params[1], g.params[2], mo, 0)]
        circles += [(hx, hy, r, mh, mo + l * mh) for l, (hx, hy, r) in enumerate(np.asarray(g.verts).reshape(k, 3))]
        pts = [np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], 1) for cx, cy, r, _, _ in circles]
        el = [off + (t * m / (2 * np.pi)).astype(int) for _, _, _, m, off in circles]
        return np.concatenate(pts), np.concatenate(el)
    if g.kind == wi.POLYGON:
        v = np.asarray(g.verts)
        seg = np.roll(v, -1, 0) - v
        ln = np.sqrt((seg ** 2).sum(1))
        cum = np.concatenate([[0], np.cumsum(ln)])
        s = (np.arange(n) + 0.5) * cum[-1] / n
        e = np.searchsorted(cum, s, side="right") - 1
        p = v[e] + ((s - cum[e]) / ln[e])[:, None] * seg[e]
        return p, (s * M / cum[-1]).astype(int)
    if g.kind == wi.BOX:
        d, nn = g.dim, g.layout[0]
        lo, hi = np.array(g.params[:d], float), np.array(g.params[d:2 * d], float)
        m = int(round(n ** (1.0 / (d - 1))))
        pts, el = [], []
        for f in range(2 * d):
            a, side = f // 2, f % 2
            others = [b for b in range(d) if b != a]
            grid = np.stack(np.meshgrid(*[(np.arange(m) + 0.5) / m] * (d - 1), indexing="ij"), -1).reshape(-1, d - 1)
            p = np.zeros((grid.shape[0], d))
            p[:, a] = hi[a] if side else lo[a]
            idx = np.zeros(grid.shape[0], int)
            for c, b in enumerate(others):
                p[:, b] = lo[b] + grid[:, c] * (hi[b] - lo[b])
                idx = idx * nn + (grid[:, c] * nn).astype(int)
            pts.append(p)
            el.append(f * nn ** (d - 1) + idx)
        return np.concatenate(pts), np.concatenate(el)
    if g.kind == wi.BALL:
        return _sphere_samples(g.params[:3], g.params[3], g.layout[0], g.layout[1], n)
    raise ValueError(g.kind)


def _sphere_samples(c, R, nz, nphi, n):
    """About n points of a (z, azimuth) grid on the sphere |x - c| = R and their equal-area cells."""
    m = int(np.sqrt(n))
    z = 1 - 2 * (np.arange(m) + 0.5) / m
    ph = (np.arange(2 * m) + 0.5) * np.pi / m
    Z, P = np.meshgrid(z, ph, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    p = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3) * R + np.asarray(c, float)
    iz = ((1 - Z) / 2 * nz).astype(int).ravel()
    ip = (P * nphi / (2 * np.pi)).astype(int).ravel()
    return p, iz * nphi + ip


@pytest.mark.parametrize("case", ["disk", "annulus", "lshape", "square", "cube", "ball", "perforated",
                                  "perforated_ball", "square_with_holes", "cube_with_hole"])
def test_distance_and_element_vs_brute_force(case):
    rng = np.random.default_rng(1)
    if case == "perforated_ball":
        holes = np.array([[0.35, 0.1, -0.05, 0.3], [-0.4, -0.2, 0.25, 0.25]])
        g = wi.Geometry(3, wi.PERFORATED, (0.02, 0.0, -0.03, 1.05), (6, 11, 4, 7), verts=holes)
    elif case == "square_with_holes":
        holes = np.array([[0.5, 0.0, 0.2], [-0.4, 0.45, 0.3]])
        g = wi.Geometry(2, wi.PERFBOX, (-1.0, -1.0, 1.0, 1.2), (13, 11), verts=holes)
    elif case == "cube_with_hole":
        g = wi.Geometry(3, wi.PERFBOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (5, 4, 6),
                        verts=np.array([[0.55, 0.45, 0.5, 0.3]]))
    elif case == "perforated":
        holes = np.array([[0.4, 0.1, 0.25], [-0.3, -0.35, 0.15], [-0.35, 0.45, 0.2]])
        g = wi.Geometry(2, wi.PERFORATED, (0.05, 0.0, 1.1), (41, 17, 3), verts=holes)
    elif case == "disk":
        g = wi.Geometry(2, wi.DISK, (0.0, 0.0, 1.0), (37,))
    elif case == "annulus":
        g = wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.3, 1.0), (29, 13))
    elif case == "lshape":
        g = wi.Geometry(2, wi.POLYGON, (), (50,), verts=wi.L_SHAPE)
    elif case == "square":
        g = wi.Geometry(2, wi.BOX, (0.0, 0.0, 1.0, 1.0), (7,))
    elif case == "cube":
        g = wi.Geometry(3, wi.BOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (5,))
    else:
        g = wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (6, 11))
    bp, be = _boundary_samples(g, 400_000 if g.dim == 2 else 360_000)
    if case in ("perforated", "square_with_holes"):  # the same angular density on every circle
        bp, be = _boundary_samples(g, 1_600_000)
    pts = wi.sample_points(g, 100 if case in ("perforated", "square_with_holes") else 300, rng)
    d, e = walks.geom_eval(g, pts)
    spacing = 2e-5 if g.dim == 2 else 6e-3
    tree = cKDTree(bp)  # exact nearest-neighbour search over the boundary samples
    dmin, jmin = tree.query(pts)
    for k in range(len(pts)):
        j = int(jmin[k])
        assert abs(d[k] - dmin[k]) <= spacing, (k, d[k], dmin[k])
        # the element of the nearest boundary sample, unless the point is close to a cell edge
        # or equidistant between two parts of the boundary
        near = be[tree.query_ball_point(pts[k], dmin[k] + 2 * spacing)]
        assert e[k] in set(near.tolist()) or len(set(near.tolist())) > 1, (k, e[k], be[j])
        assert e[k] == be[j] or len(set(near.tolist())) > 1


def test_ellipse_lower_bound_and_angle():
    g = wi.Geometry(2, wi.ELLIPSE, (0.0, 0.0, 1.0, 0.4), (40,))
    rng = np.random.default_rng(2)
    pts = wi.sample_points(g, 300, rng)
    d, e = walks.geom_eval(g, pts)
    t = (np.arange(400_000) + 0.5) * 2 * np.pi / 400_000
    bp = np.stack([np.cos(t), 0.4 * np.sin(t)], 1)
    for k in range(len(pts)):
        exact = np.sqrt(((bp - pts[k]) ** 2).sum(1)).min()
        assert d[k] <= exact + 1e-5
        f = np.hypot(pts[k, 0], pts[k, 1] / 0.4)
        assert exact <= (1 - f) / f * np.hypot(*pts[k]) / 1.0 + 1e-5  # radial point bound
        ecc = np.mod(np.arctan2(pts[k, 1] / 0.4, pts[k, 0]), 2 * np.pi)
        assert e[k] == min(int(ecc * 40 / (2 * np.pi)), 39)


# ---------------------------------------------------------------- closed forms vs quadrature

def test_disk_arc_closed_form_vs_quadrature_of_poisson_kernel():
    rng = np.random.default_rng(3)
    for _ in range(12):
        rho, phi = rng.uniform(0, 0.95), rng.uniform(0, 2 * np.pi)
        x = rho * np.array([np.cos(phi), np.sin(phi)])
        a = rng.uniform(0, 2 * np.pi)
        b = a + rng.uniform(0, 2 * np.pi)
        f = lambda t: cf.disk_density(x, np.array([np.cos(t), np.sin(t)]))
        ref = integrate.quad(f, a, b, limit=400, epsabs=1e-14, epsrel=1e-13)[0]
        assert abs(cf.disk_arc_measure(x, 1.0, a, b) - ref) < 1e-11
    # total mass 1 for any pole
    H = cf.disk_H(np.array([[0.3, -0.2], [0.0, 0.9]]), 1.0, 16)
    assert np.allclose(H.sum(1), 1.0, atol=1e-14)


def test_ball_band_closed_form_vs_quadrature():
    for a in (0.0, 0.37, 0.8):
        x = np.array([0, 0, a])
        for c in (-1.0, -0.3, 0.2, 0.8):
            f = lambda z, ph: cf.ball_density(x, np.array([np.sqrt(1 - z * z) * np.cos(ph),
                                                           np.sqrt(1 - z * z) * np.sin(ph), z]))
            ref = integrate.dblquad(f, 0, 2 * np.pi, c, 1.0, epsabs=1e-12, epsrel=1e-12)[0]
            assert abs(cf.ball_band_above(a, c) - ref) < 1e-9


def test_annulus_series_mass_and_log_term():
    for rho in (0.35, 0.6, 0.95):
        m = cf.annulus_arc_measures(np.array([rho * np.cos(1.0), rho * np.sin(1.0)]), 0.3, 1.0, 40, 24)
        assert abs(m.sum() - 1) < 1e-12
        assert abs(m[40:].sum() - cf.annulus_inner_mass(rho, 0.3, 1.0)) < 1e-12
        assert m.min() > 0
    # as the hole shrinks the Fourier modes of the outer density tend to those of the disk
    # Poisson kernel (the constant mode, the log capacity term, converges only logarithmically)
    x = np.array([0.2, 0.5])
    m = cf.annulus_arc_measures(x, 1e-12, 1.0, 32, 4)[:32]
    h = cf.disk_H(x[None], 1.0, 32)[0]
    assert np.allclose(m - m.mean(), h - h.mean(), atol=1e-12)


# ---------------------------------------------------------------- the estimator vs closed forms

def _bias_2d(P, eps):
    """O(eps) shell bias allowance per entry: the one-sided mass within eps*log(1/eps) of each arc
    end (mass moved between neighbouring elements by stopping inside the eps-shell)."""
    return 4 * eps * (1 + np.log(1 / eps)) * np.maximum(P, 1e-3) * P.shape[1] / (2 * np.pi)


def test_oracle_disk_matches_poisson_kernel():
    inst = wi.cfg1_disk()
    counts, st, _ = walks.build_instance(inst, threads=8)
    assert np.all(counts.sum(1) == inst.n_walks)
    assert st["cap_hits"] == 0 and st["escapes"] == 0
    P = cf.disk_H(inst.x_obs, 1.0, 64)
    rep = statutil.vs_probabilities(counts, inst.n_walks, P, bias=_bias_2d(P, inst.eps))
    assert rep["ok"], rep
    chi = statutil.row_chi2(counts, inst.n_walks, P)
    assert chi["ok"], chi
    # mean number of steps for a start at radius 1/2 (O(log 1/eps), Section 4.2.1)
    assert 10 < st["steps"] / st["walks"] < 16


def test_oracle_annulus_matches_series():
    g = wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.3, 1.0), (24, 12))
    x = np.array([[0.45, 0.1], [-0.2, 0.7], [0.0, -0.93], [0.31, 0.0]])
    N = 40_000
    counts, st, _ = walks.build_measure(g, np.eye(2), x, 1e-4, seed=3, walk_end=N, threads=8)
    P = np.stack([cf.annulus_arc_measures(p, 0.3, 1.0, 24, 12) for p in x])
    rep = statutil.vs_probabilities(counts, N, P, bias=_bias_2d(P, 1e-4))
    assert rep["ok"], rep
    inner = counts[:, 24:].sum(1) / N
    mass = cf.annulus_inner_mass(np.hypot(x[:, 0], x[:, 1]), 0.3, 1.0)
    assert np.all(np.abs(inner - mass) < 4.5 * np.sqrt(mass * (1 - mass) / N) + 1e-3)


def test_oracle_ball_matches_poisson_kernel():
    g = wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (8, 6))
    a_list = [0.0, 0.35, -0.6]
    x = np.array([[0.0, 0.0, a] for a in a_list])
    N = 40_000
    counts, st, _ = walks.build_measure(g, np.eye(3), x, 1e-4, seed=5, walk_end=N, threads=8)
    P = []
    for a in a_list:
        cells = cf.ball_cells_axis(abs(a), 8, 6).reshape(8, 6)
        if a < 0:  # pole below the equator: bands mirror
            cells = cells[::-1]
        P.append(cells.ravel())
    P = np.array(P)
    rep = statutil.vs_probabilities(counts, N, P, bias=4e-4)
    assert rep["ok"], rep


def _sol4(K):
    """2D-sol4 of the paper (Section 5.2): K-harmonic for the paper's K = [[1, .3], [.3, .4]]."""
    def u(p):
        x1, x2 = p[:, 0], p[:, 1]
        return ((2 * K[1, 0] - K[1, 1]) / (3 * K[0, 0]) * x1 ** 3 - x1 ** 2 * x2 + x1 * x2 ** 2
                - (2 * K[0, 1] - K[0, 0]) / (3 * K[1, 1]) * x2 ** 3)
    return u


def _exit_mean_z(geom, S, x, u, n, grad_bound, eps=1e-4, radius_mode=0, seed=11):
    """z-scores of mean u(X_stop) - u(x): E[u(Y_tau)] = u(x) for K-harmonic u (eq.
    probabilisticrepresentation); stopping in the eps-shell moves the mean by at most eps*|grad u|."""
    z = []
    for i, p in enumerate(x):
        pos = walks.walk_exits(geom, S, p, eps, n, i=i, seed=seed, radius_mode=radius_mode)
        v = u(pos)
        dev = abs(v.mean() - u(p[None])[0])
        z.append(max(dev - eps * grad_bound, 0.0) / (v.std() / np.sqrt(n)))
    return np.array(z)


def test_walk_reproduces_paper_anisotropic_solution():
    """The WoE chain with S = Khat^{1/2} reproduces the paper's K-harmonic 2D-sol4; the plausible
    slip S = Khat (forgetting the square root) does not."""
    K = np.array([[1.0, 0.3], [0.3, 0.4]])
    u = _sol4(K)
    g = wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.5, 1.0), (8, 8))
    x = wi.sample_points(g, 10, np.random.default_rng(7))
    _, Khat, S = walks.instance_setup(K, 2)
    z = _exit_mean_z(g, S, x, u, 40_000, grad_bound=3.0)
    assert np.all(z < 4.5), z
    Sw = np.zeros((3, 3))
    Sw[:2, :2] = Khat
    zw = _exit_mean_z(g, Sw, x, u, 40_000, grad_bound=3.0)
    assert zw.max() > 8, zw


def test_walk_reproduces_isotropic_paper_solutions():
    """2D-sol2 and 2D-sol3 (K = I) of the paper on the ex01-like square with a hole replaced by the
    L-shape polygon; and 3D-sol1 in the unit ball."""
    sol2 = lambda p: -p[:, 0] ** 3 / 3 - p[:, 0] ** 2 * p[:, 1] + p[:, 0] * p[:, 1] ** 2 + p[:, 1] ** 3 / 3
    sol3 = lambda p: p[:, 0] ** 2 - p[:, 1] ** 2
    g = wi.Geometry(2, wi.POLYGON, (), (16,), verts=wi.L_SHAPE)
    x = wi.sample_points(g, 6, np.random.default_rng(9))
    _, _, S = walks.instance_setup(np.eye(2), 2)
    for u in (sol2, sol3):
        assert np.all(_exit_mean_z(g, S, x, u, 30_000, grad_bound=4.0) < 4.5)
    sol1_3d = lambda p: p[:, 0] * p[:, 1] + p[:, 1] ** 2 - p[:, 2] ** 2
    gb = wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (4, 4))
    xb = wi.sample_points(gb, 6, np.random.default_rng(10))
    _, _, S3 = walks.instance_setup(np.eye(3), 3)
    assert np.all(_exit_mean_z(gb, S3, xb, sol1_3d, 30_000, grad_bound=4.0) < 4.5)


@pytest.mark.parametrize("radius_mode", [0, 1])
def test_walk_reproduces_harmonic_in_anisotropic_cube(radius_mode):
    import scipy.stats as st_
    Q = st_.special_ortho_group.rvs(3, random_state=1)
    K = Q @ np.diag([1.0, 3.0, 10.0]) @ Q.T
    g = wi.Geometry(3, wi.BOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (4,))
    Kis = wi.spd_inv_sqrt(K)
    def u(p):  # 3D-sol1 of the paper composed with y = K^{-1/2} x: K-harmonic
        y = p @ Kis.T
        return y[:, 0] * y[:, 1] + y[:, 1] ** 2 - y[:, 2] ** 2
    x = wi.sample_points(g, 6, np.random.default_rng(8), margin=0.05)
    _, _, S = walks.instance_setup(K, 3)
    z = _exit_mean_z(g, S, x, u, 30_000, grad_bound=6.0, radius_mode=radius_mode)
    assert np.all(z < 4.5), z


def test_element_level_reproduction_fine_arcs():
    """sum_j H_ij u(c_j) ~ u(x_i): the binned measure integrates the K-harmonic 2D-sol4 (midpoint
    rule on 3000 arcs: second-order error, below 2e-4 here)."""
    K = np.array([[1.0, 0.3], [0.3, 0.4]])
    u = _sol4(K)
    g = wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.5, 1.0), (2000, 1000))
    x = wi.sample_points(g, 8, np.random.default_rng(7))
    N = 60_000
    counts, st, _ = walks.build_measure(g, K, x, 1e-4, seed=11, walk_end=N, threads=8)
    H = counts / N
    ur = u(wi.element_ref_points(g))
    est = H @ ur
    se = np.sqrt(np.maximum(H @ ur ** 2 - est ** 2, 0) / N)
    assert np.all(np.abs(est - u(x)) <= 4.5 * se + 2e-4 + 3e-4), (est - u(x), se)


def test_mapped_exact_radius_same_law_fewer_steps():
    inst0 = wi.cfg3_cube(n_walks=4000, precision=wi.FP64, radius_mode=wi.RADIUS_WOE_BOUND, stride=512)
    inst1 = wi.cfg3_cube(n_walks=4000, precision=wi.FP64, radius_mode=wi.RADIUS_MAPPED_EXACT, stride=512)
    inst1.seed = 99
    c0, s0, _ = walks.build_instance(inst0, threads=8)
    c1, s1, _ = walks.build_instance(inst1, threads=8)
    assert s1["steps"] < 0.6 * s0["steps"]
    # merge 4x4 patch blocks to keep expected counts testable
    def merge(c):
        return c.reshape(c.shape[0], 6, 6, 4, 6, 4).sum((3, 5)).reshape(c.shape[0], -1)
    rep = statutil.two_sample(merge(c0), 4000, merge(c1), 4000)
    assert rep["ok"], rep


def _random_spd(dim, cond, rng):
    import scipy.stats as st_
    Q = st_.special_ortho_group.rvs(dim, random_state=int(rng.integers(1 << 30)))
    return Q @ np.diag(np.geomspace(1.0, cond, dim)) @ Q.T


def _sphere_dirs(dim, n):
    if dim == 2:
        t = 2 * np.pi * (np.arange(n) + 0.5) / n
        return np.stack([np.cos(t), np.sin(t)], 1)
    z = 1 - (2 * np.arange(n) + 1) / n
    phi = np.pi * (3 - np.sqrt(5)) * np.arange(n)
    rr = np.sqrt(1 - z * z)
    return np.stack([rr * np.cos(phi), rr * np.sin(phi), z], 1)


@pytest.mark.parametrize("case", ["disk", "annulus", "ball"])
def test_mapped_bound_radius_keeps_the_ellipsoid_inside(case):
    """Mapped bound (radius mode 2): brute force over the ellipsoid's boundary x + r S u, |u| = 1,
    shows it inside the outer circle / sphere and, for the annulus, outside the inner circle (whose
    centre stays outside the ellipsoid); r >= dist everywhere, r = dist when S = I, and for an
    anisotropic S the radius is larger than dist on average (a bound with |x - c| in place of
    |S (x - c)|, or a halved denominator of the inner bound, fails one of these)."""
    rng = np.random.default_rng({"disk": 1, "annulus": 2, "ball": 3}[case])
    if case == "disk":
        g = wi.Geometry(2, wi.DISK, (0.2, -0.1, 1.3), (8,))
    elif case == "annulus":
        g = wi.Geometry(2, wi.ANNULUS, (0.1, 0.2, 0.3, 1.0), (8, 8))
    else:
        g = wi.Geometry(3, wi.BALL, (0.1, -0.2, 0.3, 0.9), (4, 4))
    dim = g.dim
    c = np.asarray(g.params[:dim])
    R = g.params[dim] if case != "annulus" else g.params[3]
    x = wi.sample_points(g, 400, rng)
    # and points in the boundary layers, where the bound matters most
    dirs = _sphere_dirs(dim, 200)
    x = np.concatenate([x, c + dirs * (R - rng.uniform(1e-5, 1e-2, (200, 1)))])
    if case == "annulus":
        x = np.concatenate([x, c + dirs * (0.3 + rng.uniform(1e-5, 1e-2, (200, 1)))])
    U = _sphere_dirs(dim, 4096 if dim == 2 else 20000)
    gain = []
    for cond in (1.0, 4.0, 20.0):
        K = _random_spd(dim, cond, rng)
        _, _, S = walks.instance_setup(K, dim)
        Sd = S[:dim, :dim]
        r = walks.step_radii(g, S, x, 2)
        d, _ = walks.geom_eval(g, x)
        assert np.all(r >= d * (1 - 1e-12)), (cond, (r - d).min())
        if cond == 1.0:
            np.testing.assert_allclose(r, d, rtol=1e-10, atol=1e-14)
        else:
            gain.append(np.mean(r / d))
        Sinv = np.linalg.inv(Sd)
        for i in range(len(x)):
            pts = x[i] + r[i] * (U @ Sd.T) - c
            rho = np.sqrt((pts ** 2).sum(1))
            assert rho.max() <= R * (1 + 1e-12), (cond, i, rho.max() - R)
            if case == "annulus":
                assert rho.min() >= 0.3 * (1 - 1e-12), (cond, i, rho.min())
                assert np.linalg.norm(Sinv @ (c - x[i])) > r[i]
    assert min(gain) > 1.15, gain


def test_ellipse_mapped_bound_keeps_the_ellipsoid_inside_and_the_law():
    """Mapped bound on the ellipse (1 x 0.4): brute force over 4096 points of each step ellipsoid's
    boundary shows it inside the ellipse for three conductivities, r >= the Lipschitz distance bound,
    and the chain keeps the WoE chain's exit law and reproduces 2D-sol4 with far fewer steps."""
    rng = np.random.default_rng(41)
    g = wi.Geometry(2, wi.ELLIPSE, (0.1, -0.2, 1.0, 0.4), (24,))
    c, A = np.array([0.1, -0.2]), np.array([1.0, 0.4])
    x = wi.sample_points(g, 400, rng)
    t = rng.uniform(0, 2 * np.pi, 200)
    s = 1 - rng.uniform(1e-5, 1e-2, 200)
    x = np.concatenate([x, c + np.stack([A[0] * s * np.cos(t), A[1] * s * np.sin(t)], 1)])
    U = _sphere_dirs(2, 4096)
    gains = []
    for cond in (1.0, 4.0, 20.0):
        K = _random_spd(2, cond, rng)
        _, _, S = walks.instance_setup(K, 2)
        r = walks.step_radii(g, S, x, 2)
        d, _ = walks.geom_eval(g, x)
        assert np.all(r >= d)
        gains.append(np.mean(r / d))
        for i in range(len(x)):
            pts = (x[i] + r[i] * (U @ S[:2, :2].T) - c) / A
            assert np.sqrt((pts ** 2).sum(1)).max() <= 1 + 1e-12, (cond, i)
    assert min(gains) > 1.3, gains
    K = np.array([[1.0, 0.3], [0.3, 0.4]])
    x = wi.sample_points(g, 6, np.random.default_rng(23))
    N = 20_000
    c0, s0, _ = walks.build_measure(g, K, x, 1e-4, seed=5, walk_end=N, threads=8, radius_mode=0)
    c2, s2, _ = walks.build_measure(g, K, x, 1e-4, seed=6, walk_end=N, threads=8, radius_mode=2)
    assert s2["steps"] < 0.5 * s0["steps"] and s2["escapes"] == 0, (s0["steps"], s2["steps"])
    rep = statutil.two_sample(c0, N, c2, N)
    assert rep["ok"], rep
    _, _, S = walks.instance_setup(K, 2)
    assert np.all(_exit_mean_z(g, S, x, _sol4(K), 30_000, grad_bound=4.0, radius_mode=2) < 4.5)


@pytest.mark.parametrize("dim", [2, 3, "box"])
def test_perforated_mapped_bound_keeps_the_ellipsoid_inside_and_the_law(dim):
    """Mapped bound on a disc / ball / square with holes: each step ellipsoid (brute force over its
    boundary) stays in the outer circle, sphere or square and off every hole (whose centre it does not
    contain), r >= dist; the chain keeps the WoE chain's exit law with fewer steps."""
    box = dim == "box"
    dim = 2 if box else dim
    rng = np.random.default_rng(50 + dim + 7 * box)
    if box:
        g = wi.Geometry(2, wi.PERFBOX, (-1.0, -1.0, 1.0, 1.2), (13, 11),
                        verts=np.array([[0.5, 0.0, 0.2], [-0.4, 0.45, 0.3]]))
    elif dim == 2:
        g = wi.Geometry(2, wi.PERFORATED, (0.05, 0.0, 1.1), (24, 8, 3),
                        verts=np.array([[0.4, 0.1, 0.25], [-0.3, -0.35, 0.15], [-0.35, 0.45, 0.2]]))
    else:
        g = wi.Geometry(3, wi.PERFORATED, (0.02, 0.0, -0.03, 1.05), (4, 6, 3, 4),
                        verts=np.array([[0.35, 0.1, -0.05, 0.3], [-0.4, -0.2, 0.25, 0.25]]))
    c, R = np.asarray(g.params[:dim]), g.params[dim]
    lo, hi = np.asarray(g.params[:dim]), np.asarray(g.params[dim:2 * dim])
    holes = np.asarray(g.verts, float).reshape(-1, dim + 1)
    x = wi.sample_points(g, 300, rng)
    U = _sphere_dirs(dim, 2048 if dim == 2 else 6000)
    K = _random_spd(dim, 10.0, rng)
    _, _, S = walks.instance_setup(K, dim)
    Sd = S[:dim, :dim]
    r = walks.step_radii(g, S, x, 2)
    d, _ = walks.geom_eval(g, x)
    assert np.all(r >= d * (1 - 1e-12)) and np.mean(r / d) > 1.1
    Si = np.linalg.inv(Sd)
    for i in range(len(x)):
        pts = x[i] + r[i] * (U @ Sd.T)
        if box:
            assert np.all(pts >= lo - 1e-12) and np.all(pts <= hi + 1e-12)
        else:
            assert np.sqrt(((pts - c) ** 2).sum(1)).max() <= R * (1 + 1e-12)
        for h in holes:
            assert np.sqrt(((pts - h[:dim]) ** 2).sum(1)).min() >= h[dim] * (1 - 1e-12)
            assert np.linalg.norm(Si @ (h[:dim] - x[i])) > r[i]
    xs = wi.sample_points(g, 4, np.random.default_rng(60 + dim + 7 * box))
    N = 10_000
    c0, s0, _ = walks.build_measure(g, K, xs, 1e-4, seed=5, walk_end=N, threads=8, radius_mode=0)
    c2, s2, _ = walks.build_measure(g, K, xs, 1e-4, seed=6, walk_end=N, threads=8, radius_mode=2)
    assert s2["steps"] < 0.9 * s0["steps"] and s2["escapes"] == 0, (s0["steps"], s2["steps"])
    rep = statutil.two_sample(c0, N, c2, N)
    assert rep["ok"], rep


@pytest.mark.parametrize("case", ["disk", "annulus", "ball", "perforated2", "perforated3"])
def test_curved_mapped_exact_radius_is_the_largest_inscribed(case):
    """Mapped exact (radius mode 1) on circles and spheres: brute force over the boundary of each step
    ellipsoid x + r S u, |u| = 1, shows it inside the outer circle / sphere and off every inner circle,
    sphere or hole when shrunk by 1e-9; the distance from S^{-1} x to the mapped boundary, minimised
    numerically over the angles of the points c + R u(angles) of every circle / sphere (from the best of
    dense samples), equals r to 1e-9, so r is the largest inscribed radius; r >= the mapped bound,
    r = dist when S = I; the chain keeps the WoE chain's exit law with fewer steps (a root of the wrong
    matrix, S in place of S^{-1}, or a semi-axis R s_k in place of R / s_k fails one of these)."""
    rng = np.random.default_rng({"disk": 71, "annulus": 72, "ball": 73, "perforated2": 74, "perforated3": 75}[case])
    if case == "disk":
        g = wi.Geometry(2, wi.DISK, (0.2, -0.1, 1.3), (8,))
    elif case == "annulus":
        g = wi.Geometry(2, wi.ANNULUS, (0.1, 0.2, 0.3, 1.0), (8, 8))
    elif case == "ball":
        g = wi.Geometry(3, wi.BALL, (0.1, -0.2, 0.3, 0.9), (4, 4))
    elif case == "perforated2":
        g = wi.Geometry(2, wi.PERFORATED, (0.05, 0.0, 1.1), (24, 8, 3),
                        verts=np.array([[0.4, 0.1, 0.25], [-0.3, -0.35, 0.15], [-0.35, 0.45, 0.2]]))
    else:
        g = wi.Geometry(3, wi.PERFORATED, (0.02, 0.0, -0.03, 1.05), (4, 6, 3, 4),
                        verts=np.array([[0.35, 0.1, -0.05, 0.3], [-0.4, -0.2, 0.25, 0.25]]))
    dim = g.dim
    c = np.asarray(g.params[:dim])
    if g.kind == wi.ANNULUS:
        R, inner = g.params[3], [(c, g.params[2])]
    else:
        R = g.params[dim]
        inner = [(np.asarray(h[:dim]), h[dim]) for h in np.asarray(g.verts, float).reshape(-1, dim + 1)] \
            if g.kind == wi.PERFORATED else []
    x = wi.sample_points(g, 60, rng)
    U = _sphere_dirs(dim, 4096 if dim == 2 else 12000)
    Ud = _sphere_dirs(dim, 20_000)  # starting points of the local minimisation
    pieces = [(c, R)] + inner
    from scipy import optimize

    def u_of(ang):
        if dim == 2:
            return np.array([np.cos(ang[0]), np.sin(ang[0])])
        return np.array([np.sin(ang[0]) * np.cos(ang[1]), np.sin(ang[0]) * np.sin(ang[1]), np.cos(ang[0])])

    def mapped_distance(z, Si):
        best = np.inf
        for pc, pr in pieces:
            pts = (pc + pr * Ud) @ Si.T
            k = int(np.argmin(((pts - z) ** 2).sum(1)))
            u0 = Ud[k]
            a0 = [np.arctan2(u0[1], u0[0])] if dim == 2 else [np.arccos(np.clip(u0[2], -1, 1)), np.arctan2(u0[1], u0[0])]
            f = lambda a: np.linalg.norm(Si @ (pc + pr * u_of(a)) - z)
            if dim == 2:
                res = optimize.minimize_scalar(lambda t: f([t]), bracket=(a0[0] - 1e-3, a0[0], a0[0] + 1e-3),
                                               method="brent", tol=1e-14)
                val = res.fun
            else:
                res = optimize.minimize(f, a0, method="Nelder-Mead",
                                        options={"xatol": 1e-13, "fatol": 1e-16, "maxiter": 4000})
                val = res.fun
            best = min(best, val)
        return best

    def clearance(xi, ri, Sd):
        """Signed: >= 0 iff the ellipsoid x + ri S B lies in D (smallest margin over its boundary)."""
        pts = xi + ri * (U @ Sd.T)
        m = R - np.sqrt(((pts - c) ** 2).sum(1)).max()
        for hc, hr in inner:
            m = min(m, np.sqrt(((pts - hc) ** 2).sum(1)).min() - hr)
        return m

    for cond in (1.0, 6.0, 25.0):
        K = _random_spd(dim, cond, rng)
        _, _, S = walks.instance_setup(K, dim)
        Sd = S[:dim, :dim]
        r = walks.step_radii(g, S, x, 1)
        d, _ = walks.geom_eval(g, x)
        rb = walks.step_radii(g, S, x, 2)
        assert np.all(r >= rb * (1 - 1e-9)), (cond, (r - rb).min())
        if cond == 1.0:
            np.testing.assert_allclose(r, d, rtol=1e-9, atol=1e-13)
        Si = np.linalg.inv(Sd)
        for i in range(len(x)):
            assert clearance(x[i], r[i] * (1 - 1e-9), Sd) >= -1e-13, (cond, i)
            md = mapped_distance(Si @ x[i], Si)
            assert abs(r[i] - md) <= 1e-9 * md + 1e-14, (cond, i, r[i], md)
    xs = wi.sample_points(g, 4, np.random.default_rng(80))
    N = 10_000
    K = _random_spd(dim, 10.0, np.random.default_rng(81))
    c0, s0, _ = walks.build_measure(g, K, xs, 1e-4, seed=5, walk_end=N, threads=8, radius_mode=0)
    c1, s1, _ = walks.build_measure(g, K, xs, 1e-4, seed=6, walk_end=N, threads=8, radius_mode=1)
    assert s1["steps"] < 0.9 * s0["steps"] and s1["escapes"] == 0, (s0["steps"], s1["steps"])
    rep = statutil.two_sample(c0, N, c1, N)
    assert rep["ok"], rep


def test_mapped_bound_radius_same_law_fewer_steps():
    """The mapped-bound chain has the exit law of the WoE-bound chain (the two estimates agree within
    their sampling error) and takes far fewer steps on the anisotropic annulus."""
    g = wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.3, 1.0), (16, 16))
    K = np.array([[1.0, 0.5], [0.5, 2.0]])
    x = wi.sample_points(g, 6, np.random.default_rng(21))
    N = 20_000
    c0, s0, _ = walks.build_measure(g, K, x, 1e-4, seed=5, walk_end=N, threads=8, radius_mode=0)
    c2, s2, _ = walks.build_measure(g, K, x, 1e-4, seed=6, walk_end=N, threads=8, radius_mode=2)
    assert s2["steps"] < 0.6 * s0["steps"], (s0["steps"], s2["steps"])
    assert s2["escapes"] == 0
    rep = statutil.two_sample(c0, N, c2, N)
    assert rep["ok"], rep


def test_mapped_bound_reproduces_harmonic_functions():
    """E u(X_N) = u(x) under the mapped-bound chain: the paper's K-harmonic 2D-sol4 on an annulus and
    3D-sol1 composed with K^{-1/2} in an anisotropic ball."""
    K = np.array([[1.0, 0.3], [0.3, 0.4]])
    u = _sol4(K)
    g = wi.Geometry(2, wi.ANNULUS, (0.0, 0.0, 0.5, 1.0), (8, 8))
    x = wi.sample_points(g, 8, np.random.default_rng(7))
    _, _, S = walks.instance_setup(K, 2)
    z = _exit_mean_z(g, S, x, u, 40_000, grad_bound=3.0, radius_mode=2)
    assert np.all(z < 4.5), z
    import scipy.stats as st_
    Q = st_.special_ortho_group.rvs(3, random_state=3)
    K3 = Q @ np.diag([1.0, 2.0, 6.0]) @ Q.T
    Kis = wi.spd_inv_sqrt(K3)
    def u3(p):
        y = p @ Kis.T
        return y[:, 0] * y[:, 1] + y[:, 1] ** 2 - y[:, 2] ** 2
    gb = wi.Geometry(3, wi.BALL, (0.0, 0.0, 0.0, 1.0), (4, 4))
    xb = wi.sample_points(gb, 6, np.random.default_rng(10))
    _, _, S3 = walks.instance_setup(K3, 3)
    assert np.all(_exit_mean_z(gb, S3, xb, u3, 30_000, grad_bound=6.0, radius_mode=2) < 4.5)


def _inside_polygon(P, V):
    """Crossing-number point-in-polygon test (points P, vertices V counter-clockwise)."""
    inside = np.zeros(len(P), bool)
    for a, b in zip(V, np.roll(V, -1, 0)):
        crosses = (a[1] > P[:, 1]) != (b[1] > P[:, 1])
        with np.errstate(divide="ignore", invalid="ignore"):
            xc = a[0] + (P[:, 1] - a[1]) * (b[0] - a[0]) / (b[1] - a[1])
        inside ^= crosses & (P[:, 0] < xc)
    return inside


def _in_l_shape(P):
    """Closed-form membership in the L-shape (0, 1)^2 minus [0.5, 1) x [0.5, 1)."""
    x, y = P[:, 0], P[:, 1]
    return (x > 0) & (x < 1) & (y > 0) & (y < 1) & ~((x >= 0.5) & (y >= 0.5))


def test_polygon_distance_is_signed():
    """The polygon's distance is negative outside D (a start point there stops at once and counts as
    an escape): its sign against the closed-form membership of the L-shape, its magnitude against the
    nearest of dense boundary samples, on points around the shape and in its notch."""
    g = wi.Geometry(2, wi.POLYGON, (), (50,), verts=wi.L_SHAPE)
    rng = np.random.default_rng(21)
    P = rng.uniform(-0.4, 1.4, size=(4000, 2))
    bp, _ = _boundary_samples(g, 400_000)
    dmin, _ = cKDTree(bp).query(P)
    keep = dmin > 1e-4  # the sign is only defined away from the boundary
    P, dmin = P[keep], dmin[keep]
    d, _ = walks.geom_eval(g, P)
    inside = _in_l_shape(P)
    assert inside.sum() > 500 and (~inside).sum() > 500
    assert np.array_equal(d > 0, inside)
    assert np.max(np.abs(np.abs(d) - dmin)) <= 2e-5


def test_walks_from_outside_the_polygon_stop_at_once_as_escapes():
    """Start points outside D (the notch, beyond an edge, beyond a corner) stop with zero steps in the
    cell of their projection and count as escapes; the start points inside walk as usual."""
    g = wi.Geometry(2, wi.POLYGON, (), (50,), verts=wi.L_SHAPE)
    x = np.array([[0.75, 0.75], [1.2, 0.3], [-0.1, -0.2], [0.501, 0.9], [0.25, 0.25], [0.8, 0.2]])
    out = ~_in_l_shape(x)
    assert out.tolist() == [True, True, True, True, False, False]
    inst = wi.Instance(g, np.array([[1.0, 0.5], [0.5, 2.0]]), x, 200, eps=1e-4, seed=77, precision=wi.FP64)
    c, st, tr = walks.build_instance(inst, trace=True)
    _, e_proj = walks.geom_eval(g, x)
    assert np.all(tr[out, :, 1] == 0)
    assert np.all(tr[out, :, 0] == e_proj[out][:, None])
    assert st["escapes"] == out.sum() * 200
    assert np.all(tr[~out, :, 1] > 0)
    assert np.all(c.sum(1) == 200)


def test_polygon_mapped_exact_radius_is_the_largest_inscribed():
    """Mapped-exact radius on the L-shape: the ellipsoid x + r S B(0,1) shrunk by 1e-9 lies inside
    the polygon (brute force over its boundary), and a dense sampling of the polygon's edges finds a
    point at mapped distance |S^{-1}(z - x)| within 1e-4 of r, so no larger ellipsoid fits; r >= dist,
    r = dist for S = I."""
    rng = np.random.default_rng(31)
    V = np.asarray(wi.L_SHAPE, float)
    g = wi.Geometry(2, wi.POLYGON, (), (24,), verts=V)
    x = wi.sample_points(g, 150, rng)
    # edge samples for the maximality check
    Z = np.concatenate([a + np.linspace(0, 1, 20001)[:, None] * (b - a) for a, b in zip(V, np.roll(V, -1, 0))])
    U = _sphere_dirs(2, 4096)
    for cond in (1.0, 4.0, 20.0):
        K = _random_spd(2, cond, rng)
        _, _, S = walks.instance_setup(K, 2)
        Sd = S[:2, :2]
        r = walks.step_radii(g, S, x, 1)
        d, _ = walks.geom_eval(g, x)
        assert np.all(r >= d * (1 - 1e-12))
        if cond == 1.0:
            np.testing.assert_allclose(r, d, rtol=1e-12, atol=1e-15)
        Si = np.linalg.inv(Sd)
        for i in range(len(x)):
            pts = x[i] + (r[i] * (1 - 1e-9)) * (U @ Sd.T)
            assert _inside_polygon(pts, V).all(), (cond, i)
            dz = np.sqrt((((Z - x[i]) @ Si.T) ** 2).sum(1))
            k = int(np.argmin(dz))  # refine between the neighbouring samples
            lo, hi = Z[max(k - 1, 0)], Z[min(k + 1, len(Z) - 1)]
            Zf = lo + np.linspace(0, 1, 20001)[:, None] * (hi - lo)
            md = min(dz[k], np.sqrt((((Zf - x[i]) @ Si.T) ** 2).sum(1)).min())
            assert md <= r[i] * (1 + 1e-4) + 1e-12, (cond, i, md, r[i])


def test_polygon_mapped_exact_same_law_fewer_steps():
    """On the L-shape with an anisotropic K the mapped-exact chain has the WoE chain's exit law
    and reproduces the paper's K-harmonic 2D-sol4, with fewer steps."""
    K = np.array([[1.0, 0.3], [0.3, 0.4]])
    g = wi.Geometry(2, wi.POLYGON, (), (24,), verts=wi.L_SHAPE)
    x = wi.sample_points(g, 6, np.random.default_rng(22))
    N = 20_000
    c0, s0, _ = walks.build_measure(g, K, x, 1e-4, seed=5, walk_end=N, threads=8, radius_mode=0)
    c1, s1, _ = walks.build_measure(g, K, x, 1e-4, seed=6, walk_end=N, threads=8, radius_mode=1)
    assert s1["steps"] < 0.8 * s0["steps"], (s0["steps"], s1["steps"])
    assert s1["escapes"] == 0
    rep = statutil.two_sample(c0, N, c1, N)
    assert rep["ok"], rep
    _, _, S = walks.instance_setup(K, 2)
    z = _exit_mean_z(g, S, x, _sol4(K), 30_000, grad_bound=4.0, radius_mode=1)
    assert np.all(z < 4.5), z


def test_bauer_voronoi_cells():
    """Sphere layout (n, 0): the extrinsic Voronoi cells (Appendix Ex. A.2) of n nodes of Bauer's
    spiral.  The nodes follow Section 5.3's formula (unit length, z equally spaced); on the paper's
    concentric shell (Example 6: 1000 outer, 100 inner nodes) the oracle's cell of points in both
    eps-shells is the nearest node over all 1100 nodes (brute force, lowest index on ties); the cell
    measures sum to 4 pi R^2 and match the frequencies of 2e6 uniform points (z-scores below 5.5)."""
    n = 1000
    u = wi.bauer_spiral(n)
    np.testing.assert_allclose((u ** 2).sum(1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(u[:, 2], 1 - (2 * np.arange(1, n + 1) - 1) / n, atol=1e-14)
    g = wi.Geometry(3, wi.PERFORATED, (0.0, 0.0, 0.0, 1.0), (1000, 0, 100, 0),
                    verts=np.array([[0.0, 0.0, 0.0, 0.5]]))
    assert g.n_elem == 1100
    rng = np.random.default_rng(3)
    v = rng.normal(size=(6000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    t = rng.uniform(0, 1e-3, (6000, 1))
    pts = np.concatenate([v[:3000] * (1 - t[:3000]), v[3000:] * (0.5 + t[3000:])])
    _, e = walks.geom_eval(g, pts)
    nodes = np.concatenate([u, 0.5 * wi.bauer_spiral(100)])
    np.testing.assert_array_equal(e, np.argmin(((pts[:, None, :] - nodes[None]) ** 2).sum(2), 1))
    sig = walks.element_measures(g)
    assert abs(sig[:1000].sum() - 4 * np.pi) < 1e-10 and abs(sig[1000:].sum() - np.pi) < 1e-10
    gb = wi.Geometry(3, wi.BALL, (0.1, 0.0, -0.2, 1.0), (1000, 0))
    w = rng.normal(size=(2_000_000, 3))
    w /= np.linalg.norm(w, axis=1)[:, None]
    _, eb = walks.geom_eval(gb, np.asarray(gb.params[:3]) + w * (1 - 1e-6))
    cnt = np.bincount(eb, minlength=1000)
    p = walks.element_measures(gb) / (4 * np.pi)
    z = (cnt - 2e6 * p) / np.sqrt(2e6 * p * (1 - p))
    assert np.abs(z).max() < 5.5, np.abs(z).max()


def test_radius_modes_rejected_where_they_do_not_apply():
    g = wi.Geometry(2, wi.POLYGON, (), (16,), verts=wi.L_SHAPE)
    assert np.isnan(walks.step_radii(g, np.eye(3), [[0.5, 0.5]], 2)).all()
    assert np.isnan(walks.step_radii(wi.Geometry(2, wi.ELLIPSE, (0.0, 0.0, 1.0, 0.5), (8,)), np.eye(3),
                                     [[0.1, 0.1]], 1)).all()
    with pytest.raises(ValueError):
        walks.walk_exits(g, np.eye(3), [0.5, 0.5], 1e-4, 4, radius_mode=2)
    gb = wi.Geometry(2, wi.BOX, (0.0, 0.0, 1.0, 1.0), (4,))
    with pytest.raises(ValueError):
        walks.walk_exits(gb, np.eye(3), [0.5, 0.5], 1e-4, 4, radius_mode=3)
    ge = wi.Geometry(2, wi.ELLIPSE, (0.0, 0.0, 1.0, 0.5), (8,))
    with pytest.raises(ValueError):
        walks.walk_exits(ge, np.eye(3), [0.1, 0.1], 1e-4, 4, radius_mode=1)


# ---------------------------------------------------------------- exact invariants

def test_row_sums_threads_and_resume_exact():
    inst = wi.cfg2_annulus(n_walks=600, n_obs=64)
    a, sa, _ = walks.build_instance(inst, threads=1)
    b, sb, _ = walks.build_instance(inst, threads=7)
    assert np.array_equal(a, b) and sa == sb
    assert np.all(a.sum(1) == 600)
    c, _, _ = walks.build_instance(inst, walk_begin=0, walk_end=217, threads=3)
    walks.build_instance(inst, walk_begin=217, walk_end=600, threads=5, counts=c)
    assert np.array_equal(a, c)


def test_scale_invariance_of_K_is_exact():
    """Only Khat = K / lambda_max enters the walk (Section 4.2), so scaling K by a power of two
    changes nothing, bit for bit."""
    inst = wi.cfg2_annulus(n_walks=500, n_obs=48)
    a, _, _ = walks.build_instance(inst, threads=8)
    inst.K = inst.K * 4.0
    b, _, _ = walks.build_instance(inst, threads=8)
    assert np.array_equal(a, b)


def test_step_cap_and_boundary_start():
    inst = wi.cfg1_disk(n_walks=300)
    inst.max_steps = 1
    c, st, _ = walks.build_instance(inst, threads=4)
    assert np.all(c.sum(1) == 300)
    # every walk takes exactly one step; it is capped unless that step landed in the eps-shell
    assert st["walks"] == 64 * 300 and st["steps"] == st["walks"]
    assert 0.95 * st["walks"] < st["cap_hits"] < st["walks"]
    # a start inside the eps-shell stops with zero steps in the element of its projection
    g = wi.Geometry(2, wi.DISK, (0.0, 0.0, 1.0), (8,))
    x = np.array([[np.cos(0.3) * (1 - 5e-5), np.sin(0.3) * (1 - 5e-5)]])
    c, st, tr = walks.build_measure(g, np.eye(2), x, 1e-4, walk_end=50, trace=True)
    assert c[0, 0] == 50 and st["steps"] == 0 and np.all(tr[0, :, 1] == 0)


def test_empty_inputs():
    g = wi.Geometry(2, wi.DISK, (0.0, 0.0, 1.0), (8,))
    c, st, _ = walks.build_measure(g, np.eye(2), np.zeros((0, 2)), 1e-4, walk_end=10)
    assert c.shape == (0, 8) and st["walks"] == 0
    c, st, _ = walks.build_measure(g, np.eye(2), np.zeros((3, 2)), 1e-4, walk_begin=5, walk_end=5)
    assert c.sum() == 0 and st["walks"] == 0


# ---------------------------------------------------------------- perforated disc (multiply connected)

def test_perforated_with_one_concentric_hole_is_the_annulus_walk_for_walk():
    """One hole at the centre of the outer disc is an annulus: the same distances, the same nearest
    circle (ties to the outer one), the same arcs in the same order, hence identical counts."""
    gp = wi.Geometry(2, wi.PERFORATED, (0.1, -0.2, 1.0), (23, 11, 1), verts=np.array([[0.1, -0.2, 0.35]]))
    ga = wi.Geometry(2, wi.ANNULUS, (0.1, -0.2, 0.35, 1.0), (23, 11))
    x = wi.sample_points(ga, 9, np.random.default_rng(31))
    K = np.array([[1.0, 0.3], [0.3, 0.5]])
    cp, sp, tp = walks.build_measure(gp, K, x, 1e-4, seed=77, walk_end=600, trace=True)
    ca, sa, ta = walks.build_measure(ga, K, x, 1e-4, seed=77, walk_end=600, trace=True)
    assert np.array_equal(tp, ta) and np.array_equal(cp, ca) and sp == sa
    assert np.allclose(walks.element_measures(gp), walks.element_measures(ga), rtol=1e-15, atol=0)


def test_perforated_disc_matches_the_papers_average_measure():
    """The paper's Example with a disc perforated by five smaller discs (K = I): the harmonic measure
    of the holes averaged over the points of the circle at distance 0.05 from the outer one is about
    0.1126 (the paper's value; its Monte Carlo error is not stated, so the bound is loose).  100
    points x 20 000 walks: standard error 2e-4; eps = 1e-4 instead of the paper's 1e-10."""
    inst = wi.perforated_disk_example(n_walks=20_000)
    c, st, _ = walks.build_instance(inst)
    assert st["escapes"] == 0 and st["cap_hits"] == 0
    g1 = inst.geom.gamma1_mask.astype(bool)
    avg = c[:, g1].sum(1).mean() / inst.n_walks
    assert abs(avg - 0.1126) < 0.002, avg
    # symmetric under rotation by 2 pi / 5: the five holes take equal shares
    share = c[:, g1].reshape(100, 5, -1).sum((0, 2)) / c[:, g1].sum()
    assert np.all(np.abs(share - 0.2) < 0.01), share


def test_perforated_disc_reproduces_paper_solution():
    """2D-sol3 (harmonic) from the stop points: E u(X_N) = u(x) within the Monte Carlo error and the
    O(eps) bias."""
    inst = wi.perforated_disk_example()
    g = inst.geom
    x = wi.sample_points(g, 6, np.random.default_rng(12), margin=0.02)
    _, _, S = walks.instance_setup(np.eye(2), 2)
    sol3 = lambda p: p[:, 0] ** 2 - p[:, 1] ** 2
    assert np.all(_exit_mean_z(g, S, x, sol3, 30_000, grad_bound=2.0) < 4.5)


def test_fixed_iteration_walk():
    """eps = 0: the fixed-iteration loop (Remark on Algorithm MC-REM, item (i)).  Every walk makes
    exactly n steps unless it reaches dD (dist <= 0 in FP64) first, and its last point is binned.  The
    distance to the boundary shrinks geometrically, so at n = 8 the disk estimate already matches the
    Poisson-kernel closed form at N = 10^4 while n = 3 is visibly biased (walks still well inside D)."""
    inst = wi.cfg1_disk()
    P = cf.disk_H(inst.x_obs, 1.0, 64)
    c3, st3, _ = walks.build_measure(inst.geom, inst.K, inst.x_obs, 0.0, max_steps=3, walk_end=10_000, threads=8)
    assert st3["cap_hits"] == st3["walks"] == 640_000 and st3["steps"] == 3 * 640_000
    assert not statutil.vs_probabilities(c3, 10_000, P)["ok"]
    c8, st8, _ = walks.build_measure(inst.geom, inst.K, inst.x_obs, 0.0, max_steps=8, walk_end=10_000, threads=8)
    assert np.all(c8.sum(1) == 10_000) and st8["max_steps"] == 8 and st8["cap_hits"] >= 0.99 * st8["walks"]
    assert statutil.vs_probabilities(c8, 10_000, P)["ok"] and statutil.row_chi2(c8, 10_000, P)["ok"]
    # a walk that stops before n is on dD to FP64 resolution: its stop point rounds onto the circle
    _, _, S = walks.instance_setup(np.eye(2), 2)
    pos = walks.walk_exits(inst.geom, S, inst.x_obs[0], 0.0, 2000, max_steps=200)
    assert np.all(np.abs(np.hypot(pos[:, 0], pos[:, 1]) - 1.0) <= 4e-16)
    # eps = 0 needs its step count
    with pytest.raises(Exception):
        walks.build_measure(inst.geom, inst.K, inst.x_obs, 0.0, max_steps=0, walk_end=10, threads=1)


def test_concentric_spherical_shell_inner_mass():
    """Examples 6 and 7 of Section 5.3 are balls with a ball removed.  For the concentric shell
    R_1 < |x| < R_0 the harmonic measure of the inner sphere seen from radius rho is the Newtonian
    ratio (1/rho - 1/R_0) / (1/R_1 - 1/R_0) (the radial harmonic function with boundary values 1, 0),
    whatever the direction."""
    g = wi.spherical_shell_example(6).geom
    rng = np.random.default_rng(5)
    dirs = rng.standard_normal((6, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    rho = np.array([0.55, 0.6, 0.7, 0.8, 0.9, 0.95])
    x = dirs * rho[:, None]
    N = 20_000
    counts, st, _ = walks.build_measure(g, np.eye(3), x, 1e-6, seed=9, walk_end=N, threads=8)
    inner = counts[:, g.gamma1_mask == 1].sum(1) / N
    p = (1 / rho - 1.0) / (1 / 0.5 - 1.0)
    assert np.all(np.abs(inner - p) < 4.5 * np.sqrt(p * (1 - p) / N) + 1e-5), (inner, p)
    assert st["escapes"] == 0 and st["cap_hits"] == 0


def test_perforated_domains_reproduce_paper_solutions():
    """Harmonic functions from the stop points, E u(X_N) = u(x) within the Monte Carlo error and the
    O(eps) bias: 3D-sol1 and 3D-sol2 = 1/|x| (harmonic in D: the origin lies inside the removed ball)
    on the eccentric shell of Example 7; 2D-sol2 and 2D-sol3 on the square with a hole of Examples 1
    and 5."""
    _, _, S3 = walks.instance_setup(np.eye(3), 3)
    g = wi.spherical_shell_example(7).geom
    x = wi.sample_points(g, 5, np.random.default_rng(13), margin=0.02)
    sol1 = lambda p: p[:, 0] * p[:, 1] + p[:, 1] ** 2 - p[:, 2] ** 2
    sol2 = lambda p: 1.0 / np.sqrt((p ** 2).sum(1))
    assert np.all(_exit_mean_z(g, S3, x, sol1, 20_000, grad_bound=3.0) < 4.5)
    assert np.all(_exit_mean_z(g, S3, x, sol2, 20_000, grad_bound=25.0) < 4.5)
    _, _, S2 = walks.instance_setup(np.eye(2), 2)
    g = wi.square_hole_example(1).geom
    x = wi.sample_points(g, 5, np.random.default_rng(14), margin=0.02)
    sol2d = lambda p: -p[:, 0] ** 3 / 3 - p[:, 0] ** 2 * p[:, 1] + p[:, 0] * p[:, 1] ** 2 + p[:, 1] ** 3 / 3
    sol3d = lambda p: p[:, 0] ** 2 - p[:, 1] ** 2
    assert np.all(_exit_mean_z(g, S2, x, sol2d, 20_000, grad_bound=5.0) < 4.5)
    assert np.all(_exit_mean_z(g, S2, x, sol3d, 20_000, grad_bound=3.0) < 4.5)
    # log |x - c| (c the hole's centre) is harmonic in D but not in the square: reproduced by the
    # walks of D, visibly not by a planted slip that leaves the hole out of the distance
    logc = lambda p: 0.5 * np.log((p[:, 0] - 0.5) ** 2 + p[:, 1] ** 2)
    xh = np.array([[0.5, 0.25], [0.75, 0.05], [0.28, -0.05]])
    assert np.all(_exit_mean_z(g, S2, xh, logc, 20_000, grad_bound=5.0) < 4.5)
    g_nohole = wi.Geometry(2, wi.BOX, g.params, (g.layout[0],))
    assert _exit_mean_z(g_nohole, S2, xh, logc, 20_000, grad_bound=5.0).max() > 8


# ------------------------------------------------------------------------------ triangle meshes

def _tri_dist_normal_equations(T, x):
    """Distance from x to the triangle T = (a, b, c) by another route than the oracle's: the nearest
    point of the triangle's plane from the 2 x 2 normal equations in the barycentric coordinates
    (v, w) of a + v (b - a) + w (c - a); if v, w >= 0 and v + w <= 1 it is the nearest point of the
    triangle, else the nearest point lies on one of the three edges (closed-form clamped projection)."""
    a, b, c = T
    e1, e2, r = b - a, c - a, x - a
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    v, w = np.linalg.solve(G, np.array([e1 @ r, e2 @ r]))
    if v >= 0 and w >= 0 and v + w <= 1:
        return np.linalg.norm(r - v * e1 - w * e2)
    best = np.inf
    for p, q in ((a, b), (b, c), (c, a)):
        e = q - p
        t = np.clip((x - p) @ e / (e @ e), 0.0, 1.0)
        best = min(best, np.linalg.norm(x - p - t * e))
    return best


def test_triangle_distance_matches_two_independent_routes():
    """The oracle's triangle distance (projection inside the triangle by the three in-plane edge
    normals, else the nearest edge) equals the normal-equation route to 1e-12 on random triangles
    (from slivers of aspect 1/20 to equilateral) and points near faces, edges, vertices and far away,
    and lies within the sampling resolution of a dense barycentric sampling of the triangle (and
    never above it).  A one-triangle mesh gives the unsigned distance."""
    rng = np.random.default_rng(31)
    checked = 0
    for trial in range(60):
        T = rng.standard_normal((3, 3))
        if trial % 3 == 0:  # flattened triangles
            T[2] = T[0] + (T[1] - T[0]) * rng.uniform(0.2, 0.8) + rng.standard_normal(3) * 0.05
        g = wi.Geometry(3, wi.TRIMESH, (), (1,), verts=T[None])
        # points: random, near each vertex and edge midpoint, and above the face
        P = [rng.standard_normal((10, 3)) * 2.0]
        for p in (T[0], T[1], T[2], 0.5 * (T[0] + T[1]), 0.5 * (T[1] + T[2]), T.mean(0)):
            P.append(p + rng.standard_normal((4, 3)) * 0.05)
        P = np.concatenate(P)
        d, e = walks.geom_eval(g, P)
        d = np.abs(d)
        assert np.all(e == 0)
        ref = np.array([_tri_dist_normal_equations(T, p) for p in P])
        np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-14)
        s = np.linspace(0, 1, 201)
        V, W = np.meshgrid(s, s, indexing="ij")
        m = (V + W) <= 1
        pts = T[0] + V[m][:, None] * (T[1] - T[0]) + W[m][:, None] * (T[2] - T[0])
        dense = np.sqrt(((P[:, None, :] - pts[None]) ** 2).sum(2)).min(1)
        h = 0.5 / 200 * (np.linalg.norm(T[1] - T[0]) + np.linalg.norm(T[2] - T[0]))
        assert np.all(d <= dense + 1e-12) and np.all(dense <= d + h)
        checked += len(P)
    assert checked > 1000


def test_mesh_box_is_the_box_kind():
    """A box as a triangle mesh (two triangles per patch, in the BOX kind's patch order) is the BOX
    kind: the same distance at interior points (to rounding: the plane distance |n.(x - a)| / |n| and
    the coordinate difference round differently), the same cells, the same cell measures, and the
    oracle's walks on both give the same exit cell and step count walk for walk."""
    g = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.box_mesh([0.1, -0.2, 0.0], [1.1, 0.6, 1.5], 6))
    gb = wi.Geometry(3, wi.BOX, (0.1, -0.2, 0.0, 1.1, 0.6, 1.5), (6,))
    rng = np.random.default_rng(32)
    x = wi.sample_points(gb, 400, rng)
    d, e = walks.geom_eval(g, x)
    db, eb = walks.geom_eval(gb, x)
    np.testing.assert_allclose(d, db, rtol=0, atol=4e-16)
    assert np.array_equal(e, eb)
    np.testing.assert_allclose(walks.element_measures(g), walks.element_measures(gb), rtol=1e-14)
    xo = rng.uniform(-0.5, 2.0, (300, 3))
    out = ~np.all((xo > [0.1, -0.2, 0.0]) & (xo < [1.1, 0.6, 1.5]), 1)
    do, _ = walks.geom_eval(g, xo)
    assert np.all(do[out] < 0) and np.all(do[~out] > 0)
    K = _random_spd(3, 8.0, np.random.default_rng(33))
    xs = wi.sample_points(gb, 6, rng)
    c1, s1, t1 = walks.build_measure(g, K, xs, 1e-4, seed=3, walk_end=400, threads=8, trace=True)
    c0, s0, t0 = walks.build_measure(gb, K, xs, 1e-4, seed=3, walk_end=400, threads=8, trace=True)
    assert np.mean(np.all(t1 == t0, axis=2)) >= 0.999 and np.abs(c1 - c0).sum() <= 0.002 * c0.sum()


def test_mesh_start_points_outside_are_escapes_and_inside_by_winding():
    """The winding-number inside test on the non-convex L-prism equals the analytic membership of
    the prism (points in the notch, beside and above it are outside); walks from outside start points
    stop at once as escapes in the cell of the nearest triangle, walks from inside never escape."""
    T = wi.l_prism_mesh(8)
    g = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=T)
    rng = np.random.default_rng(34)
    P = rng.uniform(-0.25, 1.25, (3000, 3))
    ins = (np.all((P > 0) & (P < 1), 1) & ~((P[:, 0] > 0.5) & (P[:, 1] > 0.5)))
    far = np.abs(walks.geom_eval(g, P)[0]) > 1e-9
    d, _ = walks.geom_eval(g, P[far])
    assert np.array_equal(d > 0, ins[far])
    xo = np.array([[0.75, 0.75, 0.5], [1.2, 0.3, 0.5], [0.3, 0.3, 1.1]])
    c, st, tr = walks.build_measure(g, np.eye(3), xo, 1e-4, seed=1, walk_end=50, threads=4, trace=True)
    assert st["escapes"] == 150 and st["steps"] == 0
    _, e = walks.geom_eval(g, xo)
    assert np.all(c[np.arange(3), e] == 50)
    xi = wi.sample_points(g, 5, rng)
    _, st, _ = walks.build_measure(g, np.eye(3), xi, 1e-4, seed=1, walk_end=500, threads=4)
    assert st["escapes"] == 0 and st["steps"] > 0


def test_mesh_walk_reproduces_harmonic_functions():
    """E u(X_N) = u(x) for K-harmonic u on the non-convex L-prism with an anisotropic K (u = x^T A x
    + b.x with tr(K A) = 0); the slip S = Khat in place of Khat^{1/2} fails."""
    K = np.array([[1.0, 0.3, 0.1], [0.3, 0.6, -0.2], [0.1, -0.2, 0.4]])
    A = np.array([[1.0, 0.5, 0.0], [0.5, -0.8, 0.3], [0.0, 0.3, 0.0]])
    A[2, 2] = -(np.trace(K @ A) - K[2, 2] * A[2, 2]) / K[2, 2]
    assert abs(np.trace(K @ A)) < 1e-12
    bvec = np.array([0.3, -0.2, 0.5])
    u = lambda p: np.einsum("pi,ij,pj->p", p, A, p) + p @ bvec
    g = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.l_prism_mesh(2))  # 44 triangles
    x = wi.sample_points(g, 6, np.random.default_rng(35))
    _, Khat, S = walks.instance_setup(K, 3)
    z = _exit_mean_z(g, S, x, u, 20_000, grad_bound=6.0)
    assert np.all(z < 4.5), z
    Sw = np.zeros((3, 3))
    Sw[:3, :3] = Khat
    zw = _exit_mean_z(g, Sw, x, u, 20_000, grad_bound=6.0)
    assert zw.max() > 8, zw


def test_mesh_mapped_exact_radius():
    """Mapped-exact radius of a mesh (the distance from S^{-1} x to the mapped triangles S^{-1} T): on
    the box as a mesh it equals the BOX kind's exact radius min_a gap_a / |S e_a|; on the non-convex
    L-prism it equals a numpy route (normal equations on the mapped triangles) to 1e-12 and the step
    ellipsoid shrunk by 1e-9 lies in the prism (analytic membership of 4096 boundary points each);
    r = dist for S = I; the chain keeps the WoE chain's exit law with fewer steps (the slips S for
    S^{-1} or the transposed adjugate fail the first two checks)."""
    rng = np.random.default_rng(36)
    K = _random_spd(3, 10.0, np.random.default_rng(37))
    _, _, S = walks.instance_setup(K, 3)
    Sd = S[:3, :3]
    Si = np.linalg.inv(Sd)
    gm = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.box_mesh([0.1, -0.2, 0.0], [1.1, 0.6, 1.5], 6))
    gb = wi.Geometry(3, wi.BOX, (0.1, -0.2, 0.0, 1.1, 0.6, 1.5), (6,))
    x = wi.sample_points(gb, 300, rng)
    np.testing.assert_allclose(walks.step_radii(gm, S, x, 1), walks.step_radii(gb, S, x, 1), rtol=1e-12)
    T = wi.l_prism_mesh(4)
    g = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=T)
    x = wi.sample_points(g, 60, rng)
    r = walks.step_radii(g, S, x, 1)
    MT = T @ Si.T
    ref = np.array([min(_tri_dist_normal_equations(M, Si @ p) for M in MT) for p in x])
    np.testing.assert_allclose(r, ref, rtol=1e-12, atol=1e-15)
    U = _sphere_dirs(3, 4096)
    for p, rr in zip(x, r):
        q = p + rr * (1 - 1e-9) * (U @ Sd.T)
        inside = (np.all((q > -1e-15) & (q < 1 + 1e-15), 1) & ~((q[:, 0] > 0.5 + 1e-15) & (q[:, 1] > 0.5 + 1e-15)))
        assert inside.all()
    d, _ = walks.geom_eval(g, x)
    np.testing.assert_allclose(walks.step_radii(g, np.eye(3), x, 1), d, rtol=1e-12, atol=1e-15)
    xs = wi.sample_points(wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.l_prism_mesh(2)), 4, rng)
    g2 = wi.Geometry(3, wi.TRIMESH, (), (2,), verts=wi.l_prism_mesh(2))
    N = 10_000
    c0, s0, _ = walks.build_measure(g2, K, xs, 1e-4, seed=5, walk_end=N, threads=8, radius_mode=0)
    c1, s1, _ = walks.build_measure(g2, K, xs, 1e-4, seed=6, walk_end=N, threads=8, radius_mode=1)
    assert s1["steps"] < 0.7 * s0["steps"] and s1["escapes"] == 0, (s0["steps"], s1["steps"])
    rep = statutil.two_sample(c0, N, c1, N)
    assert rep["ok"], rep


def test_shell_bias_is_first_order_in_eps():
    """The eps-shell bias is O(eps) (the order the shell-bias allowances of the parity rules assume):
    for a harmonic u, E u(X_N) = u(x) exactly (optional stopping), so the bias of binning at the
    projection, E u(pi(X_N)) - u(x), equals E[u(pi(X_N)) - u(X_N)], whose per-walk terms are O(eps) and
    make a precise mean (standard error about 1 % of it).  Over eps = 0.04 -> 0.005 (three halvings)
    the bias divided by eps stays within 8 % of its mean on the unit disc (u = x^2 - y^2, pi(X) =
    X / |X|) and on the unit cube (u = x^2 - z^2, pi onto the nearest face): first order, not
    eps log(1/eps) (which would grow by 1.25-1.5 per halving here) nor sqrt(eps).  A projection
    skipped (binning X_N itself) makes the bias vanish and fails the nonzero check."""
    eps_list = [0.04, 0.02, 0.01, 0.005]
    n = 120_000

    def ratios(g, x0, u, proj):
        out = []
        for e in eps_list:
            X = walks.walk_exits(g, np.eye(3), x0, e, n, seed=21)
            out.append(np.mean(u(proj(X)) - u(X)) / e)
        return np.array(out)

    disk = wi.Geometry(2, wi.DISK, (0.0, 0.0, 1.0), (16,))
    r_disk = ratios(disk, np.array([0.6, 0.1]), lambda p: p[:, 0] ** 2 - p[:, 1] ** 2,
                    lambda X: X / np.linalg.norm(X, axis=1, keepdims=True))

    def cube_proj(X):
        P = X.copy()
        gaps = np.concatenate([X, 1 - X], 1)
        k = np.argmin(gaps, 1)
        rows = np.arange(len(X))
        P[rows, k % 3] = np.where(k < 3, 0.0, 1.0)
        return P

    cube = wi.Geometry(3, wi.BOX, (0.0, 0.0, 0.0, 1.0, 1.0, 1.0), (4,))
    r_cube = ratios(cube, np.array([0.3, 0.55, 0.7]), lambda p: p[:, 0] ** 2 - p[:, 2] ** 2, cube_proj)
    for r in (r_disk, r_cube):
        assert np.all(np.abs(r - r.mean()) <= 0.08 * abs(r.mean())), r
        assert abs(r.mean()) > 0.1, r
