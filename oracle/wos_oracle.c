/*
 * wos_oracle.c -- plain FP64 CPU reference of the walk-on-ellipsoids (WoE) Monte Carlo estimator
 * of the discretised elliptic measure.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the HIP path is compared against.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant generator with the
 * HIP library: it is written from the paper and from the published Philox definition.
 *
 * What it computes (paper, Section 4 and Algorithm "MC-REM" of Section 5.1):
 *   For observation point x_i and walk k:
 *     X_0 = x_i;  X_{n+1} = X_n + r(X_n) * S * U_n,  U_n uniform on the unit sphere,
 *   where S = Khat^{1/2}, Khat = K / lambda_max(K) (the paper assumes lambda_max = 1 without loss of
 *   generality; the walk-on-ellipsoids chain, Section 4.2 eq. "wos chain"), and r(x) is the step
 *   radius: r = dist(x, dD) ("WoE bound"), or, for boxes and polygons, the largest r with
 *   x + r S B(0,1) inside D ("mapped exact"), or, for discs, balls and boxes with holes, discs,
 *   annuli, balls and ellipses, a larger radius certified by a support bound ("mapped bound", see
 *   step_radius).  The chain stops at N_eps = min{ n >= 0 : dist(X_n, dD) <= eps } (eq. "N
 *   epsilon x"), tested before each step.  eps = 0 is the fixed-iteration loop of the Remark on
 *   Algorithm MC-REM, item (i): the chain makes exactly max_steps steps (it stops earlier only on
 *   reaching dD, dist <= 0) and its last point is binned.  D may also be the interior of a closed
 *   triangle surface (a mesh; the Remark on Algorithm MC-REM, item (ii), allows other distance
 *   functions): dist is then the distance to the nearest triangle, and a start point outside the
 *   surface (by its winding number) is an escape.  The stop point is projected onto dD and the element
 *   that contains the projection receives one count (intrinsic Voronoi weights, Appendix
 *   Ex. A.3; for equally spaced arcs this equals the extrinsic Voronoi cells of Ex. A.2).  So
 *   counts[i, j] / N is the Monte Carlo estimate A_{omega, eps, N} of eq. "WoE_matrix_MC".
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed_lo, seed_hi),
 * counter = (block b, walk k, point i, instance).  The q-th FP64 uniform of a walk is the top 53
 * bits of words (2(q&1), 2(q&1)+1) of block q>>1, u = m * 2^-53 + 2^-54.  In 2D step s uses
 * uniform q = s (angle 2*pi*u); in 3D step s uses q = 2s (z = 1 - 2u) and q = 2s+1 (azimuth).
 *
 * Everything is FP64, compiled with -ffp-contract=off, no blocking or reordering beyond the
 * definition.  Rows (points) are split over threads; results do not depend on the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OG_DISK 0
#define OG_ANNULUS 1
#define OG_ELLIPSE 2
#define OG_POLYGON 3
#define OG_BALL 4
#define OG_BOX 5
#define OG_PERFORATED 6
#define OG_PERFBOX 7
#define OG_TRIMESH 8

#define OG_TWO_PI 6.283185307179586

typedef struct {
    int32_t dim;
    int32_t kind;
    double p[8];          /* shape parameters, see the geometry table in the docs */
    int32_t layout[4];    /* element layout */
    const double *verts;  /* polygon loop (x0,y0,x1,y1,...), counter-clockwise; for the perforated
                             domains the holes as (centre, r), dim + 1 numbers each; for a triangle
                             mesh the corners (a, b, c) of each triangle, 9 numbers each */
    int32_t n_verts;      /* polygon vertices, holes of a perforated domain, or mesh triangles */
    const double *nodes[2]; /* Bauer-spiral unit vectors (3 per node) of the outer sphere / of the holes
                               when their layout is (n, 0); set by the entry points, not the caller */
} og_geom;

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): ten rounds of two 32x32->64 multiplies and xors with a Weyl key.      */
/* ------------------------------------------------------------------------------------------ */
void oracle_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u in (0,1) from two 32-bit words: the top 53 bits of (hi:lo), centred in its 2^-53 cell. */
double oracle_u53(uint32_t hi, uint32_t lo)
{
    uint64_t m = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
    return (double)m * (1.0 / 9007199254740992.0) + (1.0 / 18014398509481984.0);
}

/* The q-th uniform of walk (k, i) of instance inst. */
static double walk_uniform(uint32_t q, uint32_t k, uint32_t i, uint32_t inst,
                           uint32_t key0, uint32_t key1)
{
    uint32_t ctr[4] = { q >> 1, k, i, inst };
    uint32_t key[2] = { key0, key1 };
    uint32_t w[4];
    oracle_philox(ctr, key, w);
    if ((q & 1u) == 0) return oracle_u53(w[0], w[1]);
    return oracle_u53(w[2], w[3]);
}

/* Uniform direction on S^{d-1} for step s (paper: U_n i.i.d. uniform on the unit sphere). */
void oracle_direction(int dim, uint32_t s, uint32_t k, uint32_t i, uint32_t inst,
                      uint32_t key0, uint32_t key1, double *U)
{
    if (dim == 2) {
        double th = OG_TWO_PI * walk_uniform(s, k, i, inst, key0, key1);
        U[0] = cos(th);
        U[1] = sin(th);
    } else {
        /* Archimedes: z uniform on [-1,1] and an independent uniform azimuth. */
        double z = 1.0 - 2.0 * walk_uniform(2u * s, k, i, inst, key0, key1);
        double ph = OG_TWO_PI * walk_uniform(2u * s + 1u, k, i, inst, key0, key1);
        double rho = sqrt((1.0 - z) * (1.0 + z));
        U[0] = rho * cos(ph);
        U[1] = rho * sin(ph);
        U[2] = z;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Geometry: signed Euclidean distance to dD (positive inside), projection -> element index.     */
/* ------------------------------------------------------------------------------------------ */
static double seg_dist(const double *a, const double *b, const double *x, double *t_out)
{
    double ex = b[0] - a[0], ey = b[1] - a[1];
    double wx = x[0] - a[0], wy = x[1] - a[1];
    double ll = ex * ex + ey * ey;
    double t = (wx * ex + wy * ey) / ll;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double dx = wx - t * ex, dy = wy - t * ey;
    *t_out = t;
    return sqrt(dx * dx + dy * dy);
}

/* Lower bound of the distance to the ellipse (x/a)^2 + (y/b)^2 = 1 from the gauge
 * f(x) = |diag(1/a,1/b) x|, which is Lipschitz with constant 1/min(a,b): dist >= min(a,b)(1-f). */
static double ellipse_lb(const og_geom *g, const double *x)
{
    double u = (x[0] - g->p[0]) / g->p[2], v = (x[1] - g->p[1]) / g->p[3];
    double f = sqrt(u * u + v * v);
    double m = g->p[2] < g->p[3] ? g->p[2] : g->p[3];
    return m * (1.0 - f);
}

/* Perforated domains: distance to the outer boundary (ball / disc, or box) and to hole l (the
 * vector from its centre in v when v is not NULL). */
static double outer_dist(const og_geom *g, const double *x)
{
    int d = g->dim;
    if (g->kind == OG_PERFORATED) {
        double s = 0.0;
        for (int a = 0; a < d; ++a) s += (x[a] - g->p[a]) * (x[a] - g->p[a]);
        return g->p[d] - sqrt(s);
    }
    double best = INFINITY;
    for (int a = 0; a < d; ++a) {
        double lo = x[a] - g->p[a], hi = g->p[d + a] - x[a];
        if (lo < best) best = lo;
        if (hi < best) best = hi;
    }
    return best;
}

static double hole_dist(const og_geom *g, int l, const double *x, double *v)
{
    int d = g->dim;
    const double *h = g->verts + (d + 1) * l;
    double s = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = x[a] - h[a];
        if (v) v[a] = t;
        s += t * t;
    }
    return sqrt(s) - h[d];
}

/* Triangle meshes: D is the interior of a closed surface made of triangles (a, b, c), each
 * counter-clockwise seen from outside.  Vectors are combined in axis order x, y, z. */
static double dot3(const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

static void cross3(const double *u, const double *v, double *w)
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

/* Distance from x to the segment p + t e, t in [0, 1], with w = x - p. */
static double seg3_dist(const double *w, const double *e)
{
    double t = dot3(w, e) / dot3(e, e);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = w[k] - t * e[k];
    return sqrt(dot3(q, q));
}

/* Distance from x to the triangle (a, b, c), from the definition of the distance to a convex set:
 * when the orthogonal projection of x onto the triangle's plane lies in the triangle (on the inner
 * side of each edge line within the plane), the projection is the nearest point and the distance is
 * |n.(x - a)| / |n| (n = (b - a) x (c - b)); otherwise the nearest point lies on the boundary, and
 * the distance is the smallest of the distances to the three edges. */
static double tri_dist(const double *T, const double *x)
{
    const double *a = T, *b = T + 3, *c = T + 6;
    double e0[3], e1[3], e2[3], ap[3], bp[3], cp[3], n[3], m[3];
    for (int k = 0; k < 3; ++k) {
        e0[k] = b[k] - a[k];
        e1[k] = c[k] - b[k];
        e2[k] = a[k] - c[k];
        ap[k] = x[k] - a[k];
        bp[k] = x[k] - b[k];
        cp[k] = x[k] - c[k];
    }
    cross3(e0, e1, n);
    /* n x e points into the triangle from edge e (within the plane) */
    cross3(n, e0, m);
    int inside = dot3(m, ap) >= 0.0;
    cross3(n, e1, m);
    inside = inside && dot3(m, bp) >= 0.0;
    cross3(n, e2, m);
    inside = inside && dot3(m, cp) >= 0.0;
    if (inside) return fabs(dot3(n, ap)) / sqrt(dot3(n, n));
    double d = seg3_dist(ap, e0), d1 = seg3_dist(bp, e1), d2 = seg3_dist(cp, e2);
    if (d1 < d) d = d1;
    if (d2 < d) d = d2;
    return d;
}

/* Distance to the mesh and the nearest triangle (the lowest index among equally near ones). */
static double mesh_dist(const og_geom *g, const double *x, int *tri_out)
{
    double best = INFINITY;
    int tb = 0;
    for (int t = 0; t < g->n_verts; ++t) {
        double d = tri_dist(g->verts + 9 * (size_t)t, x);
        if (d < best) { best = d; tb = t; }
    }
    if (tri_out) *tri_out = tb;
    return best;
}

/* Inside test of a start point: the winding number of the surface about x, the sum over the
 * triangles of the solid angle they subtend at x over 4 pi (Van Oosterom and Strackee: the solid
 * angle of (A, B, C) seen from the origin is 2 atan2(A.(B x C), |A||B||C| + (A.B)|C| + (A.C)|B| +
 * (B.C)|A|)), is 1 inside and 0 outside; x counts as inside when it exceeds 1/2. */
static int mesh_inside(const og_geom *g, const double *x)
{
    double total = 0.0;
    for (int t = 0; t < g->n_verts; ++t) {
        const double *T = g->verts + 9 * (size_t)t;
        double A[3], B[3], C[3], bc[3];
        for (int k = 0; k < 3; ++k) {
            A[k] = T[k] - x[k];
            B[k] = T[3 + k] - x[k];
            C[k] = T[6 + k] - x[k];
        }
        double la = sqrt(dot3(A, A)), lb = sqrt(dot3(B, B)), lc = sqrt(dot3(C, C));
        cross3(B, C, bc);
        double den = la * lb * lc + dot3(A, B) * lc + dot3(A, C) * lb + dot3(B, C) * la;
        total += 2.0 * atan2(dot3(A, bc), den);
    }
    return total > 0.5 * 2.0 * OG_TWO_PI;
}

/* Signed distance of a start point: for a mesh the distance carries the sign of the inside test
 * (the walk never leaves D afterwards, each step staying within the distance, so the distance
 * along the chain is the unsigned one); for the other kinds the signed distance itself. */
double oracle_dist(const og_geom *g, const double *x);
static double start_dist(const og_geom *g, const double *x)
{
    if (g->kind != OG_TRIMESH) return oracle_dist(g, x);
    double d = mesh_dist(g, x, NULL);
    return mesh_inside(g, x) ? d : -d;
}

double oracle_dist(const og_geom *g, const double *x)
{
    switch (g->kind) {
    case OG_DISK: {
        double dx = x[0] - g->p[0], dy = x[1] - g->p[1];
        return g->p[2] - sqrt(dx * dx + dy * dy);
    }
    case OG_ANNULUS: {
        double dx = x[0] - g->p[0], dy = x[1] - g->p[1];
        double rho = sqrt(dx * dx + dy * dy);
        double d_out = g->p[3] - rho, d_in = rho - g->p[2];
        return d_out < d_in ? d_out : d_in;
    }
    case OG_ELLIPSE:
        return ellipse_lb(g, x);
    case OG_POLYGON: {
        /* |distance| to the nearest edge, negative outside: D is the polygon's interior, whose
         * points have an odd crossing number (horizontal ray towards +x, an edge counted when its
         * end points lie strictly on either side of the ray's line, or one on it and one above) */
        double best = INFINITY, t;
        int inside = 0;
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e;
            const double *b = g->verts + 2 * ((e + 1) % g->n_verts);
            double d = seg_dist(a, b, x, &t);
            if (d < best) best = d;
            if ((a[1] > x[1]) != (b[1] > x[1])) {
                double ex = b[0] - a[0], ey = b[1] - a[1];
                double side = (x[1] - a[1]) * ex - (x[0] - a[0]) * ey; /* > 0: x left of the edge (ey > 0) */
                if (ey > 0.0 ? side > 0.0 : side < 0.0) inside ^= 1;
            }
        }
        return inside ? best : -best;
    }
    case OG_BALL: {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += (x[a] - g->p[a]) * (x[a] - g->p[a]);
        return g->p[3] - sqrt(s);
    }
    case OG_BOX: {
        int d = g->dim;
        double best = INFINITY;
        for (int a = 0; a < d; ++a) {
            double lo = x[a] - g->p[a], hi = g->p[d + a] - x[a];
            if (lo < best) best = lo;
            if (hi < best) best = hi;
        }
        return best;
    }
    case OG_TRIMESH:
        return mesh_dist(g, x, NULL);
    case OG_PERFORATED:
    case OG_PERFBOX: {
        /* a disc / ball (the paper's Examples 2-4, 6, 7) or a box (Examples 1, 5) with disjoint
         * spherical holes |x - c_l| < r_l removed: the nearest of the outer boundary and the holes */
        double best = outer_dist(g, x);
        for (int l = 0; l < g->n_verts; ++l) {
            double d = hole_dist(g, l, x, NULL);
            if (d < best) best = d;
        }
        return best;
    }
    }
    return -INFINITY;
}

static int clampi(long v, int n)
{
    if (v < 0) return 0;
    if (v > n - 1) return n - 1;
    return (int)v;
}

/* Arc index of angle theta (in (-pi, pi]) among M equal arcs counted from angle 0. */
static int arc_index(double theta, int M)
{
    if (theta < 0.0) theta += OG_TWO_PI;
    return clampi((long)floor(theta * (double)M / OG_TWO_PI), M);
}

/* Equal-area cell of a direction v (any length > 0) on a sphere: band iz of the height z / |v|
 * from the top (nz bands), sector of the azimuth (nphi sectors from angle 0). */
static int sphere_cells(int nz, int nphi) { return nphi == 0 ? nz : nz * nphi; }

static int sphere_cell(const double *v, int nz, int nphi)
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double zc = v[2] / n;
    int iz = clampi((long)floor((1.0 - zc) * 0.5 * (double)nz), nz);
    return iz * nphi + arc_index(atan2(v[1], v[0]), nphi);
}

/* The n nodes of Bauer's spiral on the unit sphere as Section 5.3 gives them: polar angle
 * phi_k = arccos(1 - (2k - 1)/n), azimuth theta_k = sqrt(n pi) phi_k, k = 1..n (node k - 1 here). */
static double *bauer_nodes(int n)
{
    double *u = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int k = 1; k <= n; ++k) {
        double ph = acos(1.0 - (2.0 * k - 1.0) / n);
        double th = sqrt(n * 3.14159265358979323846) * ph;
        u[3 * (k - 1) + 0] = sin(ph) * cos(th);
        u[3 * (k - 1) + 1] = sin(ph) * sin(th);
        u[3 * (k - 1) + 2] = cos(ph);
    }
    return u;
}

/* Extrinsic Voronoi cell (Appendix Ex. A.2): the node R u_k nearest the point, v its position relative
 * to the sphere's centre; the lowest index wins ties (the disjoint cells V_i take the earlier index). */
static int bauer_cell(const double *v, double R, int n, const double *u)
{
    double best = INFINITY;
    int bk = 0;
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            double t = v[a] - R * u[3 * k + a];
            s += t * t;
        }
        if (s < best) { best = s; bk = k; }
    }
    return bk;
}

/* Cell of a sphere: layout (nz, nphi) gives nz x nphi equal-area (z band, azimuth) cells, (n, 0) the
 * extrinsic Voronoi cells of n Bauer nodes. */
static int sphere_cell_of(const double *v, int nz, int nphi, double R, const double *nodes)
{
    if (nphi == 0) return nodes ? bauer_cell(v, R, nz, nodes) : -1;
    return sphere_cell(v, nz, nphi);
}

/* Copies g and attaches the node tables its Bauer layouts need (free with detach_nodes). */
static og_geom attach_nodes(const og_geom *g)
{
    og_geom G = *g;
    G.nodes[0] = G.nodes[1] = NULL;
    if (g->dim == 3) {
        if (g->kind == OG_BALL && g->layout[1] == 0) G.nodes[0] = bauer_nodes(g->layout[0]);
        if (g->kind == OG_PERFORATED && g->layout[1] == 0) G.nodes[0] = bauer_nodes(g->layout[0]);
        if (g->kind == OG_PERFORATED && g->layout[3] == 0) G.nodes[1] = bauer_nodes(g->layout[2]);
        if (g->kind == OG_PERFBOX && g->layout[2] == 0) G.nodes[1] = bauer_nodes(g->layout[1]);
    }
    return G;
}

static void detach_nodes(og_geom *G)
{
    free((void *)G->nodes[0]);
    free((void *)G->nodes[1]);
}

/* Box: the nearest face (ties: the lowest face index), then the patch of the other coordinates. */
static int box_cell(const og_geom *g, const double *x)
{
    int d = g->dim, n = g->layout[0];
    double best = INFINITY;
    int fb = 0;
    for (int f = 0; f < 2 * d; ++f) {
        int a = f / 2;
        double df = (f % 2 == 0) ? x[a] - g->p[a] : g->p[d + a] - x[a];
        if (df < best) { best = df; fb = f; }
    }
    int a = fb / 2, idx = 0;
    for (int b = 0; b < d; ++b) {
        if (b == a) continue;
        double lo = g->p[b], hi = g->p[d + b];
        int ib = clampi((long)floor((x[b] - lo) / (hi - lo) * (double)n), n);
        idx = idx * n + ib;
    }
    int per_face = (d == 2) ? n : n * n;
    return fb * per_face + idx;
}

/* Element index of the projection pi(x) of x onto dD (intrinsic Voronoi cells; ties go to the
 * lowest index, matching the disjoint partition of the paper's Appendix). */
int oracle_element(const og_geom *g, const double *x)
{
    switch (g->kind) {
    case OG_DISK:
        return arc_index(atan2(x[1] - g->p[1], x[0] - g->p[0]), g->layout[0]);
    case OG_ANNULUS: {
        double dx = x[0] - g->p[0], dy = x[1] - g->p[1];
        double rho = sqrt(dx * dx + dy * dy);
        double th = atan2(dy, dx);
        if (g->p[3] - rho <= rho - g->p[2]) return arc_index(th, g->layout[0]);
        return g->layout[0] + arc_index(th, g->layout[1]);
    }
    case OG_ELLIPSE: {
        /* eccentric angle of the gauge projection x / f(x) */
        double u = (x[0] - g->p[0]) / g->p[2], v = (x[1] - g->p[1]) / g->p[3];
        return arc_index(atan2(v, u), g->layout[0]);
    }
    case OG_POLYGON: {
        double best = INFINITY, tb = 0.0, t, perim = 0.0, s_at = 0.0;
        int eb = 0;
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e;
            const double *b = g->verts + 2 * ((e + 1) % g->n_verts);
            double d = seg_dist(a, b, x, &t);
            if (d < best) { best = d; eb = e; tb = t; }
        }
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e;
            const double *b = g->verts + 2 * ((e + 1) % g->n_verts);
            double len = sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
            if (e == eb) s_at = perim + tb * len;
            perim += len;
        }
        int M = g->layout[0];
        return clampi((long)floor(s_at * (double)M / perim), M);
    }
    case OG_BALL: {
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = x[a] - g->p[a];
        return sphere_cell_of(v, g->layout[0], g->layout[1], g->p[3], g->nodes[0]);
    }
    case OG_BOX:
        return box_cell(g, x);
    case OG_TRIMESH: {
        /* the nearest triangle; layout[0] consecutive triangles form one element */
        int tb;
        mesh_dist(g, x, &tb);
        return tb / g->layout[0];
    }
    case OG_PERFORATED:
    case OG_PERFBOX: {
        /* the nearest piece of the boundary (ties: the outer boundary, then the lowest hole), then
         * the cell of the direction from the piece's centre (arcs from angle 0 in 2D, equal-area
         * (z band, azimuth) cells in 3D).  Outer cells come first, then each hole's in hole order. */
        int d = g->dim, comp = -1, c = 0, n_outer, hole_cells;
        double best = outer_dist(g, x), v[3] = { 0.0, 0.0, 0.0 }, vb[3] = { 0.0, 0.0, 0.0 };
        for (int l = 0; l < g->n_verts; ++l) {
            double dl = hole_dist(g, l, x, v);
            if (dl < best) { best = dl; comp = l; vb[0] = v[0]; vb[1] = v[1]; vb[2] = v[2]; }
        }
        double Rh = comp >= 0 ? g->verts[(size_t)(d + 1) * comp + d] : 0.0;
        if (g->kind == OG_PERFORATED) {
            n_outer = d == 2 ? g->layout[0] : sphere_cells(g->layout[0], g->layout[1]);
            hole_cells = d == 2 ? g->layout[1] : sphere_cells(g->layout[2], g->layout[3]);
            if (comp < 0) {
                double w[3] = { 0.0, 0.0, 0.0 };
                for (int a = 0; a < d; ++a) w[a] = x[a] - g->p[a];
                return d == 2 ? arc_index(atan2(w[1], w[0]), g->layout[0])
                              : sphere_cell_of(w, g->layout[0], g->layout[1], g->p[d], g->nodes[0]);
            }
            c = d == 2 ? arc_index(atan2(vb[1], vb[0]), g->layout[1])
                       : sphere_cell_of(vb, g->layout[2], g->layout[3], Rh, g->nodes[1]);
        } else {
            n_outer = d == 2 ? 4 * g->layout[0] : 6 * g->layout[0] * g->layout[0];
            hole_cells = d == 2 ? g->layout[1] : sphere_cells(g->layout[1], g->layout[2]);
            if (comp < 0) return box_cell(g, x);
            c = d == 2 ? arc_index(atan2(vb[1], vb[0]), g->layout[1])
                       : sphere_cell_of(vb, g->layout[1], g->layout[2], Rh, g->nodes[1]);
        }
        return n_outer + comp * hole_cells + c;
    }
    }
    return -1;
}

/* Radius of the largest ellipsoid x + r S B(0,1) certified inside the ball B(c, R), from
 * |v + r S u|^2 = |v|^2 + 2 r (S v).u + r^2 |S u|^2 <= |v|^2 + 2 r |S v| + r^2 for |u| <= 1
 * (S symmetric, |S| <= 1, v = x - c): the positive root of r^2 + 2 a r - (R^2 - |v|^2) = 0,
 * r = sqrt(a^2 + R^2 - |v|^2) - a with a = |S v|.  q = |v|^2 and a2 = a^2 are passed in. */
static double inside_ball_radius(double q, double a2, double R)
{
    return sqrt(a2 + (R * R - q)) - sqrt(a2);
}

/* Radius certified outside the ball B(c, R_in) (a hole), from |v + r S u|^2 >= |v|^2 - 2 r |S v|:
 * r = (|v|^2 - R_in^2) / (2 |S v|). */
static double outside_ball_radius(double q, double a2, double R_in)
{
    return (q - R_in * R_in) / (2.0 * sqrt(a2));
}

/* |v|^2 and |S v|^2 for v = x - c. */
static void centred_norms(int dim, const double *S, const double *x, const double *c, double *q, double *a2)
{
    double v[3] = { 0.0, 0.0, 0.0 };
    double qq = 0.0, aa = 0.0;
    for (int a = 0; a < dim; ++a) {
        v[a] = x[a] - c[a];
        qq += v[a] * v[a];
    }
    for (int r = 0; r < dim; ++r) {
        double w = 0.0;
        for (int a = 0; a < dim; ++a) w += S[r * 3 + a] * v[a];
        aa += w * w;
    }
    *q = qq;
    *a2 = aa;
}

/* Ellipse (semi-axes a, b about c) in its own coordinates w = A^{-1}(x - c), A = diag(a, b): the step
 * ellipsoid is w + r T u, T = A^{-1} S, and |w + r T u|^2 <= |w|^2 + 2 r |T^T w| + r^2 |T|^2 for
 * |u| <= 1, so it stays in the unit disc for r <= the positive root of |T|^2 r^2 + 2 t r - g = 0,
 * t = |T^T w| = |S A^{-1} w|, g = 1 - |w|^2, which is g / (sqrt(t^2 + |T|^2 g) + t).  |T|^2 is the
 * largest eigenvalue of T^T T = S A^{-2} S. */
static double ellipse_mapped_bound(const og_geom *g, const double *S, const double *x)
{
    double a = g->p[2], b = g->p[3];
    double w0 = (x[0] - g->p[0]) / a, w1 = (x[1] - g->p[1]) / b;
    double gg = 1.0 - (w0 * w0 + w1 * w1);
    double v0 = w0 / a, v1 = w1 / b;
    double t0 = S[0] * v0 + S[1] * v1, t1 = S[3] * v0 + S[4] * v1;
    double t = sqrt(t0 * t0 + t1 * t1);
    double m00 = (S[0] / a) * (S[0] / a) + (S[3] / b) * (S[3] / b);
    double m11 = (S[1] / a) * (S[1] / a) + (S[4] / b) * (S[4] / b);
    double m01 = (S[0] / a) * (S[1] / a) + (S[3] / b) * (S[4] / b);
    double h = 0.5 * (m00 - m11);
    double sig2 = 0.5 * (m00 + m11) + sqrt(h * h + m01 * m01);
    return gg / (sqrt(t * t + sig2 * gg) + t);
}

/* Eigen-decomposition of the symmetric d x d matrix S (row-major 3 x 3 storage) by cyclic Jacobi
 * rotations: S = Q diag(ev) Q^T, column k of Q (Q[i*3+k]) the k-th eigenvector. */
static void sym_eigen(int d, const double *S, double *Q, double *ev)
{
    double A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[i][j] = (i < d && j < d) ? S[i * 3 + j] : 0.0;
            Q[i * 3 + j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = i + 1; j < d; ++j) off += A[i][j] * A[i][j];
        if (off == 0.0) break;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                if (A[p][q] == 0.0) continue;
                /* the rotation that zeroes A[p][q]: tan of the angle from the quadratic t^2 + 2 theta t - 1 = 0 */
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < d; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq;
                    A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk;
                    A[q][k] = sn * apk + c * aqk;
                }
                A[p][q] = A[q][p] = 0.0;
                for (int k = 0; k < d; ++k) {
                    double qkp = Q[k * 3 + p], qkq = Q[k * 3 + q];
                    Q[k * 3 + p] = c * qkp - sn * qkq;
                    Q[k * 3 + q] = sn * qkp + c * qkq;
                }
            }
    }
    for (int k = 0; k < 3; ++k) ev[k] = k < d ? A[k][k] : 1.0;
}

/* Distance from y to the ellipsoid sum_i (z_i / e_i)^2 = 1 in R^d, y inside or outside.  The nearest
 * point z is where y - z is normal to the ellipsoid: z_i = y_i e_i^2 / (e_i^2 + t) for a Lagrange
 * parameter t with sum_i (y_i e_i / (e_i^2 + t))^2 = 1.  The left side minus one, G(t), is convex and
 * decreasing for t > -min e_i^2, so the root is the limit of Newton's iteration started where G >= 0.
 * If y has no component along the shortest axes and G(-min e_i^2), summed over the other axes, is
 * <= 0, the nearest point has t = -min e_i^2, and its components along the shortest axes complete the
 * ellipsoid equation. */
static double ellipsoid_distance(int d, const double *e, const double *y)
{
    double b[3], a[3], bmin = INFINITY;
    for (int i = 0; i < d; ++i) {
        b[i] = e[i] * e[i];
        a[i] = fabs(y[i]) * e[i];
        if (b[i] < bmin) bmin = b[i];
    }
    double amax_short = 0.0, g_edge = -1.0;
    for (int i = 0; i < d; ++i) {
        if (b[i] == bmin) {
            if (a[i] > amax_short) amax_short = a[i];
        } else {
            double q = a[i] / (b[i] - bmin);
            g_edge += q * q;
        }
    }
    double t;
    if (amax_short > 0.0) {
        t = amax_short - bmin; /* the largest shortest-axis term alone is >= 1 here */
    } else if (g_edge > 0.0) {
        t = -bmin;
    } else {
        double d2 = 0.0, used = 0.0;
        for (int i = 0; i < d; ++i) {
            if (b[i] == bmin) continue;
            double z = y[i] * b[i] / (b[i] - bmin);
            d2 += (y[i] - z) * (y[i] - z);
            used += z * z / b[i];
        }
        double rest = 1.0 - used;
        if (rest < 0.0) rest = 0.0;
        return sqrt(d2 + bmin * rest);
    }
    for (int it = 0; it < 64; ++it) {
        double g = -1.0, h = 0.0; /* G(t) and -G'(t) / 2 */
        for (int i = 0; i < d; ++i) {
            double q = a[i] / (b[i] + t);
            g += q * q;
            h += q * q / (b[i] + t);
        }
        if (!(g > 0.0)) break;
        double tn = t + g / (2.0 * h);
        if (!(tn > t)) break;
        t = tn;
    }
    double d2 = 0.0;
    for (int i = 0; i < d; ++i) {
        double z = y[i] * b[i] / (b[i] + t);
        d2 += (y[i] - z) * (y[i] - z);
    }
    return sqrt(d2);
}

/* The distance from S^{-1} x to the image S^{-1}(c + R S^{d-1}) of the circle / sphere of centre c
 * and radius R: in the eigenbasis of S (eigenvalues s_k) an ellipsoid with semi-axes R / s_k about
 * S^{-1} c, and the point (Q^T (x - c))_k / s_k. */
static double mapped_sphere_distance(int d, const double *Q, const double *ev, const double *x,
                                     const double *c, double R)
{
    double w[3], e[3];
    for (int k = 0; k < d; ++k) {
        double acc = 0.0;
        for (int i = 0; i < d; ++i) acc += Q[i * 3 + k] * (x[i] - c[i]);
        w[k] = acc / ev[k];
        e[k] = R / ev[k];
    }
    return ellipsoid_distance(d, e, w);
}

/* Step radius.  Any ellipsoid x + r S B(0,1) inside D is a valid step of the chain (the chain is the
 * trace of the diffusion on inscribed ellipsoids, Section 4.2); the exit law does not depend on the
 * choice.  mode 0: r = dist (the ellipsoid lies in the Euclidean ball of radius r because
 * |S| <= 1).  mode 1 (boxes, polygons, discs, annuli, balls, discs and balls with holes): the
 * largest r whose ellipsoid stays inside D, the distance of S^{-1} x to the mapped boundary -- for a
 * box min over faces of (face distance)/|S e_a|, for a polygon the distance to the mapped edges, for
 * circles and spheres the distance to the mapped ellipses / ellipsoids (the smallest over them).  mode 2 (disc, annulus, ball): the bounds above for the outer
 * circle or sphere and, for the annulus, the inner circle, where dist itself is also a valid bound
 * for the inner circle: r = min(r_out, max(r_in, d)), and for a disc, ball or box with holes the
 * smallest hole bound as r_in (the box's r_out its exact radius); for the ellipse
 * max(ellipse_mapped_bound, d). */
static double step_radius(const og_geom *g, int mode, const double *S, const double *x, double d)
{
    if (mode == 0) return d;
    int dim = g->dim;
    if (mode == 1 && (g->kind == OG_DISK || g->kind == OG_ANNULUS || g->kind == OG_BALL || g->kind == OG_PERFORATED)) {
        double Q[9], ev[3];
        sym_eigen(dim, S, Q, ev);
        const double *c = g->p;
        if (g->kind == OG_ANNULUS) {
            double ro = mapped_sphere_distance(2, Q, ev, x, c, g->p[3]);
            double ri = mapped_sphere_distance(2, Q, ev, x, c, g->p[2]);
            return ro < ri ? ro : ri;
        }
        double r = mapped_sphere_distance(dim, Q, ev, x, c, g->p[dim]);
        if (g->kind == OG_PERFORATED)
            for (int l = 0; l < g->n_verts; ++l) {
                const double *h = g->verts + (size_t)(dim + 1) * l;
                double rl = mapped_sphere_distance(dim, Q, ev, x, h, h[dim]);
                if (rl < r) r = rl;
            }
        return r;
    }
    if (mode == 1 && g->kind == OG_TRIMESH) {
        /* As for polygons: x + r S B(0,1) lies in D exactly when S^{-1} x + r B(0,1) lies in S^{-1} D,
         * whose boundary is made of the mapped triangles S^{-1} T (a linear map takes triangles to
         * triangles), so the largest r is the distance from S^{-1} x to the mapped surface.  S^{-1}
         * is the adjugate of S over its determinant. */
        double c[9], Si[9];
        c[0] = S[4] * S[8] - S[5] * S[7];
        c[1] = S[5] * S[6] - S[3] * S[8];
        c[2] = S[3] * S[7] - S[4] * S[6];
        c[3] = S[2] * S[7] - S[1] * S[8];
        c[4] = S[0] * S[8] - S[2] * S[6];
        c[5] = S[1] * S[6] - S[0] * S[7];
        c[6] = S[1] * S[5] - S[2] * S[4];
        c[7] = S[2] * S[3] - S[0] * S[5];
        c[8] = S[0] * S[4] - S[1] * S[3];
        double det = S[0] * c[0] + S[1] * c[1] + S[2] * c[2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Si[i * 3 + j] = c[j * 3 + i] / det;
        double y[3], best = INFINITY;
        for (int i = 0; i < 3; ++i) y[i] = Si[i * 3 + 0] * x[0] + Si[i * 3 + 1] * x[1] + Si[i * 3 + 2] * x[2];
        for (int t = 0; t < g->n_verts; ++t) {
            const double *T = g->verts + 9 * (size_t)t;
            double M[9];
            for (int v = 0; v < 3; ++v)
                for (int i = 0; i < 3; ++i)
                    M[3 * v + i] = Si[i * 3 + 0] * T[3 * v] + Si[i * 3 + 1] * T[3 * v + 1] + Si[i * 3 + 2] * T[3 * v + 2];
            double dd = tri_dist(M, y);
            if (dd < best) best = dd;
        }
        return best;
    }
    if (mode == 1 && g->kind == OG_POLYGON) {
        /* The ellipsoid is { z : |S^{-1}(z - x)| <= r }: it misses edge [a, b] exactly while r is
         * below the distance from S^{-1} x to the mapped edge [S^{-1} a, S^{-1} b], and, being
         * connected and centred in D, lies in D while it misses every edge.  The largest inscribed
         * radius is the smallest of these distances.  S^{-1} by the 2 x 2 inverse formula. */
        double det = S[0] * S[4] - S[1] * S[3];
        double Si[4] = { S[4] / det, -S[1] / det, -S[3] / det, S[0] / det };
        double y[2] = { Si[0] * x[0] + Si[1] * x[1], Si[2] * x[0] + Si[3] * x[1] };
        double best = INFINITY, t;
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e;
            const double *b = g->verts + 2 * ((e + 1) % g->n_verts);
            double ma[2] = { Si[0] * a[0] + Si[1] * a[1], Si[2] * a[0] + Si[3] * a[1] };
            double mb[2] = { Si[0] * b[0] + Si[1] * b[1], Si[2] * b[0] + Si[3] * b[1] };
            double dd = seg_dist(ma, mb, y, &t);
            if (dd < best) best = dd;
        }
        return best;
    }
    if (mode == 2) {
        double q, a2;
        centred_norms(dim, S, x, g->p, &q, &a2);
        if (g->kind == OG_ELLIPSE) {
            double r = ellipse_mapped_bound(g, S, x);
            return r > d ? r : d;  /* d (the Lipschitz bound) is valid too */
        }
        if (g->kind == OG_PERFORATED || g->kind == OG_PERFBOX) {
            /* the outer circle / sphere (or the box's exact radius, as mode 1), then every hole as the
             * annulus's inner circle */
            double r_out, r_in = INFINITY;
            if (g->kind == OG_PERFORATED) {
                r_out = inside_ball_radius(q, a2, g->p[dim]);
            } else {
                r_out = INFINITY;
                for (int a = 0; a < dim; ++a) {
                    double cn = 0.0;
                    for (int r = 0; r < dim; ++r) cn += S[r * 3 + a] * S[r * 3 + a];
                    cn = sqrt(cn);
                    double lo = (x[a] - g->p[a]) / cn, hi = (g->p[dim + a] - x[a]) / cn;
                    if (lo < r_out) r_out = lo;
                    if (hi < r_out) r_out = hi;
                }
            }
            for (int l = 0; l < g->n_verts; ++l) {
                const double *h = g->verts + (size_t)(dim + 1) * l;
                double ql, a2l;
                centred_norms(dim, S, x, h, &ql, &a2l);
                double rl = outside_ball_radius(ql, a2l, h[dim]);
                if (rl < r_in) r_in = rl;
            }
            if (r_in < d) r_in = d;
            return r_out < r_in ? r_out : r_in;
        }
        if (g->kind == OG_DISK) return inside_ball_radius(q, a2, g->p[2]);
        if (g->kind == OG_BALL) return inside_ball_radius(q, a2, g->p[3]);
        /* annulus: p = (centre, R_in, R_out) */
        double r_out = inside_ball_radius(q, a2, g->p[3]);
        double r_in = outside_ball_radius(q, a2, g->p[2]);
        if (r_in < d) r_in = d;
        return r_out < r_in ? r_out : r_in;
    }
    double best = INFINITY;
    for (int a = 0; a < dim; ++a) {
        double cn = 0.0;
        for (int r = 0; r < dim; ++r) cn += S[r * 3 + a] * S[r * 3 + a];
        cn = sqrt(cn);
        double lo = (x[a] - g->p[a]) / cn, hi = (g->p[dim + a] - x[a]) / cn;
        if (lo < best) best = lo;
        if (hi < best) best = hi;
    }
    return best;
}

static int radius_mode_valid(const og_geom *g, int mode)
{
    if (mode == 0) return 1;
    if (mode == 1)
        return g->kind == OG_BOX || g->kind == OG_POLYGON || g->kind == OG_TRIMESH || g->kind == OG_DISK || g->kind == OG_ANNULUS ||
               g->kind == OG_BALL || g->kind == OG_PERFORATED;
    if (mode == 2)
        return g->kind == OG_DISK || g->kind == OG_ANNULUS || g->kind == OG_BALL || g->kind == OG_ELLIPSE ||
               g->kind == OG_PERFORATED || g->kind == OG_PERFBOX;
    return 0;
}

/* Radius probe for tests: the step radius of mode `mode` at each of n points (NaN where the mode
 * does not apply to the domain). */
void oracle_step_radii(const og_geom *g, const double *S, int mode, const double *x, int32_t n, double *r_out)
{
    for (int32_t i = 0; i < n; ++i) {
        const double *p = x + (size_t)i * g->dim;
        r_out[i] = radius_mode_valid(g, mode) ? step_radius(g, mode, S, p, oracle_dist(g, p)) : NAN;
    }
}

typedef struct {
    const og_geom *g;
    const double *S;
    double eps;
    int radius_mode;
    uint32_t key0, key1, inst, max_steps;
    const double *x_obs;
    int32_t n_obs;
    uint64_t wb, we;
    uint32_t *counts;
    int32_t *trace;
    const uint32_t *point_ids;
    int n_elem;
    int tid, nthr;
    uint64_t stats[5]; /* walks, steps, max_steps_seen, cap_hits, escapes */
} og_job;

static void *run_rows(void *arg)
{
    og_job *J = (og_job *)arg;
    const og_geom *g = J->g;
    int dim = g->dim;
    for (int i = J->tid; i < J->n_obs; i += J->nthr) {
        for (uint64_t k = J->wb; k < J->we; ++k) {
            double x[3] = { 0.0, 0.0, 0.0 }, U[3], y[3];
            for (int a = 0; a < dim; ++a) x[a] = J->x_obs[(size_t)i * dim + a];
            uint32_t s = 0;
            int capped = 0;
            double d;
            for (;;) {
                d = s == 0 ? start_dist(g, x) : oracle_dist(g, x);
                if (d <= J->eps) break;
                if (s >= J->max_steps) { capped = 1; break; }
                double r = step_radius(g, J->radius_mode, J->S, x, d);
                uint32_t pid = J->point_ids ? J->point_ids[i] : (uint32_t)i;
                oracle_direction(dim, s, (uint32_t)k, pid, J->inst, J->key0, J->key1, U);
                for (int rr = 0; rr < dim; ++rr) {
                    double acc = 0.0;
                    for (int c = 0; c < dim; ++c) acc += J->S[rr * 3 + c] * U[c];
                    y[rr] = acc;
                }
                for (int a = 0; a < dim; ++a) x[a] = x[a] + r * y[a];
                s += 1;
            }
            int j = oracle_element(g, x);
            J->counts[(size_t)i * J->n_elem + j] += 1u;
            J->stats[0] += 1;
            J->stats[1] += s;
            if (s > J->stats[2]) J->stats[2] = s;
            J->stats[3] += (uint64_t)capped;
            J->stats[4] += (uint64_t)(d < 0.0);
            if (J->trace) {
                size_t t = ((size_t)i * (size_t)(J->we - J->wb) + (size_t)(k - J->wb)) * 2;
                J->trace[t] = j;
                J->trace[t + 1] = (int32_t)s;
            }
        }
    }
    return NULL;
}

/*
 * Accumulates counts[i * n_elem + j] (row-major, caller-zeroed) for walks k in [walk_begin,
 * walk_end) of every point.  S is the 3x3 row-major symmetric root of K/lambda_max (only the
 * leading dim x dim block is read).  stats_out[5] = walks, steps, max steps, cap hits, escapes.
 * trace (optional) receives (element, steps) per walk, row-major over (point, walk - walk_begin).
 * point_ids (optional) gives the point index used in the random-number counter of each row (default:
 * the row index), so single rows of a large problem can be recomputed on their own.
 * Returns 0 on success, -1 on invalid arguments.
 */
int oracle_build_measure(const og_geom *g, int32_t n_elem, const double *S, double eps,
                         int radius_mode, uint32_t seed_lo, uint32_t seed_hi, uint32_t inst,
                         uint32_t max_steps, const double *x_obs, int32_t n_obs,
                         uint64_t walk_begin, uint64_t walk_end, uint32_t *counts,
                         uint64_t *stats_out, int32_t *trace, const uint32_t *point_ids,
                         int n_threads)
{
    if (!g || !S || !counts || n_obs < 0 || walk_end < walk_begin || !(eps >= 0.0)) return -1;
    if (eps == 0.0 && max_steps == 0) return -1; /* the fixed-iteration loop needs its count */
    if (!radius_mode_valid(g, radius_mode)) return -1;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    og_geom G = attach_nodes(g);
    og_job *jobs = (og_job *)calloc((size_t)n_threads, sizeof(og_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; ++t) {
        og_job *J = &jobs[t];
        J->g = &G; J->S = S; J->eps = eps; J->radius_mode = radius_mode;
        J->key0 = seed_lo; J->key1 = seed_hi; J->inst = inst; J->max_steps = max_steps;
        J->x_obs = x_obs; J->n_obs = n_obs; J->wb = walk_begin; J->we = walk_end;
        J->counts = counts; J->trace = trace; J->point_ids = point_ids; J->n_elem = n_elem;
        J->tid = t; J->nthr = n_threads;
        pthread_create(&th[t], NULL, run_rows, J);
    }
    uint64_t st[5] = { 0, 0, 0, 0, 0 };
    for (int t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        st[0] += jobs[t].stats[0];
        st[1] += jobs[t].stats[1];
        if (jobs[t].stats[2] > st[2]) st[2] = jobs[t].stats[2];
        st[3] += jobs[t].stats[3];
        st[4] += jobs[t].stats[4];
    }
    if (stats_out) memcpy(stats_out, st, sizeof(st));
    free(jobs);
    free(th);
    detach_nodes(&G);
    return 0;
}

/* Geometry probe for tests: distance and element of each of n points. */
void oracle_geom_eval(const og_geom *g, const double *x, int32_t n, double *d_out, int32_t *e_out)
{
    og_geom G = attach_nodes(g);
    for (int32_t i = 0; i < n; ++i) {
        const double *p = x + (size_t)i * G.dim;
        if (d_out) d_out[i] = start_dist(&G, p);
        if (e_out) e_out[i] = oracle_element(&G, p);
    }
    detach_nodes(&G);
}

/* Direction probe for tests: U for steps s in [0, n) of walk (k, i, inst). */
void oracle_directions(int dim, uint32_t n, uint32_t k, uint32_t i, uint32_t inst,
                       uint32_t key0, uint32_t key1, double *U_out)
{
    for (uint32_t s = 0; s < n; ++s) oracle_direction(dim, s, k, i, inst, key0, key1, U_out + (size_t)s * dim);
}

/* Stop positions of walks k in [kb, ke) from point x0 (row index i of its instance): the chain of
 * the estimator without the binning, for tests of E[u(X_{N_eps})] = u(x0) on K-harmonic u. */
int oracle_walk_exits(const og_geom *g, const double *S, double eps, int radius_mode,
                      uint32_t seed_lo, uint32_t seed_hi, uint32_t inst, uint32_t max_steps,
                      const double *x0, uint32_t i, uint64_t kb, uint64_t ke, double *pos_out)
{
    if (!g || !S || !x0 || !pos_out || ke < kb || !(eps >= 0.0)) return -1;
    if (eps == 0.0 && max_steps == 0) return -1;
    if (!radius_mode_valid(g, radius_mode)) return -1;
    int dim = g->dim;
    for (uint64_t k = kb; k < ke; ++k) {
        double x[3] = { 0.0, 0.0, 0.0 }, U[3], y[3];
        for (int a = 0; a < dim; ++a) x[a] = x0[a];
        uint32_t s = 0;
        for (;;) {
            double d = s == 0 ? start_dist(g, x) : oracle_dist(g, x);
            if (d <= eps || s >= max_steps) break;
            double r = step_radius(g, radius_mode, S, x, d);
            oracle_direction(dim, s, (uint32_t)k, i, inst, seed_lo, seed_hi, U);
            for (int rr = 0; rr < dim; ++rr) {
                double acc = 0.0;
                for (int c = 0; c < dim; ++c) acc += S[rr * 3 + c] * U[c];
                y[rr] = acc;
            }
            for (int a = 0; a < dim; ++a) x[a] = x[a] + r * y[a];
            s += 1;
        }
        for (int a = 0; a < dim; ++a) pos_out[(size_t)(k - kb) * dim + a] = x[a];
    }
    return 0;
}
