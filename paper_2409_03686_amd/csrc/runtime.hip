// runtime.hip -- host side of libwos: the C ABI declared in include/wos.h.
//
// Responsibilities: argument validation (before any device work), instance set-up (lambda_max(K),
// Khat = K / lambda_max, S = Khat^{1/2} by a symmetric Jacobi eigensolver in FP64), cell measures,
// device descriptors of batched builds staged through a ring of pinned buffers, launch shapes
// (set or autotuned), SVD workspaces, reconstruction, and HIP-graph plans of the whole path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <array>
#include <vector>

#include "../../include/wos.h"
#include "wos_internal.h"
#include "wos_runtime.h"

using namespace wos;

// ---------------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

wos_status wos::set_error(wos_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

extern "C" const char *wos_last_error(void) { return g_last_error.c_str(); }

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            if (ctx) (ctx)->poisoned = true;                                                      \
            return set_error(WOS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
        }                                                                                         \
    } while (0)

// ---------------------------------------------------------------------------------------------
// Device memory accounting
// ---------------------------------------------------------------------------------------------
wos_status wos::ctx_malloc(wos_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    size_t used = ctx->hbm_used.load();
    if (ctx->hbm_budget && used + bytes > ctx->hbm_budget)
        return set_error(WOS_ENOMEM, "HBM budget exceeded (%zu + %zu > %zu bytes)", used, bytes, ctx->hbm_budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return set_error(WOS_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    ctx->hbm_used += bytes;
    return WOS_OK;
}

void wos::ctx_free(wos_ctx *ctx, void *p, size_t bytes)
{
    if (!p) return;
    if (bytes == 0) bytes = 256;
    (void)hipFree(p);
    ctx->hbm_used -= bytes;
}

// ---------------------------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------------
// Scratch of the allocation-free walk launch (wos_build_measure_noalloc): the instance descriptor
// with its staged geometry records, then the launch's work cursors.  One copy per GPU, held until
// the process ends; every call on a GPU shares it.  Host code uses the address that
// hipGetSymbolAddress returns for the current device (kept in the context), never the name.
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocDescBytes = 64 * 1024;               // descriptor and geometry records
constexpr size_t kNoAllocCursorWords = (size_t(1) << 18) + 2;  // point-mode cursors: 2^18 points
constexpr size_t kNoAllocBytes = kNoAllocDescBytes + 4 * kNoAllocCursorWords;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {
// One piece of a descriptor, passed by value (so a captured graph holds the bytes themselves).
struct StageChunk {
    uint64_t w[256];  // 2 KiB
    uint32_t off, nwords;
};
__global__ void stage_chunk_kernel(uint8_t *dst, StageChunk c)
{
    uint64_t *d = reinterpret_cast<uint64_t *>(dst + c.off);
    for (uint32_t i = threadIdx.x; i < c.nwords; i += blockDim.x) d[i] = c.w[i];
}
}  // namespace

extern "C" wos_status wos_create(wos_ctx **out, int device, size_t hbm_budget_bytes)
{
    if (!out) return set_error(WOS_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return set_error(WOS_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) return set_error(WOS_EINVAL, "device %d out of range [0, %d)", device, n);
    wos_ctx *ctx = new wos_ctx();
    ctx->device = device;
    ctx->hbm_budget = hbm_budget_bytes;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&ctx->props, device) != hipSuccess) {
        delete ctx;
        return set_error(WOS_EDEVICE, "cannot open HIP device %d", device);
    }
    ctx->n_cu = ctx->props.multiProcessorCount;
    // this device's copy of the allocation-free scratch (the device is current)
    void *sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) == hipSuccess) ctx->noalloc_scratch = static_cast<uint8_t *>(sp);
    else (void)hipGetLastError();
    for (auto &slot : ctx->ring) {
        if (hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) != hipSuccess) {
            delete ctx;
            return set_error(WOS_EDEVICE, "hipEventCreate failed");
        }
    }
    *out = ctx;
    return WOS_OK;
}

extern "C" wos_status wos_destroy(wos_ctx *ctx)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx is NULL");
    (void)hipSetDevice(ctx->device);
    live_server_stop(ctx);  // drains requests in flight
    for (auto &slot : ctx->ring) {
        if (slot.used) (void)hipEventSynchronize(slot.done);
        (void)hipEventDestroy(slot.done);
        if (slot.host) (void)hipHostFree(slot.host);
        ctx_free(ctx, slot.dev, slot.cap);
    }
    delete ctx;
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------------------------
// Cells of a sphere: layout (n_z, n_phi) gives n_z x n_phi equal-area (z band, azimuth) cells, (n, 0)
// the extrinsic Voronoi cells (Appendix Ex. A.2) of n nodes of Bauer's spiral (Section 5.3).
static long long sphere_cells(int nz, int nphi) { return nphi == 0 ? nz : static_cast<long long>(nz) * nphi; }
static bool sphere_layout_ok(int nz, int nphi) { return nphi == 0 ? nz >= 16 : (nz >= 1 && nphi >= 1); }

static long long elements_of(const wos_geometry *g)
{
    switch (g->kind) {
    case WOS_DISK: case WOS_ELLIPSE: case WOS_POLYGON: return g->layout[0];
    case WOS_ANNULUS: return g->layout[0] + g->layout[1];
    case WOS_BALL: return sphere_cells(g->layout[0], g->layout[1]);
    case WOS_BOX: return g->dim == 2 ? 4 * g->layout[0] : 6 * g->layout[0] * g->layout[0];
    case WOS_PERFORATED:
        if (g->dim == 2) return g->layout[0] + g->layout[1] * g->layout[2];
        return sphere_cells(g->layout[0], g->layout[1]) + g->n_verts * sphere_cells(g->layout[2], g->layout[3]);
    case WOS_PERFBOX:
        if (g->dim == 2) return 4 * g->layout[0] + g->n_verts * g->layout[1];
        return 6 * g->layout[0] * g->layout[0] + g->n_verts * sphere_cells(g->layout[1], g->layout[2]);
    case WOS_TRIMESH: return g->n_verts / g->layout[0];
    }
    return -1;
}

size_t wos::vertex_doubles(const wos_geometry *g)
{
    if (!g->verts || g->n_verts <= 0) return 0;
    const size_t n = static_cast<size_t>(g->n_verts);
    switch (g->kind) {
    case WOS_PERFORATED: case WOS_PERFBOX: return n * (g->dim + 1);
    case WOS_TRIMESH: return 9 * n;
    default: return 2 * n;
    }
}

// Unit vectors of the n nodes of Bauer's spiral as Section 5.3 gives them: polar angle
// phi_k = arccos(1 - (2k - 1)/n), azimuth theta_k = sqrt(n pi) phi_k, k = 1..n (node k - 1 here).
static void bauer_nodes(int n, std::vector<double> &u)
{
    u.resize(3 * static_cast<size_t>(n));
    for (int k = 1; k <= n; ++k) {
        const double ph = std::acos(1.0 - (2.0 * k - 1.0) / n);
        const double th = std::sqrt(n * 3.14159265358979323846) * ph;
        u[3 * (k - 1) + 0] = std::sin(ph) * std::cos(th);
        u[3 * (k - 1) + 1] = std::sin(ph) * std::sin(th);
        u[3 * (k - 1) + 2] = std::cos(ph);
    }
}

// Areas of the Voronoi cells of the Bauer nodes on the unit sphere.  The cell of node c is the set of
// points p with p.(c - u_j) >= 0 for all j; in the gnomonic chart p ~ c + a e1 + b e2 around c (great
// circles become lines) each condition is the half-plane (1 - c.u_j) - a e1.u_j - b e2.u_j >= 0, so the
// cell is a convex polygon clipped from a large square.  Only nodes with |z_j - z_c| within twice the
// cell's chordal radius can clip it (a farther node is farther from every point of the cell than c is);
// the window is widened until it covers that.  The area is the sum of the solid angles of the fan
// triangles (c, p_m, p_m+1), each 2 atan2(|a.(b x c)|, 1 + a.b + b.c + c.a) (Van Oosterom-Strackee).
static void bauer_cell_areas(int n, double *area)
{
    std::vector<double> u;
    bauer_nodes(n, u);
    auto dot = [](const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    auto cross = [](const double *a, const double *b, double *c) {
        c[0] = a[1] * b[2] - a[2] * b[1];
        c[1] = a[2] * b[0] - a[0] * b[2];
        c[2] = a[0] * b[1] - a[1] * b[0];
    };
    for (int i = 0; i < n; ++i) {
        const double *c = &u[3 * static_cast<size_t>(i)];
        const double h[3] = {std::fabs(c[2]) < 0.9 ? 0.0 : 1.0, 0.0, std::fabs(c[2]) < 0.9 ? 1.0 : 0.0};
        double e1[3], e2[3];
        cross(h, c, e1);
        const double l1 = std::sqrt(dot(e1, e1));
        for (double &v : e1) v /= l1;
        cross(c, e1, e2);
        double win = 8.0 / std::sqrt(static_cast<double>(n));
        std::vector<std::array<double, 2>> P;
        for (;;) {
            const double L = 8.0;
            P = {{-L, -L}, {L, -L}, {L, L}, {-L, L}};
            for (int j = 0; j < n && !P.empty(); ++j) {
                const double *w = &u[3 * static_cast<size_t>(j)];
                if (j == i || std::fabs(w[2] - c[2]) > win) continue;
                const double k0 = 1.0 - dot(c, w), ka = -dot(e1, w), kb = -dot(e2, w);
                std::vector<std::array<double, 2>> Q;
                for (size_t m = 0; m < P.size(); ++m) {
                    const auto &A = P[m], &B = P[(m + 1) % P.size()];
                    const double fa = k0 + ka * A[0] + kb * A[1], fb = k0 + ka * B[0] + kb * B[1];
                    if (fa >= 0) Q.push_back(A);
                    if ((fa >= 0) != (fb >= 0)) {
                        const double t = fa / (fa - fb);
                        Q.push_back({A[0] + t * (B[0] - A[0]), A[1] + t * (B[1] - A[1])});
                    }
                }
                P.swap(Q);
            }
            double rmax = 0.0;  // chordal radius of the cell around c
            for (const auto &q : P) {
                double pv[3];
                for (int a = 0; a < 3; ++a) pv[a] = c[a] + q[0] * e1[a] + q[1] * e2[a];
                const double ln = std::sqrt(dot(pv, pv));
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) d2 += (pv[a] / ln - c[a]) * (pv[a] / ln - c[a]);
                rmax = std::max(rmax, std::sqrt(d2));
            }
            if (2.0 * rmax <= win || win > 2.0) break;
            win = 2.0 * rmax + 1e-9;
        }
        double acc = 0.0;
        for (size_t m = 0; m < P.size(); ++m) {
            double p0[3], p1[3], x[3];
            const auto &A = P[m], &B = P[(m + 1) % P.size()];
            for (int a = 0; a < 3; ++a) {
                p0[a] = c[a] + A[0] * e1[a] + A[1] * e2[a];
                p1[a] = c[a] + B[0] * e1[a] + B[1] * e2[a];
            }
            const double n0 = std::sqrt(dot(p0, p0)), n1 = std::sqrt(dot(p1, p1));
            for (int a = 0; a < 3; ++a) {
                p0[a] /= n0;
                p1[a] /= n1;
            }
            cross(p0, p1, x);
            acc += 2.0 * std::atan2(std::fabs(dot(c, x)), 1.0 + dot(c, p0) + dot(p0, p1) + dot(p1, c));
        }
        area[i] = acc;
    }
}

// Measures of the cells of a sphere of radius R (see sphere_cells).
static void sphere_measures(int nz, int nphi, double R, double *sigma)
{
    if (nphi == 0) {
        bauer_cell_areas(nz, sigma);
        for (int j = 0; j < nz; ++j) sigma[j] *= R * R;
    } else {
        for (int j = 0; j < nz * nphi; ++j) sigma[j] = 4.0 * M_PI * R * R / (nz * nphi);
    }
}

// Holes of a perforated domain: k disjoint balls (centre, r), dim + 1 numbers each, strictly inside
// the outer disc / ball (outer = true) or box.
static wos_status validate_holes(const wos_geometry *g, int k)
{
    const int d = g->dim, st = d + 1;
    const double *p = g->params;
    if (k < 1 || k > WOS_MAX_HOLES) return set_error(WOS_EINVAL, "a perforated domain needs 1..%d holes", WOS_MAX_HOLES);
    if (!g->verts || g->n_verts != k)
        return set_error(WOS_EINVAL, "a perforated domain needs verts = %d (centre, r) records of %d numbers", k, st);
    auto dist = [d](const double *a, const double *b) {
        double s = 0.0;
        for (int c = 0; c < d; ++c) s += (a[c] - b[c]) * (a[c] - b[c]);
        return std::sqrt(s);
    };
    for (int l = 0; l < k; ++l) {
        const double *h = g->verts + st * l;
        for (int c = 0; c <= d; ++c)
            if (!std::isfinite(h[c])) return set_error(WOS_EINVAL, "hole %d is not finite", l);
        if (!(h[d] > 0)) return set_error(WOS_EINVAL, "hole %d needs r > 0", l);
        bool inside = true;
        if (g->kind == WOS_PERFORATED) {
            inside = dist(h, p) + h[d] < p[d];
        } else {
            for (int c = 0; c < d; ++c) inside = inside && h[c] - h[d] > p[c] && h[c] + h[d] < p[d + c];
        }
        if (!inside) return set_error(WOS_EINVAL, "hole %d is not strictly inside the outer boundary", l);
        for (int m = 0; m < l; ++m) {
            const double *o = g->verts + st * m;
            if (!(dist(h, o) > h[d] + o[d])) return set_error(WOS_EINVAL, "holes %d and %d overlap", m, l);
        }
    }
    return WOS_OK;
}

wos_status wos::validate_geometry(const wos_geometry *g, int *n_elem)
{
    if (!g) return set_error(WOS_EINVAL, "geometry is NULL");
    for (double v : g->params)
        if (!std::isfinite(v)) return set_error(WOS_EINVAL, "geometry parameters must be finite");
    const double *p = g->params;
    switch (g->kind) {
    case WOS_DISK:
        if (g->dim != 2 || !(p[2] > 0)) return set_error(WOS_EINVAL, "disk needs dim 2 and R > 0");
        break;
    case WOS_ANNULUS:
        if (g->dim != 2 || !(p[2] > 0) || !(p[3] > p[2]))
            return set_error(WOS_EINVAL, "annulus needs dim 2 and 0 < R_in < R_out");
        if (g->layout[1] < 1) return set_error(WOS_EINVAL, "annulus needs layout (M_out >= 1, M_in >= 1)");
        break;
    case WOS_ELLIPSE:
        if (g->dim != 2 || !(p[2] > 0) || !(p[3] > 0)) return set_error(WOS_EINVAL, "ellipse needs dim 2, a, b > 0");
        break;
    case WOS_POLYGON: {
        if (g->dim != 2) return set_error(WOS_EINVAL, "polygon needs dim 2");
        if (!g->verts || g->n_verts < 3 || g->n_verts > WOS_MAX_POLY_VERTS)
            return set_error(WOS_EINVAL, "polygon needs 3..%d vertices", WOS_MAX_POLY_VERTS);
        double area2 = 0.0;
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e, *b = g->verts + 2 * ((e + 1) % g->n_verts);
            if (!std::isfinite(a[0]) || !std::isfinite(a[1])) return set_error(WOS_EINVAL, "polygon vertex not finite");
            if (a[0] == b[0] && a[1] == b[1]) return set_error(WOS_EINVAL, "polygon has a zero-length edge");
            area2 += a[0] * b[1] - a[1] * b[0];
        }
        if (!(area2 > 0)) return set_error(WOS_EINVAL, "polygon loop must be counter-clockwise");
        break;
    }
    case WOS_BALL:
        if (g->dim != 3 || !(p[3] > 0)) return set_error(WOS_EINVAL, "ball needs dim 3 and R > 0");
        if (!sphere_layout_ok(g->layout[0], g->layout[1]))
            return set_error(WOS_EINVAL, "ball needs layout (n_z >= 1, n_phi >= 1) or (n >= 16, 0)");
        break;
    case WOS_BOX:
        if (g->dim != 2 && g->dim != 3) return set_error(WOS_EINVAL, "box needs dim 2 or 3");
        for (int a = 0; a < g->dim; ++a)
            if (!(p[g->dim + a] > p[a])) return set_error(WOS_EINVAL, "box needs lo < hi on every axis");
        break;
    case WOS_PERFORATED: {
        if ((g->dim != 2 && g->dim != 3) || !(p[g->dim] > 0))
            return set_error(WOS_EINVAL, "perforated disc / ball needs dim 2 or 3 and R > 0");
        if (g->dim == 2 && (g->layout[1] < 1 || g->layout[2] < 1))
            return set_error(WOS_EINVAL, "perforated disc needs layout (M_out >= 1, M_hole >= 1, holes >= 1)");
        if (g->dim == 3 && (!sphere_layout_ok(g->layout[0], g->layout[1]) || !sphere_layout_ok(g->layout[2], g->layout[3])))
            return set_error(WOS_EINVAL, "perforated ball needs sphere layouts (n_z >= 1, n_phi >= 1) or (n >= 16, 0) "
                                         "for the ball and the holes");
        const wos_status st = validate_holes(g, g->dim == 2 ? g->layout[2] : g->n_verts);
        if (st != WOS_OK) return st;
        break;
    }
    case WOS_TRIMESH: {
        if (g->dim != 3) return set_error(WOS_EINVAL, "triangle mesh needs dim 3");
        if (!g->verts || g->n_verts < 4 || g->n_verts > WOS_MAX_TRIANGLES)
            return set_error(WOS_EINVAL, "triangle mesh needs 4..%d triangles", WOS_MAX_TRIANGLES);
        if (g->layout[0] < 1 || g->n_verts % g->layout[0] != 0)
            return set_error(WOS_EINVAL, "triangle mesh layout (g) needs g >= 1 dividing the triangle count");
        for (int t = 0; t < g->n_verts; ++t) {
            const double *T = g->verts + 9 * static_cast<size_t>(t);
            for (int k = 0; k < 9; ++k)
                if (!std::isfinite(T[k])) return set_error(WOS_EINVAL, "triangle %d has a coordinate that is not finite", t);
            double e1[3], e2[3], n[3], l1 = 0.0, l2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                e1[k] = T[3 + k] - T[k];
                e2[k] = T[6 + k] - T[k];
                l1 += e1[k] * e1[k];
                l2 += e2[k] * e2[k];
            }
            n[0] = e1[1] * e2[2] - e1[2] * e2[1];
            n[1] = e1[2] * e2[0] - e1[0] * e2[2];
            n[2] = e1[0] * e2[1] - e1[1] * e2[0];
            if (!(std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]) > 1e-9 * std::max(l1, l2)))
                return set_error(WOS_EINVAL, "triangle %d is degenerate", t);
        }
        break;
    }
    case WOS_PERFBOX: {
        if (g->dim != 2 && g->dim != 3) return set_error(WOS_EINVAL, "perforated box needs dim 2 or 3");
        for (int a = 0; a < g->dim; ++a)
            if (!(p[g->dim + a] > p[a])) return set_error(WOS_EINVAL, "perforated box needs lo < hi on every axis");
        if ((g->dim == 2 && g->layout[1] < 1) || (g->dim == 3 && !sphere_layout_ok(g->layout[1], g->layout[2])))
            return set_error(WOS_EINVAL, "perforated box needs layout (n, M_hole) or (n, n_z hole, n_phi hole) with "
                                         "the sphere layout (n_z >= 1, n_phi >= 1) or (n >= 16, 0)");
        const wos_status st = validate_holes(g, g->n_verts);
        if (st != WOS_OK) return st;
        break;
    }
    default:
        return set_error(WOS_EINVAL, "unknown geometry kind %d", g->kind);
    }
    if (g->layout[0] < 1) return set_error(WOS_EINVAL, "layout[0] must be >= 1");
    const long long m = elements_of(g);
    if (m < 1 || m > WOS_MAX_ELEMENTS)
        return set_error(WOS_ENOTSUP, "%lld cells (supported: 1..%d)", m, WOS_MAX_ELEMENTS);
    if (n_elem) *n_elem = static_cast<int>(m);
    return WOS_OK;
}

extern "C" wos_status wos_element_count(const wos_geometry *geom, int32_t *n_elem)
{
    if (!n_elem) return set_error(WOS_EINVAL, "n_elem is NULL");
    int m = 0;
    wos_status st = validate_geometry(geom, &m);
    if (st != WOS_OK) return st;
    *n_elem = m;
    return WOS_OK;
}

// Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n (for the ellipse arc lengths).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            const double z1 = z;
            z = z1 - p1 / pp;
            if (std::fabs(z - z1) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

extern "C" wos_status wos_element_measures(const wos_geometry *g, double *sigma)
{
    int M = 0;
    wos_status st = validate_geometry(g, &M);
    if (st != WOS_OK) return st;
    if (!sigma) return set_error(WOS_EINVAL, "sigma_host is NULL");
    const double *p = g->params;
    switch (g->kind) {
    case WOS_DISK:
        for (int j = 0; j < M; ++j) sigma[j] = 2.0 * M_PI * p[2] / M;
        break;
    case WOS_ANNULUS:
        for (int j = 0; j < g->layout[0]; ++j) sigma[j] = 2.0 * M_PI * p[3] / g->layout[0];
        for (int j = 0; j < g->layout[1]; ++j) sigma[g->layout[0] + j] = 2.0 * M_PI * p[2] / g->layout[1];
        break;
    case WOS_ELLIPSE: {
        std::vector<double> xg, wg;
        gauss_legendre(48, xg, wg);
        for (int j = 0; j < M; ++j) {
            const double t0 = 2.0 * M_PI * j / M, t1 = 2.0 * M_PI * (j + 1) / M;
            double acc = 0.0;
            for (size_t q = 0; q < xg.size(); ++q) {
                const double t = 0.5 * (t1 - t0) * xg[q] + 0.5 * (t1 + t0);
                acc += wg[q] * std::sqrt(p[2] * p[2] * std::sin(t) * std::sin(t) + p[3] * p[3] * std::cos(t) * std::cos(t));
            }
            sigma[j] = 0.5 * (t1 - t0) * acc;
        }
        break;
    }
    case WOS_POLYGON: {
        double L = 0.0;
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e, *b = g->verts + 2 * ((e + 1) % g->n_verts);
            L += std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
        }
        for (int j = 0; j < M; ++j) sigma[j] = L / M;
        break;
    }
    case WOS_BALL:
        sphere_measures(g->layout[0], g->layout[1], p[3], sigma);
        break;
    case WOS_TRIMESH:  // the areas |(b - a) x (c - a)| / 2 of each element's triangles
        for (int j = 0; j < M; ++j) sigma[j] = 0.0;
        for (int t = 0; t < g->n_verts; ++t) {
            const double *T = g->verts + 9 * static_cast<size_t>(t);
            double e1[3], e2[3];
            for (int k = 0; k < 3; ++k) {
                e1[k] = T[3 + k] - T[k];
                e2[k] = T[6 + k] - T[k];
            }
            const double n0 = e1[1] * e2[2] - e1[2] * e2[1], n1 = e1[2] * e2[0] - e1[0] * e2[2],
                         n2 = e1[0] * e2[1] - e1[1] * e2[0];
            sigma[t / g->layout[0]] += 0.5 * std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        }
        break;
    case WOS_PERFORATED: case WOS_PERFBOX: {
        // outer cells (arcs / equal-area sphere cells of the disc or ball, or box patches), then the
        // cells of each hole: 2 pi r / m arcs or 4 pi r^2 / (n_z n_phi) sphere cells
        const int d = g->dim;
        int n_out = 0, hc = 0;
        if (g->kind == WOS_PERFORATED) {
            n_out = d == 2 ? g->layout[0] : static_cast<int>(sphere_cells(g->layout[0], g->layout[1]));
            if (d == 2)
                for (int j = 0; j < n_out; ++j) sigma[j] = 2.0 * M_PI * p[d] / n_out;
            else
                sphere_measures(g->layout[0], g->layout[1], p[d], sigma);
            hc = d == 2 ? g->layout[1] : static_cast<int>(sphere_cells(g->layout[2], g->layout[3]));
        } else {
            const int n = g->layout[0], per_face = d == 2 ? n : n * n;
            for (int f = 0; f < 2 * d; ++f) {
                double area = 1.0;
                for (int b = 0; b < d; ++b)
                    if (b != f / 2) area *= (p[d + b] - p[b]) / n;
                for (int j = 0; j < per_face; ++j) sigma[f * per_face + j] = area;
            }
            n_out = 2 * d * per_face;
            hc = d == 2 ? g->layout[1] : static_cast<int>(sphere_cells(g->layout[1], g->layout[2]));
        }
        const int k = (M - n_out) / hc;
        for (int l = 0; l < k; ++l) {
            const double r = g->verts[(d + 1) * l + d];
            if (d == 2) {
                for (int j = 0; j < hc; ++j) sigma[n_out + l * hc + j] = 2.0 * M_PI * r / hc;
            } else {
                const int nz = g->kind == WOS_PERFORATED ? g->layout[2] : g->layout[1];
                const int nphi = g->kind == WOS_PERFORATED ? g->layout[3] : g->layout[2];
                sphere_measures(nz, nphi, r, sigma + n_out + l * hc);
            }
        }
        break;
    }
    case WOS_BOX: {
        const int d = g->dim, n = g->layout[0];
        const int per_face = d == 2 ? n : n * n;
        for (int f = 0; f < 2 * d; ++f) {
            double area = 1.0;
            for (int b = 0; b < d; ++b)
                if (b != f / 2) area *= (p[d + b] - p[b]) / n;
            for (int j = 0; j < per_face; ++j) sigma[f * per_face + j] = area;
        }
        break;
    }
    }
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Instance set-up: lambda_max(K) and S = (K / lambda_max)^{1/2} (cyclic Jacobi eigensolver).
// ---------------------------------------------------------------------------------------------
wos_status wos::conductivity_root(const double *K, int d, double S[9], double *lam_max, double *lam_min,
                                  double *evec, double *eval)
{
    double A[3][3] = {}, V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double scale = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const double v = K[i * 3 + j];
            if (!std::isfinite(v)) return set_error(WOS_EINVAL, "K has a non-finite entry");
            A[i][j] = v;
            scale = std::max(scale, std::fabs(v));
        }
    for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j)
            if (std::fabs(A[i][j] - A[j][i]) > 1e-12 * scale) return set_error(WOS_EINVAL, "K is not symmetric");
    if (!(scale > 0)) return set_error(WOS_EINVAL, "K is zero");
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = i + 1; j < d; ++j) off += A[i][j] * A[i][j];
        if (off == 0.0) break;
        for (int p = 0; p < d; ++p)
            for (int q = p + 1; q < d; ++q) {
                if (A[p][q] == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < d; ++k) {  // A <- A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < d; ++k) {  // A <- J^T A
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                A[p][q] = A[q][p] = 0.0;
                for (int k = 0; k < d; ++k) {  // V <- V J
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    double lmax = -1e300, lmin = 1e300;
    for (int i = 0; i < d; ++i) {
        lmax = std::max(lmax, A[i][i]);
        lmin = std::min(lmin, A[i][i]);
    }
    if (!(lmin > 0)) return set_error(WOS_EINVAL, "K is not positive definite (smallest eigenvalue %g)", lmin);
    for (int i = 0; i < 9; ++i) S[i] = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double acc = 0.0;
            for (int k = 0; k < d; ++k) acc += V[i][k] * std::sqrt(A[k][k] / lmax) * V[j][k];
            S[i * 3 + j] = acc;
        }
    if (lam_max) *lam_max = lmax;
    if (lam_min) *lam_min = lmin;
    if (evec)
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) evec[i * 3 + k] = i < d && k < d ? V[i][k] : (i == k ? 1.0 : 0.0);
    if (eval)
        for (int k = 0; k < 3; ++k) eval[k] = k < d ? std::sqrt(A[k][k] / lmax) : 1.0;
    return WOS_OK;
}

wos_status wos::validate_walk(const wos_geometry *g, const wos_walk_params *w)
{
    if (!w) return set_error(WOS_EINVAL, "walk params are NULL");
    if (!(w->eps >= 0) || !std::isfinite(w->eps)) return set_error(WOS_EINVAL, "eps must be finite and >= 0");
    if (w->eps == 0 && (w->precision != WOS_FP64 || w->max_steps == 0))
        return set_error(WOS_EINVAL, "eps = 0 (the fixed-iteration walk) needs WOS_FP64 and max_steps >= 1");
    if (w->walk_end < w->walk_begin) return set_error(WOS_EINVAL, "walk_end < walk_begin");
    if (w->walk_end > (1ull << 32)) return set_error(WOS_EINVAL, "walk ids must be below 2^32");
    if (w->walk_end - w->walk_begin >= (1ull << 32)) return set_error(WOS_EINVAL, "at most 2^32 - 1 walks per call");
    if (w->max_steps >= (1u << 31)) return set_error(WOS_EINVAL, "max_steps must be below 2^31");
    if (w->precision != WOS_FP64 && w->precision != WOS_FP32_GEOM_FP64_EXIT)
        return set_error(WOS_EINVAL, "unknown precision %d", w->precision);
    if (w->radius_mode != WOS_RADIUS_WOE_BOUND && w->radius_mode != WOS_RADIUS_MAPPED_EXACT &&
        w->radius_mode != WOS_RADIUS_MAPPED_BOUND)
        return set_error(WOS_EINVAL, "unknown radius mode %d", w->radius_mode);
    const bool curved = g->kind == WOS_DISK || g->kind == WOS_ANNULUS || g->kind == WOS_BALL ||
                        g->kind == WOS_PERFORATED;
    if (g->kind == WOS_TRIMESH && w->radius_mode == WOS_RADIUS_MAPPED_BOUND)
        return set_error(WOS_ENOTSUP, "triangle meshes take r = dist or the mapped-exact radius");
    if (w->radius_mode == WOS_RADIUS_MAPPED_EXACT && g->kind != WOS_BOX && g->kind != WOS_POLYGON &&
        g->kind != WOS_TRIMESH && !curved)
        return set_error(WOS_ENOTSUP, "mapped-exact radius is implemented for boxes, polygons, meshes, discs, annuli, "
                                      "balls and discs / balls with holes only");
    if (w->radius_mode == WOS_RADIUS_MAPPED_EXACT && curved && w->precision != WOS_FP64)
        return set_error(WOS_ENOTSUP, "the mapped-exact radius of circles and spheres (an iterative distance to "
                                      "an ellipse or ellipsoid) runs with FP64 geometry only");
    if (w->radius_mode == WOS_RADIUS_MAPPED_BOUND && g->kind != WOS_DISK && g->kind != WOS_ANNULUS &&
        g->kind != WOS_BALL && g->kind != WOS_ELLIPSE && g->kind != WOS_PERFORATED && g->kind != WOS_PERFBOX)
        return set_error(WOS_ENOTSUP, "mapped-bound radius is implemented for discs and balls (with or without holes), "
                                      "boxes with holes, annuli and ellipses only");
    return WOS_OK;
}

// Domain scale for the FP32 error bound: the largest coordinate magnitude the walk can reach.
static double domain_scale(const wos_geometry *g)
{
    const double *p = g->params;
    double s = 0.0;
    switch (g->kind) {
    case WOS_DISK: s = std::fabs(p[0]) + std::fabs(p[1]) + p[2]; break;
    case WOS_PERFORATED:
        for (int a = 0; a < g->dim; ++a) s += std::fabs(p[a]);
        s += p[g->dim];
        break;
    case WOS_ANNULUS: s = std::fabs(p[0]) + std::fabs(p[1]) + p[3]; break;
    case WOS_ELLIPSE: s = std::fabs(p[0]) + std::fabs(p[1]) + std::max(p[2], p[3]); break;
    case WOS_POLYGON:
        for (int e = 0; e < 2 * g->n_verts; ++e) s = std::max(s, std::fabs(g->verts[e]));
        break;
    case WOS_BALL: s = std::fabs(p[0]) + std::fabs(p[1]) + std::fabs(p[2]) + p[3]; break;
    case WOS_BOX: case WOS_PERFBOX:
        for (int a = 0; a < 2 * g->dim; ++a) s = std::max(s, std::fabs(p[a]));
        break;
    case WOS_TRIMESH:
        for (size_t e = 0; e < 9 * static_cast<size_t>(g->n_verts); ++e) s = std::max(s, std::fabs(g->verts[e]));
        break;
    }
    return std::max(s, 1e-30);
}

// Bounding-volume hierarchy of a triangle mesh and its device records, appended to segs (read from
// HBM, not staged in LDS): the nodes depth first (first child next, `skip` past the subtree), leaves of
// at most 4 triangles, inner nodes split by the surface-area heuristic; FP32 boxes rounded outward;
// then the FP32 and the FP64 triangle records in leaf order.
namespace {
struct BvhBuild {
    const double *v;
    std::vector<int> idx;
    std::vector<MeshNode> nodes;
    double tri_lo(int t, int k) const { return std::min({v[9 * t + k], v[9 * t + 3 + k], v[9 * t + 6 + k]}); }
    double tri_hi(int t, int k) const { return std::max({v[9 * t + k], v[9 * t + 3 + k], v[9 * t + 6 + k]}); }
    double cen(int t, int k) const { return (v[9 * t + k] + v[9 * t + 3 + k] + v[9 * t + 6 + k]) / 3.0; }
    // Split of idx[b, e) by the surface-area heuristic over 16 centroid bins per axis: the plane
    // between bins that minimises area(left box) x count(left) + area(right box) x count(right), the
    // expected cost of searching the two children; triangles are partitioned by bin (stable, so the
    // tree does not depend on anything but the input order).  Falls back to the median centroid
    // along the longest axis when the centroids do not spread.  Returns the first index on the right.
    int split(int b, int e, const double *clo, const double *chi)
    {
        constexpr int kBins = 16;
        double best = INFINITY;
        int bax = -1, bcut = 0;
        auto area = [](const double *lo, const double *hi) {
            const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
            return dx * dy + dy * dz + dz * dx;
        };
        auto bin_of = [&](int t, int ax) {
            const int bb = static_cast<int>(kBins * (cen(t, ax) - clo[ax]) / (chi[ax] - clo[ax]));
            return bb < 0 ? 0 : (bb >= kBins ? kBins - 1 : bb);
        };
        for (int ax = 0; ax < 3; ++ax) {
            if (!(chi[ax] > clo[ax])) continue;
            double blo[kBins][3], bhi[kBins][3];
            int cnt[kBins] = {};
            for (int q = 0; q < kBins; ++q)
                for (int k = 0; k < 3; ++k) {
                    blo[q][k] = INFINITY;
                    bhi[q][k] = -INFINITY;
                }
            for (int q = b; q < e; ++q) {
                const int t = idx[q], bb = bin_of(t, ax);
                ++cnt[bb];
                for (int k = 0; k < 3; ++k) {
                    blo[bb][k] = std::min(blo[bb][k], tri_lo(t, k));
                    bhi[bb][k] = std::max(bhi[bb][k], tri_hi(t, k));
                }
            }
            // right-hand boxes and counts for every cut, then a sweep from the left
            double rlo[kBins][3], rhi[kBins][3];
            int rc[kBins];
            for (int q = kBins - 1; q >= 0; --q) {
                rc[q] = cnt[q] + (q + 1 < kBins ? rc[q + 1] : 0);
                for (int k = 0; k < 3; ++k) {
                    rlo[q][k] = std::min(blo[q][k], q + 1 < kBins ? rlo[q + 1][k] : INFINITY);
                    rhi[q][k] = std::max(bhi[q][k], q + 1 < kBins ? rhi[q + 1][k] : -INFINITY);
                }
            }
            double llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
            int lc = 0;
            for (int cut = 1; cut < kBins; ++cut) {  // bins [0, cut) left, [cut, kBins) right
                lc += cnt[cut - 1];
                for (int k = 0; k < 3; ++k) {
                    llo[k] = std::min(llo[k], blo[cut - 1][k]);
                    lhi[k] = std::max(lhi[k], bhi[cut - 1][k]);
                }
                const int nr = rc[cut];
                if (lc == 0 || nr == 0) continue;
                const double cost = area(llo, lhi) * lc + area(rlo[cut], rhi[cut]) * nr;
                if (cost < best) {
                    best = cost;
                    bax = ax;
                    bcut = cut;
                }
            }
        }
        if (bax >= 0) {
            const auto it = std::stable_partition(idx.begin() + b, idx.begin() + e,
                                                  [&](int t) { return bin_of(t, bax) < bcut; });
            return static_cast<int>(it - idx.begin());
        }
        int ax = 0;
        for (int k = 1; k < 3; ++k)
            if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
        const int mid = (b + e) / 2;
        std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e,
                         [&](int s, int u) { return cen(s, ax) < cen(u, ax) || (cen(s, ax) == cen(u, ax) && s < u); });
        return mid;
    }
    void build(int b, int e)
    {
        const int me = static_cast<int>(nodes.size());
        nodes.push_back(MeshNode{});
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int q = b; q < e; ++q)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], tri_lo(idx[q], k));
                hi[k] = std::max(hi[k], tri_hi(idx[q], k));
                clo[k] = std::min(clo[k], cen(idx[q], k));
                chi[k] = std::max(chi[k], cen(idx[q], k));
            }
        MeshNode nd{};
        for (int k = 0; k < 3; ++k) {
            float fl = static_cast<float>(lo[k]), fh = static_cast<float>(hi[k]);
            if (static_cast<double>(fl) > lo[k]) fl = std::nextafter(fl, -INFINITY);
            if (static_cast<double>(fh) < hi[k]) fh = std::nextafter(fh, INFINITY);
            nd.lo[k] = fl;
            nd.hi[k] = fh;
        }
        if (e - b <= 4) {
            nd.leaf = (b << 3) | (e - b);
        } else {
            const int mid = split(b, e, clo, chi);
            nd.leaf = -1;
            build(b, mid);
            build(mid, e);
        }
        nd.skip = static_cast<int32_t>(nodes.size());
        nodes[me] = nd;
    }
};
}  // namespace

// verts: the triangles (9 numbers each); base: 0 for the surface, 4 for the mapped triangles.
static void mesh_records(const double *verts, int nt, int base, DevInst &I, std::vector<PolySeg> &segs)
{
    BvhBuild B{verts, std::vector<int>(nt), {}};
    for (int t = 0; t < nt; ++t) B.idx[t] = t;
    B.build(0, nt);
    const size_t nn = B.nodes.size();
    const size_t at = segs.size();
    int32_t *off = I.mesh_off + base;
    off[0] = static_cast<int32_t>(at);
    off[1] = static_cast<int32_t>(nn);
    off[2] = static_cast<int32_t>(at + (nn + 1) / 2);
    off[3] = static_cast<int32_t>(off[2] + 2 * static_cast<size_t>(nt));
    segs.resize(static_cast<size_t>(off[3]) + 2 * static_cast<size_t>(nt));
    std::memcpy(segs.data() + at, B.nodes.data(), nn * sizeof(MeshNode));
    MeshTri32 *t32 = reinterpret_cast<MeshTri32 *>(segs.data() + off[2]);
    MeshTri64 *t64 = reinterpret_cast<MeshTri64 *>(segs.data() + off[3]);
    for (int q = 0; q < nt; ++q) {
        const int t = B.idx[q];
        const double *a = verts + 9 * static_cast<size_t>(t), *b = a + 3, *c = a + 6;
        MeshTri64 &D = t64[q];
        std::memset(&D, 0, sizeof D);
        for (int k = 0; k < 3; ++k) {
            D.a[k] = a[k];
            D.b[k] = b[k];
            D.c[k] = c[k];
        }
        D.orig = t;
        double e[3][3], n[3];
        for (int k = 0; k < 3; ++k) {
            e[0][k] = b[k] - a[k];
            e[1][k] = c[k] - b[k];
            e[2][k] = a[k] - c[k];
        }
        n[0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
        n[1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
        n[2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
        const double nl = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) n[k] /= nl;
        auto f4 = [](double x, double y, double z, float w) {
            return float4{static_cast<float>(x), static_cast<float>(y), static_cast<float>(z), w};
        };
        MeshTri32 &F = t32[q];
        F.a = f4(a[0], a[1], a[2], 0.0f);
        float4 *E[3] = {&F.e0, &F.e1, &F.e2}, *Mv[3] = {&F.m0, &F.m1, &F.m2};
        for (int s = 0; s < 3; ++s) {
            const double ll = e[s][0] * e[s][0] + e[s][1] * e[s][1] + e[s][2] * e[s][2];
            *E[s] = f4(e[s][0], e[s][1], e[s][2], static_cast<float>(1.0 / ll));
            // n x e: the inward normal of edge s within the plane
            *Mv[s] = f4(n[1] * e[s][2] - n[2] * e[s][1], n[2] * e[s][0] - n[0] * e[s][2], n[0] * e[s][1] - n[1] * e[s][0], 0.0f);
        }
        int32_t ob = t;
        float ow;
        std::memcpy(&ow, &ob, 4);
        F.n = f4(n[0], n[1], n[2], ow);
    }
}

wos_status wos::fill_inst(const wos_geometry *g, const wos_walk_params *w, int n_elem, DevInst &I,
                          std::vector<PolySeg> &segs)
{
    std::memset(&I, 0, sizeof I);
    I.dim = g->dim;
    I.kind = g->kind;
    I.radius_mode = w->radius_mode;
    I.n_elem = n_elem;
    for (int k = 0; k < 4; ++k) I.layout[k] = g->layout[k];
    I.precision = w->precision;
    for (int k = 0; k < 8; ++k) {
        I.p[k] = g->params[k];
        I.pf[k] = static_cast<float>(g->params[k]);
    }
    if (g->kind == WOS_ANNULUS) {
        const double m = 0.5 * (g->params[2] + g->params[3]), w = 0.5 * (g->params[3] - g->params[2]);
        I.pf[4] = static_cast<float>(m);
        I.pf[5] = static_cast<float>(w);
        // FP32 circle decision of the binning: inner below (m - w/4)^2, outer above (m + w/4)^2
        I.pf[6] = static_cast<float>((m - 0.25 * w) * (m - 0.25 * w));
        I.pf[7] = static_cast<float>((m + 0.25 * w) * (m + 0.25 * w));
    }
    if (g->kind == WOS_ELLIPSE) {
        I.pf[4] = static_cast<float>(1.0 / g->params[2]);
        I.pf[5] = static_cast<float>(1.0 / g->params[3]);
        I.pf[6] = static_cast<float>(std::min(g->params[2], g->params[3]));
    }
    double lmax = 0, lmin = 0;
    wos_status st = conductivity_root(w->K, g->dim, I.S, &lmax, &lmin, I.Sq, I.Se);
    if (st != WOS_OK) return st;
    for (int k = 0; k < 9; ++k) I.Sf[k] = static_cast<float>(I.S[k]);
    if (g->dim == 2) {  // S^{-1} by the 2 x 2 inverse formula
        const double det = I.S[0] * I.S[4] - I.S[1] * I.S[3];
        I.Si[0] = I.S[4] / det;
        I.Si[1] = -I.S[1] / det;
        I.Si[2] = -I.S[3] / det;
        I.Si[3] = I.S[0] / det;
        for (int k = 0; k < 4; ++k) I.Sif[k] = static_cast<float>(I.Si[k]);
    }
    for (int a = 0; a < 3; ++a) {
        double cn = 0.0;
        for (int r = 0; r < g->dim; ++r) cn += I.S[r * 3 + a] * I.S[r * 3 + a];
        I.cn[a] = std::sqrt(cn);
        I.icnf[a] = a < g->dim ? static_cast<float>(1.0 / I.cn[a]) : 0.0f;
    }
    I.eps = w->eps;
    // FP32 distance error bound delta = 16 (32 for the ellipse and polygon) units of 2^-24 times the
    // largest coordinate magnitude: differences, squares, one hardware square root (2 ulps) and one
    // subtraction cost at most about 5 such units for circles, spheres and boxes, about 8 for the
    // ellipse gauge and the segment distances of a polygon.
    // Triangle meshes: 64 units (a CPU replay of the FP32 triangle distance in the tests stays below 8).
    const int dexp = g->kind == WOS_TRIMESH ? -18 : (g->kind == WOS_ELLIPSE || g->kind == WOS_POLYGON) ? -19 : -20;
    const double delta = std::ldexp(domain_scale(g), dexp);
    I.delta = static_cast<float>(delta);
    I.neg2delta = -2.0f * I.delta;
    // Relative radius shrink c of the FP32 step.  Each hardware sine / cosine of a direction is
    // within 2^-20 (checked on every input they take by a GPU test), so the step S U' misses S U by
    // at most sqrt(dim) 2^-20 (|S| = 1).  With r = dist the ellipsoid lies in the ball of radius r and
    // c = 2^-16 covers that.  A mapped radius's ellipsoid may touch the boundary: shrinking it by c r
    // leaves a gap of c r sigma_min(S) around the shrunken one, so c >= sqrt(dim) 2^-20 / sigma_min;
    // twice that is used.
    double shrink = 0x1.0p-16;
    if (w->radius_mode != WOS_RADIUS_WOE_BOUND)
        shrink = std::max(shrink, 2.0 * std::sqrt(static_cast<double>(g->dim)) * 0x1.0p-20 / std::sqrt(lmin / lmax));
    I.rshrink = static_cast<float>(1.0 - shrink);
    if (g->dim == 2) {
        for (int a = 0; a < 2; ++a) {
            const double A = std::hypot(I.S[a * 3 + 0], I.S[a * 3 + 1]);
            const double phi = std::atan2(I.S[a * 3 + 1], I.S[a * 3 + 0]) / (2.0 * M_PI);  // revolutions
            I.fold_off[a] = static_cast<float>(0x1.0p-25 - phi);
            // FP32 rounding moves these by 2^-24 relative at most, well inside the shrink
            I.fold_rs[a] = static_cast<float>(A * (1.0 - shrink));
            I.fold_rn[a] = static_cast<float>(A * static_cast<double>(I.neg2delta));
        }
    }
    if (w->radius_mode == WOS_RADIUS_MAPPED_BOUND && g->kind == WOS_ELLIPSE) {
        // |T|^2, T = A^{-1} S: the largest eigenvalue of T^T T = S A^{-2} S (2 x 2)
        const double a = g->params[2], b = g->params[3];
        const double m00 = (I.S[0] / a) * (I.S[0] / a) + (I.S[3] / b) * (I.S[3] / b);
        const double m11 = (I.S[1] / a) * (I.S[1] / a) + (I.S[4] / b) * (I.S[4] / b);
        const double m01 = (I.S[0] / a) * (I.S[1] / a) + (I.S[3] / b) * (I.S[4] / b);
        const double h = 0.5 * (m00 - m11);
        I.msig2 = 0.5 * (m00 + m11) + std::sqrt(h * h + m01 * m01);
        // FP32 error bound of the radius: |w|^2 and g carry about 6 units of 2^-24, t, s, the
        // reciprocal and the product some 16 relative units of a radius at most 1/m, where
        // m = min(sigma_min(S) / max(a, b), |T|) bounds s + t from below; three times that
        const double m = std::min(std::sqrt(lmin / lmax) / std::max(a, b), std::sqrt(I.msig2));
        I.mbf[0] = static_cast<float>(I.msig2);
        I.mbf[1] = static_cast<float>(0x1.0p-24 * 64.0 / m);
    } else if (w->radius_mode == WOS_RADIUS_MAPPED_BOUND) {
        // FP32 mapped bound (centred positions, |v| <= R_out): R_out^2, R_in^2 and absolute error
        // bounds of the two radii, subtracted on the device so that they never exceed the exact ones.
        // With u = 2^-24 and s = sigma_min(S) = (lambda_min / lambda_max)^{1/2}: |S v| and |v|^2
        // carry about 6 u |v| and 3 u R_out^2; sqrt(a^2 + R^2 - |v|^2) >= s R_out turns the latter into
        // 1.5 u R_out / s; the inner bound divides by 2 a >= 2 s R_in.  Twice the estimates are used.
        const double u = 0x1.0p-24, sg = std::sqrt(lmin / lmax);
        const double Ro = g->kind == WOS_ANNULUS ? g->params[3] : g->params[g->dim];  // disc, ball, perforated
        I.mbf[0] = static_cast<float>(Ro * Ro);
        I.mbf[1] = static_cast<float>(u * Ro * (16.0 / sg + 16.0));
        if (g->kind == WOS_ANNULUS) {
            const double Ri = g->params[2];
            I.mbf[2] = static_cast<float>(Ri * Ri);
            I.mbf[3] = static_cast<float>(u * (4.0 * Ro * Ro / (sg * Ri) + Ro * (22.0 / sg + 20.0)));
        }
    }
    // thresholds rounded outward so that the certain-exit test stays certain after rounding
    float lo = static_cast<float>(w->eps - delta), hi = static_cast<float>(w->eps + delta);
    if (static_cast<double>(lo) > w->eps - delta) lo = std::nextafter(lo, -INFINITY);
    if (static_cast<double>(hi) < w->eps + delta) hi = std::nextafter(hi, INFINITY);
    I.eps_lo = lo;
    I.eps_hi = hi;
    if (w->precision == WOS_FP32_GEOM_FP64_EXIT && !(w->eps > 8.0 * delta))
        return set_error(WOS_ENOTSUP, "eps %g is too small for FP32 geometry at domain scale %g (needs eps > %g)",
                         w->eps, domain_scale(g), 8.0 * delta);
    I.key0 = static_cast<uint32_t>(w->seed & 0xFFFFFFFFu);
    I.key1 = static_cast<uint32_t>(w->seed >> 32);
    I.inst = w->instance;
    I.max_steps = w->max_steps ? w->max_steps : 10000u;
    I.walk_begin = w->walk_begin;
    I.n_walks = static_cast<uint32_t>(w->walk_end - w->walk_begin);
    segs.clear();
    if (g->kind == WOS_POLYGON) {
        I.n_verts = g->n_verts;
        double cum = 0.0;
        for (int e = 0; e < g->n_verts; ++e) {
            const double *a = g->verts + 2 * e, *b = g->verts + 2 * ((e + 1) % g->n_verts);
            PolySeg s{};
            s.ax = a[0];
            s.ay = a[1];
            s.ex = b[0] - a[0];
            s.ey = b[1] - a[1];
            s.ll = s.ex * s.ex + s.ey * s.ey;
            s.len = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]));
            s.cum = cum;
            cum += s.len;
            s.fax = static_cast<float>(s.ax);
            s.fay = static_cast<float>(s.ay);
            s.fex = static_cast<float>(s.ex);
            s.fey = static_cast<float>(s.ey);
            s.finv_ll = static_cast<float>(1.0 / s.ll);
            segs.push_back(s);
        }
        I.perim = cum;
        if (w->radius_mode == WOS_RADIUS_MAPPED_EXACT) {
            // the mapped edges S^{-1}[a, b] after the edges, for the mapped-exact radius
            for (int e = 0; e < g->n_verts; ++e) {
                const double *a = g->verts + 2 * e, *b = g->verts + 2 * ((e + 1) % g->n_verts);
                const double ma[2] = {I.Si[0] * a[0] + I.Si[1] * a[1], I.Si[2] * a[0] + I.Si[3] * a[1]};
                const double mb[2] = {I.Si[0] * b[0] + I.Si[1] * b[1], I.Si[2] * b[0] + I.Si[3] * b[1]};
                PolySeg s{};
                s.ax = ma[0];
                s.ay = ma[1];
                s.ex = mb[0] - ma[0];
                s.ey = mb[1] - ma[1];
                s.ll = s.ex * s.ex + s.ey * s.ey;
                s.fax = static_cast<float>(s.ax);
                s.fay = static_cast<float>(s.ay);
                s.fex = static_cast<float>(s.ex);
                s.fey = static_cast<float>(s.ey);
                s.finv_ll = static_cast<float>(1.0 / s.ll);
                segs.push_back(s);
            }
            // FP32 error bound of the mapped distance: the polygon distance's 32 units of 2^-24 at
            // the mapped scale (at most the domain scale / sigma_min(S)), doubled for the mapping of
            // x and the rounding of the mapped edges
            I.mbf[1] = static_cast<float>(std::ldexp(domain_scale(g), -18) / std::sqrt(lmin / lmax));
        }
    }
    if (g->kind == WOS_PERFORATED || g->kind == WOS_PERFBOX) {
        // holes as (centre (ax, ay, ey), radius ex) records; FP32 centres relative to the outer
        // centre for the disc / ball (like the FP32 walk positions of the centred kinds), absolute
        // for the box
        const int d = g->dim;
        I.n_verts = g->n_verts;
        const bool centred = g->kind == WOS_PERFORATED;
        for (int l = 0; l < I.n_verts; ++l) {
            const double *h = g->verts + (d + 1) * l;
            PolySeg s{};
            s.ax = h[0];
            s.ay = h[1];
            s.ey = d == 3 ? h[2] : 0.0;
            s.ex = h[d];
            s.fax = static_cast<float>(h[0] - (centred ? g->params[0] : 0.0));
            s.fay = static_cast<float>(h[1] - (centred ? g->params[1] : 0.0));
            s.fey = d == 3 ? static_cast<float>(h[2] - (centred ? g->params[2] : 0.0)) : 0.0f;
            s.fex = static_cast<float>(h[d]);
            if (w->radius_mode == WOS_RADIUS_MAPPED_BOUND) {
                // the hole's mapped bound in FP32: R_l^2 and its error bound, the annulus's inner-circle
                // bound with |v| <= Ro (v from the hole's centre): twice the outer radius, or for the
                // box (absolute positions) twice the larger of its diagonal and the coordinate scale
                double Ro = 2.0 * g->params[d];
                if (!centred) {
                    double diag = 0.0;
                    for (int a = 0; a < d; ++a) diag += (g->params[d + a] - g->params[a]) * (g->params[d + a] - g->params[a]);
                    Ro = 2.0 * std::max(std::sqrt(diag), domain_scale(g));
                }
                const double u = 0x1.0p-24, sg = std::sqrt(lmin / lmax), Rl = h[d];
                s.fpad0 = static_cast<float>(Rl * Rl);
                s.fpad1 = static_cast<float>(u * (4.0 * Ro * Ro / (sg * Rl) + Ro * (22.0 / sg + 20.0)));
            }
            segs.push_back(s);
        }
    }
    I.n_segs = static_cast<int32_t>(segs.size());
    if (g->kind == WOS_TRIMESH) {
        I.n_verts = g->n_verts;
        mesh_records(g->verts, g->n_verts, 0, I, segs);
        double scale = domain_scale(g);
        if (w->radius_mode == WOS_RADIUS_MAPPED_EXACT) {
            // S^{-1} (the adjugate over the determinant) and the mapped triangles S^{-1} T, searched for
            // the distance from S^{-1} x
            const double *S = I.S;
            double c[9];
            c[0] = S[4] * S[8] - S[5] * S[7];
            c[1] = S[5] * S[6] - S[3] * S[8];
            c[2] = S[3] * S[7] - S[4] * S[6];
            c[3] = S[2] * S[7] - S[1] * S[8];
            c[4] = S[0] * S[8] - S[2] * S[6];
            c[5] = S[1] * S[6] - S[0] * S[7];
            c[6] = S[1] * S[5] - S[2] * S[4];
            c[7] = S[2] * S[3] - S[0] * S[5];
            c[8] = S[0] * S[4] - S[1] * S[3];
            const double det = S[0] * c[0] + S[1] * c[1] + S[2] * c[2];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    I.Si3[i * 3 + j] = c[j * 3 + i] / det;
                    I.Sif3[i * 3 + j] = static_cast<float>(I.Si3[i * 3 + j]);
                }
            const size_t nv = 9 * static_cast<size_t>(g->n_verts);
            std::vector<double> mv(nv);
            double ms = 0.0;
            for (size_t v = 0; v < nv; v += 3)
                for (int i = 0; i < 3; ++i) {
                    mv[v + i] = I.Si3[i * 3 + 0] * g->verts[v] + I.Si3[i * 3 + 1] * g->verts[v + 1] +
                                I.Si3[i * 3 + 2] * g->verts[v + 2];
                    ms = std::max(ms, std::fabs(mv[v + i]));
                }
            mesh_records(mv.data(), g->n_verts, 4, I, segs);
            // FP32 error bound of the mapped distance: the mesh distance's bound (64 units of 2^-24) at
            // the mapped scale, doubled for the mapping of x and the rounding of the mapped records
            I.mbf[1] = static_cast<float>(std::ldexp(ms, -17));
            scale = std::max(scale, ms);
            // sigma_min(S), shrunk below its rounding so that sigma_min r stays below dist
            const double sg = std::sqrt(lmin / lmax);
            I.mesh_sig64 = sg * (1.0 - 0x1.0p-40);
            I.mesh_sig32 = static_cast<float>(sg * (1.0 - 0x1.0p-18));
        }
        // pruning margins: far above the rounding of a distance (FP64: some 100 units of 2^-53 of the
        // coordinate scale; FP32: the box gap's few units of 2^-24)
        I.mesh_m64 = std::ldexp(scale, -40);
        I.mesh_m32 = static_cast<float>(std::ldexp(scale, -20));
    }
    // Bauer node tables of the spheres with layout (n, 0), after the staged records (not staged)
    auto add_nodes = [&](int n, int slot) {
        std::vector<double> u;
        bauer_nodes(n, u);
        I.node_off[slot] = static_cast<int32_t>(segs.size());
        for (int k = 0; k < n; ++k) {
            PolySeg s{};
            s.ax = u[3 * k];
            s.ay = u[3 * k + 1];
            s.ey = u[3 * k + 2];
            segs.push_back(s);
        }
    };
    if (g->dim == 3) {
        if ((g->kind == WOS_BALL || g->kind == WOS_PERFORATED) && g->layout[1] == 0) add_nodes(g->layout[0], 0);
        if (g->kind == WOS_PERFORATED && g->layout[3] == 0) add_nodes(g->layout[2], 1);
        if (g->kind == WOS_PERFBOX && g->layout[2] == 0) add_nodes(g->layout[1], 1);
    }
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Launch shapes
// ---------------------------------------------------------------------------------------------
static int tune_key(int dim, int kind, int precision) { return (precision * 4 + dim) * 16 + (kind + 1); }

wos_tuning wos::get_tuning(wos_ctx *ctx, int dim, int kind, int precision)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tuning.find(tune_key(dim, kind, precision));
    if (it != ctx->tuning.end()) return it->second;
    it = ctx->tuning.find(tune_key(dim, -1, precision));
    if (it != ctx->tuning.end()) return it->second;
    return wos_tuning{256, 16, WOS_ITEMS_AUTO};
}

static bool valid_tuning(const wos_tuning *t)
{
    return t && (t->block == 64 || t->block == 128 || t->block == 256 || t->block == 512 || t->block == 1024) &&
           t->walks_per_lane >= 1 && t->walks_per_lane <= 4096 && t->items >= WOS_ITEMS_AUTO &&
           t->items <= WOS_ITEMS_POINT;
}



extern "C" wos_status wos_set_tuning(wos_ctx *ctx, int32_t dim, int32_t kind, int32_t precision, const wos_tuning *t)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx is NULL");
    if (!valid_tuning(t))
        return set_error(WOS_EINVAL, "block must be 64..1024 (power of two), walks_per_lane 1..4096, items a wos_item_mode");
    if ((dim != 2 && dim != 3) || precision < 0 || precision > 1 || kind < -1 || kind > WOS_TRIMESH)
        return set_error(WOS_EINVAL, "bad (dim, kind, precision)");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuning[tune_key(dim, kind, precision)] = *t;
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Batched measure build
// ---------------------------------------------------------------------------------------------
struct Group {
    int precision, dim;
    std::vector<int> jobs;
};

// Prepares the descriptors of one (precision, dim) group into host memory `buf` (DevInst array
// followed by the polygon segments) and returns the launch shape.
wos_status wos::prepare_group(wos_ctx *ctx, const wos_measure_job *jobs, const std::vector<int> &idx,
                              const wos_tuning *force, std::vector<uint8_t> &buf, GroupLaunch &gl)
{
    const int n = static_cast<int>(idx.size());
    std::vector<DevInst> insts(n);
    std::vector<std::vector<PolySeg>> segs(n);
    gl = GroupLaunch{};
    wos_tuning tn = force ? *force : get_tuning(ctx, jobs[idx[0]].geom.dim, jobs[idx[0]].geom.kind, jobs[idx[0]].walk.precision);
    int max_elem = 1, seg_max = 0;
    for (int q = 0; q < n; ++q) {
        const wos_measure_job &J = jobs[idx[q]];
        int M = 0;
        wos_status st = validate_geometry(&J.geom, &M);
        if (st != WOS_OK) return st;
        st = fill_inst(&J.geom, &J.walk, M, insts[q], segs[q]);
        if (st != WOS_OK) return st;
        max_elem = std::max(max_elem, M);
        seg_max = std::max(seg_max, static_cast<int>(insts[q].n_segs));  // the records staged in LDS
    }
    gl.hist_words = (max_elem + 3) & ~3;
    gl.seg_bytes = static_cast<int>(sizeof(PolySeg)) * seg_max;
    gl.precision = jobs[idx[0]].walk.precision;
    gl.dim = jobs[idx[0]].geom.dim;
    gl.block = tn.block;
    // automatic choice: point mode for FP64 walks (5 % faster on the annulus: the reservations cut
    // the drains, and an FP64 step costs enough to hide their bookkeeping), block mode for FP32
    // (there the bookkeeping costs about what the drains did)
    gl.mode = tn.items == WOS_ITEMS_WAVE ? 1 : tn.items == WOS_ITEMS_POINT ? 2 : tn.items == WOS_ITEMS_BLOCK ? 0
            : (gl.precision == WOS_FP64 ? 2 : 0);
    // point mode keeps each point's 32-bit walk cursor clear of wrapping (failed reservations add to
    // it too): at most 2^30 walks per point
    for (int q = 0; q < n && gl.mode == 2; ++q)
        if (jobs[idx[q]].walk.walk_end - jobs[idx[q]].walk.walk_begin > (1ull << 30)) gl.mode = 0;
    // wave mode holds two histogram rows per wave: with many cells it does not fit in LDS
    if (gl.mode == 1 && walk_lds_bytes(gl.precision, gl.dim, gl.block, gl.hist_words, gl.seg_bytes, 1) > 64 * 1024)
        gl.mode = 0;
    // a work item holds walks_per_lane walks per lane of its owner (a wave or a block); in point
    // mode a wave reserves walks_per_lane walks per lane at a time
    const uint32_t chunk = static_cast<uint32_t>(gl.mode != 0 ? 64 : tn.block) * static_cast<uint32_t>(tn.walks_per_lane);
    uint64_t items = 0;
    size_t seg_off = sizeof(DevInst) * n;
    for (int q = 0; q < n; ++q) {
        DevInst &I = insts[q];
        const wos_measure_job &J = jobs[idx[q]];
        // big items of 4 chunks first, then at least 3 chunks' worth of small items per point
        I.chunk = chunk;
        I.big_chunk = 4 * chunk;
        I.n_big = I.n_walks >= 3 * chunk + I.big_chunk ? (I.n_walks - 3 * chunk) / I.big_chunk : 0;
        const uint32_t rest = I.n_walks - I.n_big * I.big_chunk;
        I.n_chunks = (rest + chunk - 1) / chunk;
        I.n_obs = J.n_obs;
        I.item_begin = items;
        // point mode: the "items" are the points
        I.n_items = gl.mode == 2 ? static_cast<uint64_t>(J.n_obs) : static_cast<uint64_t>(J.n_obs) * (I.n_big + I.n_chunks);
        items += I.n_items;
        I.x_obs = J.x_obs_dev;
        I.counts = J.counts_dev;
        I.stats = reinterpret_cast<unsigned long long *>(J.stats_dev);
        I.trace = J.trace_dev;
        // segs pointer is patched with the device base address at upload time (offset stored)
        I.segs = reinterpret_cast<const PolySeg *>(static_cast<uintptr_t>(seg_off));
        seg_off += sizeof(PolySeg) * segs[q].size();
    }
    // every block or wave takes one item past the end before it stops: keep the 32-bit cursor clear of wrapping
    if (items >= (1ull << 32) - (1ull << 20)) return set_error(WOS_ENOTSUP, "more than 2^32 - 2^20 work items in one launch");
    buf.assign(seg_off, 0);
    std::memcpy(buf.data(), insts.data(), sizeof(DevInst) * n);
    size_t off = sizeof(DevInst) * n;
    for (int q = 0; q < n; ++q) {
        if (!segs[q].empty()) std::memcpy(buf.data() + off, segs[q].data(), sizeof(PolySeg) * segs[q].size());
        off += sizeof(PolySeg) * segs[q].size();
    }
    gl.n_inst = n;
    gl.items = items;
    gl.block = tn.block;
    // one kind (and radius variant) for the whole launch: compiled in; else read per instance
    auto kernel_kind = [&](int q) {
        const wos_measure_job &j = jobs[idx[q]];
        const bool mapped = j.walk.radius_mode == WOS_RADIUS_MAPPED_BOUND ||
                            (j.geom.kind == WOS_POLYGON && j.walk.radius_mode == WOS_RADIUS_MAPPED_EXACT);
        const bool curved_exact = j.walk.radius_mode == WOS_RADIUS_MAPPED_EXACT && j.geom.kind != WOS_BOX &&
                                  j.geom.kind != WOS_POLYGON;
        if (j.geom.kind == WOS_TRIMESH) return static_cast<int>(kTriMesh);  // reads its radius mode per instance
        if (curved_exact) return -1;  // no compiled variant: the kernel reads the radius mode per instance
        return j.geom.kind + (mapped ? kRadiusVariant : 0);
    };
    gl.kind_sel = kernel_kind(0);
    for (int q = 1; q < n && gl.kind_sel >= 0; ++q)
        if (kernel_kind(q) != gl.kind_sel) gl.kind_sel = -1;
    const size_t lds = walk_lds_bytes(gl.precision, gl.dim, gl.block, gl.hist_words, gl.seg_bytes, gl.mode);
    if (lds > 160 * 1024) return set_error(WOS_ENOTSUP, "LDS need %zu bytes exceeds 160 KiB", lds);
    int per_cu = 0;
    const void *fn = walk_kernel_ptr(gl.precision, gl.dim, gl.kind_sel, gl.mode);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, gl.block, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    gl.per_cu = per_cu;
    uint64_t grid = static_cast<uint64_t>(per_cu) * ctx->n_cu;
    if (gl.mode != 2) grid = std::min<uint64_t>(grid, std::max<uint64_t>(items, 1));  // points can be shared
    gl.grid = static_cast<int>(grid);
    return WOS_OK;
}

// Patches the segment offsets of a staged descriptor buffer to device addresses.
static void patch_segs(std::vector<uint8_t> &buf, int n_inst, uintptr_t dev_base)
{
    DevInst *I = reinterpret_cast<DevInst *>(buf.data());
    for (int q = 0; q < n_inst; ++q)
        I[q].segs = reinterpret_cast<const PolySeg *>(dev_base + reinterpret_cast<uintptr_t>(I[q].segs));
}

int wos::stream_cus(const wos_ctx *ctx, hipStream_t s)
{
    if (!s) return ctx->n_cu;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return ctx->n_cu;
    constexpr int kWords = 64;  // up to 2048 CUs
    uint32_t mask[kWords] = {};
    const int words = std::min(kWords, (ctx->n_cu + 31) / 32);
    if (hipExtStreamGetCUMask(s, static_cast<uint32_t>(words), mask) != hipSuccess) return ctx->n_cu;
    int c = 0;
    for (int w = 0; w < words; ++w) c += __builtin_popcount(w == words - 1 && ctx->n_cu % 32 ? mask[w] & ((1u << (ctx->n_cu % 32)) - 1u) : mask[w]);
    return c >= 1 ? c : ctx->n_cu;
}

extern "C" wos_status wos_streams_create(wos_ctx *ctx, int32_t spectral_cus, void **walk_stream, void **spectral_stream)
{
    if (!ctx || !walk_stream || !spectral_stream) return set_error(WOS_EINVAL, "NULL argument");
    if (spectral_cus < 1 || spectral_cus >= ctx->n_cu)
        return set_error(WOS_EINVAL, "spectral_cus must be in [1, %d]", ctx->n_cu - 1);
    *walk_stream = *spectral_stream = nullptr;
    const int words = (ctx->n_cu + 31) / 32;
    std::vector<uint32_t> mw(words, 0u), ms(words, 0u);
    for (int c = 0; c < ctx->n_cu; ++c) {
        std::vector<uint32_t> &m = c >= ctx->n_cu - spectral_cus ? ms : mw;
        m[c / 32] |= 1u << (c % 32);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t a = nullptr, b = nullptr;
    hipError_t e = hipExtStreamCreateWithCUMask(&a, static_cast<uint32_t>(words), mw.data());
    if (e == hipSuccess) e = hipExtStreamCreateWithCUMask(&b, static_cast<uint32_t>(words), ms.data());
    if (e != hipSuccess) {
        if (a) (void)hipStreamDestroy(a);
        return set_error(WOS_EDEVICE, "hipExtStreamCreateWithCUMask failed: %s", hipGetErrorString(e));
    }
    *walk_stream = a;
    *spectral_stream = b;
    return WOS_OK;
}

extern "C" wos_status wos_streams_destroy(wos_ctx *ctx, void *walk_stream, void *spectral_stream)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx NULL");
    (void)hipSetDevice(ctx->device);
    if (walk_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(walk_stream));
    if (spectral_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(spectral_stream));
    return WOS_OK;
}

wos_status wos::stage_and_launch(wos_ctx *ctx, std::vector<uint8_t> &buf, const GroupLaunch &gl, hipStream_t stream)
{
    // ring slot: waits only if the launch that used it last has not finished
    RingSlot &slot = ctx->ring[ctx->ring_next];
    ctx->ring_next = (ctx->ring_next + 1) % ctx->ring.size();
    if (slot.used) HIP_TRY(ctx, hipEventSynchronize(slot.done));
    const size_t need = ((buf.size() + 15) & ~size_t(15)) + 4 * walk_cursor_words(gl.mode, gl.items) + 64;
    if (slot.cap < need) {
        if (slot.host) (void)hipHostFree(slot.host);
        ctx_free(ctx, slot.dev, slot.cap);
        slot.host = nullptr;
        slot.dev = nullptr;
        slot.cap = 0;
        size_t cap = 4096;
        while (cap < need) cap *= 2;
        wos_status st = ctx_malloc(ctx, &slot.dev, cap);
        if (st != WOS_OK) return st;
        if (hipHostMalloc(&slot.host, cap, hipHostMallocDefault) != hipSuccess) {
            ctx_free(ctx, slot.dev, cap);
            slot.dev = nullptr;
            return set_error(WOS_ENOMEM, "hipHostMalloc(%zu) failed", cap);
        }
        slot.cap = cap;
    }
    uint8_t *dev = static_cast<uint8_t *>(slot.dev);
    patch_segs(buf, gl.n_inst, reinterpret_cast<uintptr_t>(dev));
    std::memcpy(slot.host, buf.data(), buf.size());
    uint32_t *cursor = reinterpret_cast<uint32_t *>(dev + ((buf.size() + 15) & ~size_t(15)));
    HIP_TRY(ctx, hipMemcpyAsync(dev, slot.host, buf.size(), hipMemcpyHostToDevice, stream));
    // a persistent grid for the CUs this stream may use (fewer on a CU-masked stream)
    uint64_t grid = static_cast<uint64_t>(gl.per_cu) * stream_cus(ctx, stream);
    if (gl.mode != 2) grid = std::min<uint64_t>(grid, std::max<uint64_t>(gl.items, 1));
    HIP_TRY(ctx, launch_walks(gl.precision, gl.dim, gl.kind_sel, gl.mode, reinterpret_cast<const DevInst *>(dev), gl.n_inst,
                              gl.items, cursor, gl.hist_words, gl.seg_bytes, gl.block, static_cast<int>(grid), stream));
    HIP_TRY(ctx, hipEventRecord(slot.done, stream));
    slot.used = true;
    return WOS_OK;
}

static wos_status check_job(const wos_measure_job *J)
{
    int M = 0;
    wos_status st = validate_geometry(&J->geom, &M);
    if (st != WOS_OK) return st;
    st = validate_walk(&J->geom, &J->walk);
    if (st != WOS_OK) return st;
    if (J->n_obs < 0) return set_error(WOS_EINVAL, "n_obs < 0");
    if (J->n_obs > 0 && J->walk.walk_end > J->walk.walk_begin) {
        if (!J->x_obs_dev) return set_error(WOS_EINVAL, "x_obs_dev is NULL");
        if (!J->counts_dev) return set_error(WOS_EINVAL, "counts_dev is NULL");
    }
    return WOS_OK;
}

wos_status wos::group_jobs(const wos_measure_job *jobs, int n, std::vector<std::vector<int>> &groups)
{
    groups.clear();
    std::map<int, std::vector<int>> by;
    for (int q = 0; q < n; ++q) {
        wos_status st = check_job(&jobs[q]);
        if (st != WOS_OK) return set_error(st, "job %d: %s", q, wos_last_error());
        if (jobs[q].n_obs == 0 || jobs[q].walk.walk_end == jobs[q].walk.walk_begin) continue;  // nothing to do
        // meshes launch on their own (their compiled kernel is not part of the mixed-kind ones)
        by[jobs[q].walk.precision * 4 + jobs[q].geom.dim + (jobs[q].geom.kind == WOS_TRIMESH ? 16 : 0)].push_back(q);
    }
    for (auto &kv : by) groups.push_back(kv.second);
    return WOS_OK;
}

wos_status wos::build_batch(wos_ctx *ctx, const wos_measure_job *jobs, int32_t n_jobs, hipStream_t stream,
                            const wos_tuning *force)
{
    std::vector<std::vector<int>> groups;
    wos_status st = group_jobs(jobs, n_jobs, groups);
    if (st != WOS_OK) return st;
    // validate every group before enqueuing anything
    std::vector<std::vector<uint8_t>> bufs(groups.size());
    std::vector<GroupLaunch> gls(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        st = prepare_group(ctx, jobs, groups[g], force, bufs[g], gls[g]);
        if (st != WOS_OK) return st;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (size_t g = 0; g < groups.size(); ++g) {
        st = stage_and_launch(ctx, bufs[g], gls[g], stream);
        if (st != WOS_OK) return st;
    }
    return WOS_OK;
}

extern "C" wos_status wos_build_measure_batch(wos_ctx *ctx, const wos_measure_job *jobs, int32_t n_jobs, void *stream)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx is NULL");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return set_error(WOS_EINVAL, "bad job list");
    std::lock_guard<std::recursive_mutex> lk(ctx->launch_mu);
    return build_batch(ctx, jobs, n_jobs, static_cast<hipStream_t>(stream), nullptr);
}

extern "C" wos_status wos_build_measure(wos_ctx *ctx, const wos_geometry *geom, const wos_walk_params *walk,
                                        const double *x_obs_dev, int32_t n_obs, uint32_t *counts_dev,
                                        uint64_t *stats_dev, int32_t *trace_dev, void *stream)
{
    if (!geom || !walk) return set_error(WOS_EINVAL, "geometry or walk params NULL");
    wos_measure_job J;
    J.geom = *geom;
    J.walk = *walk;
    J.x_obs_dev = x_obs_dev;
    J.n_obs = n_obs;
    J.counts_dev = counts_dev;
    J.stats_dev = stats_dev;
    J.trace_dev = trace_dev;
    return wos_build_measure_batch(ctx, &J, 1, stream);
}

extern "C" wos_status wos_build_measure_noalloc(wos_ctx *ctx, const wos_geometry *geom, const wos_walk_params *walk,
                                                const double *x_obs_dev, int32_t n_obs, uint32_t *counts_dev,
                                                uint64_t *stats_dev, int32_t *trace_dev, void *stream)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx is NULL");
    if (!geom || !walk) return set_error(WOS_EINVAL, "geometry or walk params NULL");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    if (!ctx->noalloc_scratch) return set_error(WOS_EDEVICE, "the allocation-free scratch has no device address");
    wos_measure_job J;
    J.geom = *geom;
    J.walk = *walk;
    J.x_obs_dev = x_obs_dev;
    J.n_obs = n_obs;
    J.counts_dev = counts_dev;
    J.stats_dev = stats_dev;
    J.trace_dev = trace_dev;
    std::lock_guard<std::recursive_mutex> lk(ctx->launch_mu);
    std::vector<std::vector<int>> groups;
    wos_status st = group_jobs(&J, 1, groups);
    if (st != WOS_OK || groups.empty()) return st;  // invalid, or nothing to do
    std::vector<uint8_t> buf;
    GroupLaunch gl;
    st = prepare_group(ctx, &J, groups[0], nullptr, buf, gl);
    if (st != WOS_OK) return st;
    const size_t desc = (buf.size() + 15) & ~size_t(15);
    const size_t words = walk_cursor_words(gl.mode, gl.items);
    if (desc > kNoAllocDescBytes)
        return set_error(WOS_EINVAL, "descriptor of %zu bytes exceeds the allocation-free scratch (%zu)", desc,
                         kNoAllocDescBytes);
    if (words > kNoAllocCursorWords)
        return set_error(WOS_EINVAL, "%zu work cursors exceed the allocation-free scratch (%zu)", words,
                         kNoAllocCursorWords);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    uint8_t *dev = ctx->noalloc_scratch;
    hipStream_t s = static_cast<hipStream_t>(stream);
    patch_segs(buf, gl.n_inst, reinterpret_cast<uintptr_t>(dev));
    buf.resize(desc, 0);
    for (size_t off = 0; off < desc; off += sizeof(StageChunk::w)) {
        StageChunk c{};
        const size_t n = std::min(sizeof(c.w), desc - off);
        std::memcpy(c.w, buf.data() + off, n);
        c.off = static_cast<uint32_t>(off);
        c.nwords = static_cast<uint32_t>(n / 8);
        stage_chunk_kernel<<<1, 256, 0, s>>>(dev, c);
    }
    HIP_TRY(ctx, hipGetLastError());
    uint64_t grid = static_cast<uint64_t>(gl.per_cu) * stream_cus(ctx, s);
    if (gl.mode != 2) grid = std::min<uint64_t>(grid, std::max<uint64_t>(gl.items, 1));
    HIP_TRY(ctx, launch_walks(gl.precision, gl.dim, gl.kind_sel, gl.mode, reinterpret_cast<const DevInst *>(dev), gl.n_inst,
                              gl.items, reinterpret_cast<uint32_t *>(dev + kNoAllocDescBytes), gl.hist_words,
                              gl.seg_bytes, gl.block, static_cast<int>(grid), s));
    return WOS_OK;
}

extern "C" wos_status wos_autotune(wos_ctx *ctx, const wos_measure_job *job, uint64_t sample_walks, wos_tuning *best,
                                   void *stream)
{
    if (!ctx || !job) return set_error(WOS_EINVAL, "ctx or job NULL");
    wos_status st = check_job(job);
    if (st != WOS_OK) return st;
    if (job->n_obs == 0) return set_error(WOS_EINVAL, "autotune needs points");
    std::lock_guard<std::recursive_mutex> lk(ctx->launch_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    wos_measure_job J = *job;
    const uint64_t avail = J.walk.walk_end - J.walk.walk_begin;
    J.walk.walk_end = J.walk.walk_begin + std::min<uint64_t>(avail, std::max<uint64_t>(sample_walks, 1));
    J.stats_dev = nullptr;
    J.trace_dev = nullptr;
    int M = 0;
    (void)validate_geometry(&J.geom, &M);
    const size_t cbytes = static_cast<size_t>(J.n_obs) * M * sizeof(uint32_t);
    void *scratch = nullptr;
    st = ctx_malloc(ctx, &scratch, cbytes);
    if (st != WOS_OK) return st;
    J.counts_dev = static_cast<uint32_t *>(scratch);  // timing runs never touch the caller's counts
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    const int blocks[] = {128, 256, 512, 1024};
    const int wpls[] = {4, 8, 16, 32, 64};
    const int modes[] = {WOS_ITEMS_BLOCK, WOS_ITEMS_WAVE, WOS_ITEMS_POINT};
    float best_ms = 1e30f;
    wos_tuning bt{256, 16, WOS_ITEMS_AUTO};
    for (int md : modes)
    for (int b : blocks)
        for (int w : wpls) {
            wos_tuning t{b, w, md};
            float ms_min = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                HIP_TRY(ctx, hipEventRecord(e0, s));
                st = build_batch(ctx, &J, 1, s, &t);
                if (st != WOS_OK) break;
                HIP_TRY(ctx, hipEventRecord(e1, s));
                HIP_TRY(ctx, hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
                ms_min = std::min(ms_min, ms);
            }
            if (st != WOS_OK) {  // e.g. LDS need too large for this block: skip the shape
                st = WOS_OK;
                continue;
            }
            if (ms_min < best_ms) {
                best_ms = ms_min;
                bt = t;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    ctx_free(ctx, scratch, cbytes);
    {
        std::lock_guard<std::mutex> lk2(ctx->mu);
        ctx->tuning[tune_key(job->geom.dim, job->geom.kind, job->walk.precision)] = bt;
    }
    if (best) *best = bt;
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Diagnostic: the hardware sine and cosine (in revolutions) that the FP32 directions use, on the
// inputs they take, x_i = fma(i, 2^-24, offset) in FP32.
// ---------------------------------------------------------------------------------------------
namespace {
__global__ void trig32_kernel(float offset, uint32_t n, float *__restrict__ c, float *__restrict__ s)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float x = __builtin_fmaf(static_cast<float>(i), 0x1.0p-24f, offset);
        c[i] = __builtin_amdgcn_cosf(x);
        s[i] = __builtin_amdgcn_sinf(x);
    }
}
}  // namespace

extern "C" wos_status wos_diag_trig32(float offset, uint32_t n, float *cos_dev, float *sin_dev, void *stream)
{
    if (n > (1u << 24)) return set_error(WOS_EINVAL, "n = %u exceeds 2^24", n);
    if (n == 0) return WOS_OK;
    if (!cos_dev || !sin_dev) return set_error(WOS_EINVAL, "output pointer NULL");
    const uint32_t grid = std::min<uint32_t>((n + 255) / 256, 4096u);
    trig32_kernel<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(offset, n, cos_dev, sin_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(WOS_EDEVICE, "trig32 launch failed: %s", hipGetErrorString(e));
    return WOS_OK;
}
