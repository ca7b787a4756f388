// wos_device.hpp -- device-side building blocks of the walk-on-ellipsoids kernels (gfx950).
//
// Philox4x32-10 counter-based generator, uniform-direction samplers, signed distance functions,
// step radii and the cell index of the projection onto the boundary.  All of it is written for
// 64-wide wavefronts: per-walk state lives in VGPRs, per-instance constants are wave-uniform and
// are read through scalar loads from the instance descriptor.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wos {

enum Kind : int32_t {
    kDisk = 0, kAnnulus = 1, kEllipse = 2, kPolygon = 3, kBall = 4, kBox = 5, kPerforated = 6, kPerfBox = 7,
    kTriMesh = 8
};

constexpr int kMaxPolyVerts = 64;
constexpr double kTwoPi = 6.283185307179586;  // nearest double to 2 pi

// One polygon edge a -> b in FP64 (exit tests and cell indices) and FP32 (bulk distance); for the
// perforated domains one hole: centre (ax, ay[, ey]), radius ex, and in FP32 the centre (fax, fay
// [, fey]) -- relative to the outer centre for the disc / ball, absolute for the box -- and the
// radius fex.
struct PolySeg {
    double ax, ay, ex, ey, ll, cum, len, pad;
    float fax, fay, fex, fey, finv_ll, fpad0, fpad1, fpad2;
};

// Device descriptor of one instance of a (batched) measure build.  Filled on the host.
struct alignas(16) DevInst {
    int32_t dim, kind, radius_mode, n_elem;
    int32_t layout[4];
    int32_t n_verts, precision;
    int32_t n_segs, pad0;  // PolySeg records to stage in LDS: n_verts, or 2 n_verts with the mapped edges
    int32_t node_off[2];   // record index in segs of the Bauer node table (unit vectors in ax, ay, ey) of
                           // the outer sphere / of the holes, for sphere layouts (n, 0); read from HBM
    int32_t mesh_off[8];   // triangle meshes (read from HBM): record index in segs of the BVH nodes, the
                           // node count, record index of the FP32 and of the FP64 triangle records; then the
                           // same for the mapped triangles S^{-1} T (mapped-exact radius)
    double mesh_m64;       // pruning margin of the FP64 nearest-triangle search (a distance)
    float mesh_m32;        // the same for the FP32 search
    float mesh_sig32;      // mapped-exact radius of meshes: sigma_min(S), rounded down (FP32 and FP64 use
    double mesh_sig64;     // sigma_min r <= dist <= r to skip the surface search away from the boundary)
    double p[8];
    double S[9];      // Khat^{1/2}, Khat = K / lambda_max(K), row-major 3x3
    double msig2;     // ellipse, mapped bound: |A^{-1} S|^2 (A = diag(a, b))
    double Si[4];     // 2D: S^{-1}, row-major 2x2 (mapped-exact radius of polygons)
    double Si3[9];    // 3D: S^{-1}, row-major (mapped-exact radius of meshes)
    float Sif3[9];
    double Sq[9];     // eigenvectors of S, row-major: column k is the k-th (mapped-exact radius of
    double Se[3];     // circles and spheres), and the eigenvalues of S
    double cn[3];     // |S e_a|: the half-extent of the unit ellipsoid S B(0,1) along axis a
    double eps;
    double perim;     // polygon perimeter
    float pf[8];
    float Sf[9];
    float Sif[4];
    float icnf[3];    // 1 / |S e_a|
    float eps_lo;     // FP32 distance <= eps_lo: certainly inside the eps-shell
    float eps_hi;     // FP32 distance >  eps_hi: certainly outside it
    float delta;      // bound on |dist_fp32 - dist| for this domain (absolute)
    float neg2delta;  // -2 delta (radius shrink)
    float rshrink;    // 1 - c: the FP32 step's relative radius shrink (covers the direction's error)
    // 2D FP32 step with S folded into the direction: for U = (cos 2 pi u, sin 2 pi u),
    // (S U)_a = A_a cos 2 pi (u - phi_a), A_a the length of row a of S and phi_a its polar angle in
    // revolutions, so one cosine per coordinate replaces the cosine, the sine and the 2 x 2 product.
    float fold_off[2];  // 2^-25 - phi_a: the angle of coordinate a is (w >> 8) 2^-24 + fold_off[a]
    float fold_rs[2];   // A_a (1 - 2^-16)
    float fold_rn[2];   // A_a (-2 delta): step of coordinate a = (r fold_rs + fold_rn) cos(angle)
    float mbf[4];       // mapped-bound radius (FP32): R_out^2, its error bound, R_in^2, its error bound;
                        // ellipse: |A^{-1} S|^2, error bound; polygons: mbf[1] = error bound of the
                        // FP32 mapped distance
    uint32_t key0, key1, inst, max_steps;
    uint64_t walk_begin;  // first walk id of the range
    uint32_t n_walks;     // walks per point in this call
    // Work items of a point: n_big items of big_chunk walks (walk offsets [0, n_big big_chunk)), then
    // n_chunks items of chunk walks for the rest.  All big items (every point) come first in the
    // cursor order, so the last items handed out are small and the blocks finish together.
    uint32_t chunk;       // walks per small work item
    uint32_t n_chunks;    // small work items per point
    uint32_t big_chunk;   // walks per big work item
    uint32_t n_big;       // big work items per point
    int32_t n_obs;
    uint64_t item_begin;  // first global work item of this instance
    uint64_t n_items;
    const double *x_obs;
    uint32_t *counts;
    unsigned long long *stats;
    int32_t *trace;
    const PolySeg *segs;
};

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key schedule is wave-uniform, so the
// key additions run on the scalar unit; each round is two 32x32->64 products (one v_mad_u64_u32
// each, high and low halves together) and four xors.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = static_cast<uint32_t>(p1);
        c2 = n2;
        c3 = static_cast<uint32_t>(p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in (0,1]: the top 53 bits of hi:lo at the centre of their 2^-53 cell.
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo)
{
    const uint64_t m = ((static_cast<uint64_t>(hi) << 32) | lo) >> 11;
    return static_cast<double>(m) * 0x1.0p-53 + 0x1.0p-54;
}

// sin(2 pi u) and cos(2 pi u) for u in [0, 1], the direction of an FP64 step.  u splits exactly into
// a quarter turn q = rint(4u) and r = u - q/4 in [-1/8, 1/8]; x = 2 pi r lies in [-pi/4, pi/4],
// where the Taylor series of sin x through x^17 and of cos x through x^18 leave a truncation below
// 10^-19 (the next terms are x^19/19! and x^20/20!); the quarter turn then rotates (sin x, cos x).
// About 30 arithmetic instructions against some 75 for the general sincos, whose argument reduction
// serves any argument.  Within a few ulps of the correctly rounded values (host-side test).
__host__ __device__ inline void sincos2pi(double u, double *sp, double *cp)
{
#pragma clang fp contract(off)
    const double q = __builtin_rint(4.0 * u);
    const double r = __builtin_fma(q, -0.25, u);  // exact: u and q / 4 are multiples of 2^-54 here
    const double x = r * 6.283185307179586;       // 2 pi rounded to double
    const double x2 = x * x;
    double ps = 1.0 / 355687428096000.0;           // 1/17!
    ps = __builtin_fma(ps, x2, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, x2, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, x2, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, x2, 1.0 / 362880.0);
    ps = __builtin_fma(ps, x2, -1.0 / 5040.0);
    ps = __builtin_fma(ps, x2, 1.0 / 120.0);
    ps = __builtin_fma(ps, x2, -1.0 / 6.0);
    const double sn = __builtin_fma(x * x2, ps, x);
    double pc = 1.0 / 6402373705728000.0;          // 1/18!
    pc = __builtin_fma(pc, x2, -1.0 / 20922789888000.0);
    pc = __builtin_fma(pc, x2, 1.0 / 87178291200.0);
    pc = __builtin_fma(pc, x2, -1.0 / 479001600.0);
    pc = __builtin_fma(pc, x2, 1.0 / 3628800.0);
    pc = __builtin_fma(pc, x2, -1.0 / 40320.0);
    pc = __builtin_fma(pc, x2, 1.0 / 720.0);
    pc = __builtin_fma(pc, x2, -1.0 / 24.0);
    pc = __builtin_fma(pc, x2, 0.5);
    const double cs = __builtin_fma(-x2, pc, 1.0);
    // angle = q pi/2 + x
    const int k = static_cast<int>(q) & 3;
    const double s1 = (k & 1) ? cs : sn, c1 = (k & 1) ? sn : cs;
    *sp = (k & 2) ? -s1 : s1;
    *cp = ((k + 1) & 2) ? -c1 : c1;
}

// Uniform in (0,1]: the top 24 bits of w at the centre of their 2^-24 cell.
__device__ __forceinline__ float u24(uint32_t w)
{
    return static_cast<float>(w >> 8) * 0x1.0p-24f + 0x1.0p-25f;
}

// ------------------------------------------------------------------------------------------
// Scalar-type helpers
// ------------------------------------------------------------------------------------------
template <typename R> struct RT;
template <> struct RT<double> {
    static __device__ __forceinline__ double p(const DevInst &I, int k) { return I.p[k]; }
    static __device__ __forceinline__ double S(const DevInst &I, int k) { return I.S[k]; }
    static __device__ __forceinline__ double sqrt_(double v) { return __builtin_sqrt(v); }
};
template <> struct RT<float> {
    static __device__ __forceinline__ float p(const DevInst &I, int k) { return I.pf[k]; }
    static __device__ __forceinline__ float S(const DevInst &I, int k) { return I.Sf[k]; }
    static __device__ __forceinline__ float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
};

template <typename R> __device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }

// ------------------------------------------------------------------------------------------
// Triangle meshes.  The surface's triangles sit in a bounding-volume hierarchy stored depth first:
// a node's first child follows it, `skip` is the node after its subtree, so a search that drops a
// subtree jumps to `skip` and needs no stack.  Leaves hold up to 7 consecutive triangles (the host
// builds leaves of at most 4).  Boxes are
// FP32, rounded outward, so they contain their triangles exactly.
// ------------------------------------------------------------------------------------------
struct MeshNode {
    float lo[3];
    int32_t skip;
    float hi[3];
    int32_t leaf;  // (first triangle << 3) | count for a leaf, -1 for an inner node
};
// FP32 record: corner a, edges e0 = b - a, e1 = c - b, e2 = a - c (w: 1 / |e|^2), the unit normal n
// (w: the triangle's original index as bits), and the in-plane inward edge normals n x e_k.
struct MeshTri32 {
    float4 a, e0, e1, e2, n, m0, m1, m2;
};
// FP64 record: the corners as given (all derived quantities are computed from them per query).
struct MeshTri64 {
    double a[3], b[3], c[3];
    int32_t orig, pad0;
    double pad[6];
};
static_assert(sizeof(MeshNode) == 32 && sizeof(MeshTri32) == 128 && sizeof(MeshTri64) == 128, "mesh records");

__device__ __forceinline__ double dot3d(const double *u, const double *v)
{
#pragma clang fp contract(off)
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}
__device__ __forceinline__ void cross3d(const double *u, const double *v, double *w)
{
#pragma clang fp contract(off)
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}
// distance from x to the segment p + t e (t in [0, 1]), w = x - p
__device__ __forceinline__ double seg3_dist64(const double *w, const double *e)
{
#pragma clang fp contract(off)
    double t = dot3d(w, e) / dot3d(e, e);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    double q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) q[k] = w[k] - t * e[k];
    return __builtin_sqrt(dot3d(q, q));
}
// Distance from x to the triangle (a, b, c): the plane distance |n.(x - a)| / |n|, n = (b - a) x
// (c - b), when the projection of x onto the plane lies on the inner side of all three edge lines
// (within the plane the inner side of edge e is where n x e points); else the nearest of the
// three edges.
__device__ __forceinline__ double tri_dist64(const MeshTri64 &T, const double *x)
{
#pragma clang fp contract(off)
    double e0[3], e1[3], e2[3], ap[3], bp[3], cp[3], n[3], m[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e0[k] = T.b[k] - T.a[k];
        e1[k] = T.c[k] - T.b[k];
        e2[k] = T.a[k] - T.c[k];
        ap[k] = x[k] - T.a[k];
        bp[k] = x[k] - T.b[k];
        cp[k] = x[k] - T.c[k];
    }
    cross3d(e0, e1, n);
    cross3d(n, e0, m);
    bool inside = dot3d(m, ap) >= 0.0;
    cross3d(n, e1, m);
    inside = inside && dot3d(m, bp) >= 0.0;
    cross3d(n, e2, m);
    inside = inside && dot3d(m, cp) >= 0.0;
    if (inside) return __builtin_fabs(dot3d(n, ap)) / __builtin_sqrt(dot3d(n, n));
    double d = seg3_dist64(ap, e0);
    const double d1 = seg3_dist64(bp, e1), d2 = seg3_dist64(cp, e2);
    d = d1 < d ? d1 : d;
    return d2 < d ? d2 : d;
}

// The records live in global memory: pointers in the global address space let the compiler use
// global loads (a generic pointer becomes flat loads, which also wait on the LDS counter).
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using GPtr = const __attribute__((address_space(1))) T *;
#else  // the host pass parses these functions but never emits them
template <typename T> using GPtr = const T *;
#endif
template <typename T> __device__ __forceinline__ GPtr<T> mesh_rec(const DevInst &I, int slot)
{
    return (GPtr<T>)(I.segs + I.mesh_off[slot]);
}

// Squared distance from x to a node's box (0 inside it).
template <typename R> __device__ __forceinline__ R box_gap2(const MeshNode &nd, const R *x)
{
#pragma clang fp contract(off)
    R g2 = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R lo = static_cast<R>(nd.lo[k]) - x[k], hi = x[k] - static_cast<R>(nd.hi[k]);
        R gk = lo > hi ? lo : hi;
        gk = gk > R(0) ? gk : R(0);
        g2 += gk * gk;
    }
    return g2;
}

// The leaf reached by always stepping into the child whose box is nearer x (the first child on
// ties): its triangles give the search a first bound close to the final distance, so that the pass
// over the hierarchy drops most subtrees at their root.
__device__ __forceinline__ int mesh_greedy_leaf(GPtr<MeshNode> nodes, const float *xf)
{
    int i = 0;
    MeshNode nd = nodes[0];
    while (nd.leaf < 0) {
        const MeshNode l = nodes[i + 1], r = nodes[l.skip];
        const bool left = box_gap2<float>(l, xf) <= box_gap2<float>(r, xf);
        i = left ? i + 1 : l.skip;
        nd = left ? l : r;
    }
    return i;
}

// Result of a nearest-triangle search: the distance, the triangle's original index (FP64 only) and its
// position in the hierarchy's triangle order (the next search's hint).
struct MeshHit64 {
    double d;
    int orig, q;
};
struct MeshHit32 {
    float d;
    int q;
};

// Nearest triangle in FP64: the distance and the original index of the nearest triangle (the lowest
// among equally near ones, as a scan of all triangles in index order finds).  A subtree is dropped
// only when its box lies farther than the best distance plus a margin that covers the rounding of
// both distances, so the search returns exactly what the full scan returns.
// hint >= 0: the triangle (hierarchy position) nearest the walk's previous position, whose distance
// starts the search in place of the greedy leaf; the result does not depend on it.
// base: 0 for the surface itself, 4 for the mapped triangles.
static __device__ __attribute__((noinline)) MeshHit64 mesh_dist64(const DevInst &I, int base, double x0, double x1,
                                                          double x2, int hint)
{
#pragma clang fp contract(off)
    const double x[3] = {x0, x1, x2};
    const GPtr<MeshNode> nodes = mesh_rec<MeshNode>(I, base);
    const GPtr<MeshTri64> tris = mesh_rec<MeshTri64>(I, base + 3);
    const int nn = I.mesh_off[base + 1];
    double best = __builtin_inf(), lim = __builtin_inf();
    int bo = 0x7FFFFFFF, bq = 0;
    // One node or one triangle per iteration (lanes of a wave are at different places of the
    // search, so an iteration costs the larger of the two, not a whole leaf): the hint's triangle or
    // the greedy leaf's triangles first, then the pass from the root (that skips the greedy leaf).
    int g = -1, q, qe, i = 0;
    if (hint >= 0) {
        q = hint;
        qe = hint + 1;
    } else {
        const float xf[3] = {static_cast<float>(x[0]), static_cast<float>(x[1]), static_cast<float>(x[2])};
        g = mesh_greedy_leaf(nodes, xf);
        q = nodes[g].leaf >> 3;
        qe = q + (nodes[g].leaf & 7);
    }
    while (q < qe || i < nn) {
        if (q < qe) {
            const MeshTri64 T = tris[q];
            const double d = tri_dist64(T, x);
            const int o = T.orig;
            if (d < best || (d == best && o < bo)) {
                best = d;
                bo = o;
                bq = q;
                lim = (best + I.mesh_m64) * (best + I.mesh_m64);
            }
            ++q;
        } else {
            const MeshNode nd = nodes[i];
            if (box_gap2<double>(nd, x) > lim) {
                i = nd.skip;
            } else if (nd.leaf >= 0) {
                if (i != g) {
                    q = nd.leaf >> 3;
                    qe = q + (nd.leaf & 7);
                }
                i = nd.skip;
            } else {
                ++i;
            }
        }
    }
    return MeshHit64{best, bo, bq};
}

// Squared distance to a triangle in FP32 (the same definition; the projection test and the edge
// projections use the record's precomputed normals and inverse squared lengths).
__device__ __forceinline__ float tri_dist2_32(const MeshTri32 &T, const float *x)
{
    const float ap0 = x[0] - T.a.x, ap1 = x[1] - T.a.y, ap2 = x[2] - T.a.z;
    const float bp0 = ap0 - T.e0.x, bp1 = ap1 - T.e0.y, bp2 = ap2 - T.e0.z;
    const float cp0 = bp0 - T.e1.x, cp1 = bp1 - T.e1.y, cp2 = bp2 - T.e1.z;
    const float s0 = __builtin_fmaf(T.m0.z, ap2, __builtin_fmaf(T.m0.y, ap1, T.m0.x * ap0));
    const float s1 = __builtin_fmaf(T.m1.z, bp2, __builtin_fmaf(T.m1.y, bp1, T.m1.x * bp0));
    const float s2 = __builtin_fmaf(T.m2.z, cp2, __builtin_fmaf(T.m2.y, cp1, T.m2.x * cp0));
    const float dp = __builtin_fmaf(T.n.z, ap2, __builtin_fmaf(T.n.y, ap1, T.n.x * ap0));
    auto seg = [](float w0, float w1, float w2, const float4 &e) {
        float t = __builtin_fmaf(e.z, w2, __builtin_fmaf(e.y, w1, e.x * w0)) * e.w;
        t = __builtin_fminf(__builtin_fmaxf(t, 0.0f), 1.0f);
        const float q0 = __builtin_fmaf(-t, e.x, w0), q1 = __builtin_fmaf(-t, e.y, w1), q2 = __builtin_fmaf(-t, e.z, w2);
        return __builtin_fmaf(q2, q2, __builtin_fmaf(q1, q1, q0 * q0));
    };
    const float de = __builtin_fminf(seg(ap0, ap1, ap2, T.e0), __builtin_fminf(seg(bp0, bp1, bp2, T.e1), seg(cp0, cp1, cp2, T.e2)));
    const bool inside = s0 >= 0.0f && s1 >= 0.0f && s2 >= 0.0f;
    return inside ? dp * dp : de;
}

// Distance to the mesh in FP32 (within the FP32 error bound of the instance).
static __device__ __attribute__((noinline)) MeshHit32 mesh_dist32(const DevInst &I, int base, float x0, float x1, float x2,
                                                          int hint)
{
    const float x[3] = {x0, x1, x2};
    const GPtr<MeshNode> nodes = mesh_rec<MeshNode>(I, base);
    const GPtr<MeshTri32> tris = mesh_rec<MeshTri32>(I, base + 2);
    const int nn = I.mesh_off[base + 1];
    float best2 = __builtin_inff(), lim = __builtin_inff();
    int bq = 0;
    // one node or one triangle per iteration, the hint's triangle or the greedy leaf first, as in the
    // FP64 search
    int g = -1, q, qe, i = 0;
    if (hint >= 0) {
        q = hint;
        qe = hint + 1;
    } else {
        g = mesh_greedy_leaf(nodes, x);
        q = nodes[g].leaf >> 3;
        qe = q + (nodes[g].leaf & 7);
    }
    while (q < qe || i < nn) {
        if (q < qe) {
            const MeshTri32 T = tris[q];
            const float d2 = tri_dist2_32(T, x);
            if (d2 < best2) {
                best2 = d2;
                bq = q;
                const float b = __builtin_amdgcn_sqrtf(best2) + I.mesh_m32;
                lim = b * b;
            }
            ++q;
        } else {
            const MeshNode nd = nodes[i];
            if (box_gap2<float>(nd, x) > lim) {
                i = nd.skip;
            } else if (nd.leaf >= 0) {
                if (i != g) {
                    q = nd.leaf >> 3;
                    qe = q + (nd.leaf & 7);
                }
                i = nd.skip;
            } else {
                ++i;
            }
        }
    }
    return MeshHit32{__builtin_amdgcn_sqrtf(best2), bq};
}

// Inside test of a start point (all 64 lanes of the wave call it with the same x): the winding
// number of the surface about x, from the solid angles of the triangles seen from x (Van Oosterom and
// Strackee: 2 atan2(A.(B x C), |A||B||C| + (A.B)|C| + (A.C)|B| + (B.C)|A|) for corners A, B, C
// relative to x), lanes taking every 64th triangle; inside when the total exceeds 2 pi (winding 1/2).
static __device__ __attribute__((noinline)) bool mesh_inside_wave(const DevInst &I, double x0, double x1, double x2)
{
#pragma clang fp contract(off)
    const double x[3] = {x0, x1, x2};
    const GPtr<MeshTri64> tris = mesh_rec<MeshTri64>(I, 3);
    double acc = 0.0;
    for (int t = static_cast<int>(__lane_id()); t < I.n_verts; t += 64) {
        double A[3], B[3], C[3], bc[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            A[k] = tris[t].a[k] - x[k];
            B[k] = tris[t].b[k] - x[k];
            C[k] = tris[t].c[k] - x[k];
        }
        const double la = __builtin_sqrt(dot3d(A, A)), lb = __builtin_sqrt(dot3d(B, B)), lc = __builtin_sqrt(dot3d(C, C));
        cross3d(B, C, bc);
        const double den = la * lb * lc + dot3d(A, B) * lc + dot3d(A, C) * lb + dot3d(B, C) * la;
        acc += 2.0 * atan2(dot3d(A, bc), den);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    return acc > kTwoPi;
}

// ------------------------------------------------------------------------------------------
// Signed distance to dD, positive inside.  FP64 instantiations keep the evaluation order of the
// plain definition (no contraction), FP32 ones are the bulk path of the FP32-geometry mode.
// ------------------------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R seg_dist_sq(R ax, R ay, R ex, R ey, R ll, R x, R y,
                                                               R *t_out);
template <> __device__ __forceinline__ double seg_dist_sq<double>(double ax, double ay, double ex,
                                                                   double ey, double ll, double x,
                                                                   double y, double *t_out)
{
#pragma clang fp contract(off)
    const double wx = x - ax, wy = y - ay;
    double t = (wx * ex + wy * ey) / ll;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    const double dx = wx - t * ex, dy = wy - t * ey;
    *t_out = t;
    return dx * dx + dy * dy;
}
template <> __device__ __forceinline__ float seg_dist_sq<float>(float ax, float ay, float ex, float ey,
                                                                 float inv_ll, float x, float y,
                                                                 float *t_out)
{
    const float wx = x - ax, wy = y - ay;
    float t = (wx * ex + wy * ey) * inv_ll;
    t = __builtin_fminf(__builtin_fmaxf(t, 0.0f), 1.0f);
    const float dx = wx - t * ex, dy = wy - t * ey;
    *t_out = t;
    return dx * dx + dy * dy;
}

// Perforated domains (FP64, absolute coordinates): distance to the outer boundary (disc / ball, or
// box), and to hole h with the vector from its centre in v.
template <int KIND, int DIM> __device__ __forceinline__ double outer_dist64(const DevInst &I, const double *x)
{
#pragma clang fp contract(off)
    if constexpr (KIND == kPerforated) {
        double s = 0.0;
        for (int a = 0; a < DIM; ++a) s += (x[a] - I.p[a]) * (x[a] - I.p[a]);
        return I.p[DIM] - __builtin_sqrt(s);
    } else {
        double best = __builtin_inf();
        for (int a = 0; a < DIM; ++a) {
            const double lo = x[a] - I.p[a], hi = I.p[DIM + a] - x[a];
            best = lo < best ? lo : best;
            best = hi < best ? hi : best;
        }
        return best;
    }
}

template <int DIM> __device__ __forceinline__ double hole_dist64(const PolySeg &h, const double *x, double *v)
{
#pragma clang fp contract(off)
    v[0] = x[0] - h.ax;
    v[1] = x[1] - h.ay;
    double s = v[0] * v[0] + v[1] * v[1];
    if constexpr (DIM == 3) {
        v[2] = x[2] - h.ey;
        s += v[2] * v[2];
    }
    return __builtin_sqrt(s) - h.ex;
}

// hint (meshes only, may be null): in, the walk's previous nearest triangle (or -1); out, this one's
template <int KIND, int DIM> __device__ __forceinline__ double dist64(const DevInst &I, const double *x,
                                                                      const PolySeg *segs, int *hint = nullptr)
{
#pragma clang fp contract(off)
    if constexpr (KIND == kDisk) {
        const double dx = x[0] - I.p[0], dy = x[1] - I.p[1];
        return I.p[2] - __builtin_sqrt(dx * dx + dy * dy);
    } else if constexpr (KIND == kAnnulus) {
        const double dx = x[0] - I.p[0], dy = x[1] - I.p[1];
        const double rho = __builtin_sqrt(dx * dx + dy * dy);
        const double a = I.p[3] - rho, b = rho - I.p[2];
        return a < b ? a : b;
    } else if constexpr (KIND == kEllipse) {
        const double u = (x[0] - I.p[0]) / I.p[2], v = (x[1] - I.p[1]) / I.p[3];
        const double f = __builtin_sqrt(u * u + v * v);
        const double m = I.p[2] < I.p[3] ? I.p[2] : I.p[3];
        return m * (1.0 - f);
    } else if constexpr (KIND == kPolygon) {
        // signed: negative outside the polygon, by the parity of the edges that a ray from x
        // towards +x crosses (the straddle test reads the vertices, so two edges that share a vertex
        // agree on it)
        double best = __builtin_inf();
        bool inside = false;
        for (int e = 0; e < I.n_verts; ++e) {
            double t;
            const double q = seg_dist_sq<double>(segs[e].ax, segs[e].ay, segs[e].ex, segs[e].ey,
                                                 segs[e].ll, x[0], x[1], &t);
            const double d = __builtin_sqrt(q);
            best = d < best ? d : best;
            const double by = segs[e + 1 == I.n_verts ? 0 : e + 1].ay;
            if ((segs[e].ay > x[1]) != (by > x[1])) {
                const double side = (x[1] - segs[e].ay) * segs[e].ex - (x[0] - segs[e].ax) * segs[e].ey;
                inside ^= segs[e].ey > 0.0 ? side > 0.0 : side < 0.0;
            }
        }
        return inside ? best : -best;
    } else if constexpr (KIND == kBall) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += (x[a] - I.p[a]) * (x[a] - I.p[a]);
        return I.p[3] - __builtin_sqrt(s);
    } else if constexpr (KIND == kTriMesh) {
        // unsigned: walks start inside (an outside start point is decided by the winding number at
        // the start) and every step stays within the distance
        const MeshHit64 h = mesh_dist64(I, 0, x[0], x[1], x[2], hint ? *hint : -1);
        if (hint) *hint = h.q;
        return h.d;
    } else if constexpr (KIND == kPerforated || KIND == kPerfBox) {
        // the nearest of the outer boundary and the holes
        double best = outer_dist64<KIND, DIM>(I, x), v[DIM];
        for (int l = 0; l < I.n_verts; ++l) {
            const double d = hole_dist64<DIM>(segs[l], x, v);
            best = d < best ? d : best;
        }
        return best;
    } else {  // kBox
        double best = __builtin_inf();
        for (int a = 0; a < DIM; ++a) {
            const double lo = x[a] - I.p[a], hi = I.p[DIM + a] - x[a];
            best = lo < best ? lo : best;
            best = hi < best ? hi : best;
        }
        return best;
    }
}

// FP32 walk positions of the kinds with a centre (disk, annulus, ellipse, ball) are stored relative
// to that centre, which saves the subtractions in every distance; the FP64 exit test and the
// binning add it back.  FP64 positions are absolute.
template <int KIND> constexpr bool centred32()
{
    return KIND == kDisk || KIND == kAnnulus || KIND == kEllipse || KIND == kBall || KIND == kPerforated;
}
template <typename R, int KIND> __device__ __forceinline__ double origin(const DevInst &I, int a)
{
    if constexpr (sizeof(R) == 4 && centred32<KIND>()) return I.p[a];
    else return 0.0;
}

template <int KIND, int DIM> __device__ __forceinline__ float dist32(const DevInst &I, const float *x,
                                                                     const PolySeg *segs, int *hint = nullptr)
{
    if constexpr (KIND == kDisk) {
        return I.pf[2] - __builtin_amdgcn_sqrtf(x[0] * x[0] + x[1] * x[1]);
    } else if constexpr (KIND == kAnnulus) {
        // min(R_out - rho, rho - R_in) = w - |rho - m|, m = (R_in + R_out) / 2 = pf[4], w = (R_out - R_in) / 2 = pf[5]
        const float rho = __builtin_amdgcn_sqrtf(x[0] * x[0] + x[1] * x[1]);
        return I.pf[5] - __builtin_fabsf(rho - I.pf[4]);
    } else if constexpr (KIND == kEllipse) {
        // pf[4] = 1/a, pf[5] = 1/b, pf[6] = min(a, b)
        const float u = x[0] * I.pf[4], v = x[1] * I.pf[5];
        return I.pf[6] * (1.0f - __builtin_amdgcn_sqrtf(u * u + v * v));
    } else if constexpr (KIND == kPolygon) {
        float best = __builtin_inff();
        for (int e = 0; e < I.n_verts; ++e) {
            float t;
            best = __builtin_fminf(best, seg_dist_sq<float>(segs[e].fax, segs[e].fay, segs[e].fex,
                                                            segs[e].fey, segs[e].finv_ll, x[0], x[1], &t));
        }
        return __builtin_amdgcn_sqrtf(best);
    } else if constexpr (KIND == kBall) {
        return I.pf[3] - __builtin_amdgcn_sqrtf(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    } else if constexpr (KIND == kTriMesh) {
        const MeshHit32 h = mesh_dist32(I, 0, x[0], x[1], x[2], hint ? *hint : -1);
        if (hint) *hint = h.q;
        return h.d;
    } else if constexpr (KIND == kPerforated || KIND == kPerfBox) {
        float best;
        if constexpr (KIND == kPerforated) {  // centred positions
            float s = x[0] * x[0] + x[1] * x[1];
            if constexpr (DIM == 3) s = __builtin_fmaf(x[2], x[2], s);
            best = I.pf[DIM] - __builtin_amdgcn_sqrtf(s);
        } else {
            best = __builtin_inff();
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                best = __builtin_fminf(best, __builtin_fminf(x[a] - I.pf[a], I.pf[DIM + a] - x[a]));
        }
        for (int l = 0; l < I.n_verts; ++l) {
            const float hx = x[0] - segs[l].fax, hy = x[1] - segs[l].fay;
            float s = hx * hx + hy * hy;
            if constexpr (DIM == 3) {
                const float hz = x[2] - segs[l].fey;
                s = __builtin_fmaf(hz, hz, s);
            }
            best = __builtin_fminf(best, __builtin_amdgcn_sqrtf(s) - segs[l].fex);
        }
        return best;
    } else {
        float best = __builtin_inff();
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            best = __builtin_fminf(best, __builtin_fminf(x[a] - I.pf[a], I.pf[DIM + a] - x[a]));
        return best;
    }
}

// Step radius.  WoE bound: r = dist (the ellipsoid x + r S B(0,1) lies in B(x, r) since |S| <= 1).
// Mapped exact (boxes): the largest r with x + r S B(0,1) inside the box, min_a gap_a / |S e_a|.
// Ellipse (semi-axes a, b): in w = A^{-1}(x - c) the step ellipsoid is w + r T u, T = A^{-1} S, inside the
// unit disc for r <= g / (sqrt(t^2 + |T|^2 g) + t), t = |S A^{-1} w|, g = 1 - |w|^2 (the support bound
// |w + r T u|^2 <= |w|^2 + 2 r t + r^2 |T|^2); the Lipschitz distance bound stays valid: r = max(., d).
// Mapped bound (discs, annuli, balls): with v = x - c and a = |S v|, |v + r S u|^2 lies between
// |v|^2 - 2 r a and |v|^2 + 2 r a + r^2 for |u| <= 1, so r_out = sqrt(a^2 + R^2 - |v|^2) - a keeps the
// ellipsoid inside the circle / sphere of radius R and r_in = (|v|^2 - R_in^2) / (2 a) keeps it off
// the inner circle of an annulus, where dist is valid as well: r = min(r_out, max(r_in, dist)).
// RV: the radius variant of a launch, fixed at compile time (0: dist, or the box's radius by its mode;
// 1: mapped bound, or mapped exact for polygons) or -1: read the instance's radius mode.  A launch-wide kind selector adds
// kRadiusVariant to the kind for the mapped bound.
constexpr bool mapped_bound_kind(int kind)
{
    return kind == kDisk || kind == kAnnulus || kind == kBall || kind == kEllipse || kind == kPerforated ||
           kind == kPerfBox;
}
constexpr int kRadiusVariant = 16;

// Distance from y to the ellipsoid sum_i (z_i / e_i)^2 = 1 (y inside or outside), with b_i = e_i^2 and
// a_i = |y_i| e_i.  The nearest point is z_i = y_i b_i / (b_i + t) for the root t of
// G(t) = sum_i (a_i / (b_i + t))^2 - 1, which is convex and decreasing on t > -b_min; Newton's method
// from a point left of the root (G >= 0 there) increases monotonically to it.  When y has no
// component along the shortest axes (J) and the other terms leave G(-b_min) <= 0, the nearest point
// has t = -b_min and its J components fill the ellipsoid equation.
template <int DIM> __device__ __forceinline__ double ellipsoid_dist(const double *e, const double *y)
{
#pragma clang fp contract(off)
    double b[DIM], a[DIM], bmin = __builtin_inf();
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        b[i] = e[i] * e[i];
        a[i] = __builtin_fabs(y[i]) * e[i];
        bmin = b[i] < bmin ? b[i] : bmin;
    }
    double aj = 0.0, gd = -1.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        if (b[i] == bmin) aj = a[i] > aj ? a[i] : aj;
        else {
            const double q = a[i] / (b[i] - bmin);
            gd += q * q;
        }
    }
    double t;
    if (aj > 0.0) {
        t = aj - bmin;
    } else if (gd > 0.0) {
        t = -bmin;
    } else {  // the nearest point leaves the plane of the shortest axes
        double d2 = 0.0, used = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i)
            if (b[i] != bmin) {
                const double z = y[i] * b[i] / (b[i] - bmin);
                d2 += (y[i] - z) * (y[i] - z);
                used += z * z / b[i];
            }
        const double rest = 1.0 - used;
        return __builtin_sqrt(d2 + bmin * (rest > 0.0 ? rest : 0.0));
    }
    for (int it = 0; it < 64; ++it) {
        double g = -1.0, dg = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            const double q = a[i] / (b[i] + t);
            g += q * q;
            dg += q * q / (b[i] + t);
        }
        if (!(g > 0.0)) break;
        const double tn = t + g / (2.0 * dg);  // G' = -2 dg
        if (!(tn > t)) break;
        t = tn;
    }
    double d2 = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        const double z = y[i] * b[i] / (b[i] + t);
        d2 += (y[i] - z) * (y[i] - z);
    }
    return __builtin_sqrt(d2);
}

// Mapped-exact radius of a circle / sphere of centre c and radius R: in the eigenbasis of S
// (S = Q diag(s) Q^T) the mapped boundary S^{-1}(c + R S^{d-1}) is the ellipsoid with semi-axes R / s_k
// about S^{-1} c, and the point is w_k = (Q^T (x - c))_k / s_k.
template <int DIM> __device__ __forceinline__ double mapped_sphere_dist(const DevInst &I, const double *x,
                                                                        const double *c, double R)
{
#pragma clang fp contract(off)
    double w[DIM], e[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc += I.Sq[a * 3 + k] * (x[a] - c[a]);
        w[k] = acc / I.Se[k];
        e[k] = R / I.Se[k];
    }
    return ellipsoid_dist<DIM>(e, w);
}

// Circles and spheres (discs, annuli, balls, discs and balls with holes), mapped exact: the largest r
// is the distance from S^{-1} x to the mapped boundary, the smallest over its circles / spheres.
template <int KIND, int DIM> __device__ __forceinline__ double mapped_exact_curved(const DevInst &I, const double *x,
                                                                                   const PolySeg *segs)
{
    const double c[3] = {I.p[0], I.p[1], DIM == 3 ? I.p[2] : 0.0};
    if constexpr (KIND == kAnnulus) {
        const double ro = mapped_sphere_dist<2>(I, x, c, I.p[3]), ri = mapped_sphere_dist<2>(I, x, c, I.p[2]);
        return ro < ri ? ro : ri;
    } else {
        double r = mapped_sphere_dist<DIM>(I, x, c, I.p[DIM]);
        if constexpr (KIND == kPerforated) {
            for (int l = 0; l < I.n_verts; ++l) {
                const double h[3] = {segs[l].ax, segs[l].ay, segs[l].ey};
                const double rl = mapped_sphere_dist<DIM>(I, x, h, segs[l].ex);
                r = rl < r ? rl : r;
            }
        }
        return r;
    }
}

// Polygons (mapped exact): the ellipsoid is { z : |S^{-1}(z - x)| <= r }, so the largest inscribed r is
// the distance from S^{-1} x to the mapped edges, staged after the edges (segs[n_verts + e]).
template <int KIND, int DIM, int RV> __device__ __forceinline__ double radius64(const DevInst &I, const double *x,
                                                                                double d, const PolySeg *segs)
{
#pragma clang fp contract(off)
    if constexpr ((KIND == kDisk || KIND == kAnnulus || KIND == kBall || KIND == kPerforated) && RV < 0) {
        // mapped exact for circles and spheres: FP64 only, launched with the per-instance radius mode
        if (I.radius_mode == 1) return mapped_exact_curved<KIND, DIM>(I, x, segs);
    }
    if constexpr (KIND == kPolygon && RV != 0) {
        if (RV == 1 || I.radius_mode == 1) {
            const double y0 = I.Si[0] * x[0] + I.Si[1] * x[1], y1 = I.Si[2] * x[0] + I.Si[3] * x[1];
            double best = __builtin_inf();
            for (int e = 0; e < I.n_verts; ++e) {
                const PolySeg &m = segs[I.n_verts + e];
                double t;
                const double dd = __builtin_sqrt(seg_dist_sq<double>(m.ax, m.ay, m.ex, m.ey, m.ll, y0, y1, &t));
                best = dd < best ? dd : best;
            }
            return best;
        }
    }
    if constexpr (KIND == kEllipse && RV != 0) {
        if (RV == 1 || I.radius_mode == 2) {
            const double a = I.p[2], b = I.p[3];
            const double w0 = (x[0] - I.p[0]) / a, w1 = (x[1] - I.p[1]) / b;
            const double g = 1.0 - (w0 * w0 + w1 * w1);
            const double v0 = w0 / a, v1 = w1 / b;
            const double t0 = I.S[0] * v0 + I.S[1] * v1, t1 = I.S[3] * v0 + I.S[4] * v1;
            const double t = __builtin_sqrt(t0 * t0 + t1 * t1);
            const double r = g / (__builtin_sqrt(t * t + I.msig2 * g) + t);
            return r > d ? r : d;
        }
    } else if constexpr ((KIND == kPerforated || KIND == kPerfBox) && RV != 0) {
        if (RV == 1 || I.radius_mode == 2) {  // the outer circle / sphere (the box's exact radius), then
                                              // each hole as an inner circle
            double r_out, r_in = __builtin_inf();
            if constexpr (KIND == kPerfBox) {
                r_out = __builtin_inf();
                for (int a = 0; a < DIM; ++a) {  // min of the two gaps first: the same as min of the quotients
                    const double lo = x[a] - I.p[a], hi = I.p[DIM + a] - x[a];
                    const double g = (hi < lo ? hi : lo) / I.cn[a];
                    r_out = g < r_out ? g : r_out;
                }
            } else {
                double q = 0.0, a2 = 0.0, v[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    v[a] = x[a] - I.p[a];
                    q += v[a] * v[a];
                }
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    double w = 0.0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) w += I.S[r * 3 + a] * v[a];
                    a2 += w * w;
                }
                r_out = __builtin_sqrt(a2 + (I.p[DIM] * I.p[DIM] - q)) - __builtin_sqrt(a2);
            }
            for (int l = 0; l < I.n_verts; ++l) {
                const double c[3] = {segs[l].ax, segs[l].ay, segs[l].ey};
                double q = 0.0, a2 = 0.0, v[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    v[a] = x[a] - c[a];
                    q += v[a] * v[a];
                }
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    double w = 0.0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) w += I.S[r * 3 + a] * v[a];
                    a2 += w * w;
                }
                const double rl = (q - segs[l].ex * segs[l].ex) / (2.0 * __builtin_sqrt(a2));
                r_in = rl < r_in ? rl : r_in;
            }
            if (r_in < d) r_in = d;
            return r_out < r_in ? r_out : r_in;
        }
    } else if constexpr (mapped_bound_kind(KIND) && RV != 0) {
        if (RV == 1 || I.radius_mode == 2) {
            double v[DIM], q = 0.0, a2 = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                v[a] = x[a] - I.p[a];
                q += v[a] * v[a];
            }
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                double w = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) w += I.S[r * 3 + a] * v[a];
                a2 += w * w;
            }
            const double R = KIND == kAnnulus ? I.p[3] : I.p[DIM];
            const double r_out = __builtin_sqrt(a2 + (R * R - q)) - __builtin_sqrt(a2);
            if constexpr (KIND != kAnnulus) {
                return r_out;
            } else {
                double r_in = (q - I.p[2] * I.p[2]) / (2.0 * __builtin_sqrt(a2));
                if (r_in < d) r_in = d;
                return r_out < r_in ? r_out : r_in;
            }
        }
    }
    if constexpr (KIND == kTriMesh) {
        if (I.radius_mode == 1) {  // the distance from S^{-1} x to the mapped triangles
#pragma clang fp contract(off)
            double y[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) y[k] = I.Si3[k * 3 + 0] * x[0] + I.Si3[k * 3 + 1] * x[1] + I.Si3[k * 3 + 2] * x[2];
            return mesh_dist64(I, 4, y[0], y[1], y[2], -1).d;
        }
    }
    if constexpr (KIND == kBox) {
        if (I.radius_mode == 1) {
            // min over axes of min(lo gap, hi gap) / |S e_a|: a correctly rounded division by a positive
            // number is monotone, so dividing the smaller gap gives min of the two quotients bit for bit
            // with one division per axis in place of two
            double best = __builtin_inf();
            for (int a = 0; a < DIM; ++a) {
                const double lo = x[a] - I.p[a], hi = I.p[DIM + a] - x[a];
                const double g = (hi < lo ? hi : lo) / I.cn[a];
                best = g < best ? g : best;
            }
            return best;
        }
    }
    return d;
}

// |v|^2 and |S v|^2 in FP32.
template <int DIM> __device__ __forceinline__ void centred_norms32(const DevInst &I, const float *v, float &q, float &a2)
{
    if constexpr (DIM == 2) {
        q = __builtin_fmaf(v[0], v[0], v[1] * v[1]);
        const float w0 = __builtin_fmaf(I.Sf[0], v[0], I.Sf[1] * v[1]);
        const float w1 = __builtin_fmaf(I.Sf[3], v[0], I.Sf[4] * v[1]);
        a2 = __builtin_fmaf(w0, w0, w1 * w1);
    } else {
        q = __builtin_fmaf(v[2], v[2], __builtin_fmaf(v[1], v[1], v[0] * v[0]));
        a2 = 0.0f;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float w = __builtin_fmaf(I.Sf[r * 3 + 2], v[2], __builtin_fmaf(I.Sf[r * 3 + 1], v[1], I.Sf[r * 3] * v[0]));
            a2 = __builtin_fmaf(w, w, a2);
        }
    }
}

// FP32 form of the mapped bound on centred positions; the error bounds in mbf are subtracted.
template <int KIND, int DIM, int RV> __device__ __forceinline__ float radius32(const DevInst &I, const float *x,
                                                                               float d, const PolySeg *segs)
{
    if constexpr (KIND == kPolygon && RV != 0) {
        if (RV == 1 || I.radius_mode == 1) {
            const float y0 = __builtin_fmaf(I.Sif[0], x[0], I.Sif[1] * x[1]);
            const float y1 = __builtin_fmaf(I.Sif[2], x[0], I.Sif[3] * x[1]);
            float best = __builtin_inff();
            for (int e = 0; e < I.n_verts; ++e) {
                const PolySeg &m = segs[I.n_verts + e];
                float t;
                best = __builtin_fminf(best, seg_dist_sq<float>(m.fax, m.fay, m.fex, m.fey, m.finv_ll, y0, y1, &t));
            }
            return __builtin_amdgcn_sqrtf(best) - I.mbf[1];
        }
    }
    if constexpr (KIND == kEllipse && RV != 0) {
        if (RV == 1 || I.radius_mode == 2) {  // centred position; pf[4] = 1/a, pf[5] = 1/b
            const float w0 = x[0] * I.pf[4], w1 = x[1] * I.pf[5];
            const float g = 1.0f - __builtin_fmaf(w0, w0, w1 * w1);
            const float v0 = w0 * I.pf[4], v1 = w1 * I.pf[5];
            const float t0 = __builtin_fmaf(I.Sf[0], v0, I.Sf[1] * v1);
            const float t1 = __builtin_fmaf(I.Sf[3], v0, I.Sf[4] * v1);
            const float t2 = __builtin_fmaf(t0, t0, t1 * t1);
            const float t = __builtin_amdgcn_sqrtf(t2);
            const float sq = __builtin_amdgcn_sqrtf(__builtin_fmaf(I.mbf[0], g, t2));
            const float r = __builtin_fmaf(g, __builtin_amdgcn_rcpf(sq + t), -I.mbf[1]);
            return __builtin_fmaxf(r, d);
        }
    } else if constexpr ((KIND == kPerforated || KIND == kPerfBox) && RV != 0) {
        if (RV == 1 || I.radius_mode == 2) {  // hole records: centre (relative to the disc / ball's centre,
                                              // absolute for the box), R_l, R_l^2 (fpad0), the FP32 error
                                              // bound of the hole's radius (fpad1)
            float r_in = __builtin_inff();
            for (int l = 0; l < I.n_verts; ++l) {
                float v[DIM];
                v[0] = x[0] - segs[l].fax;
                v[1] = x[1] - segs[l].fay;
                if constexpr (DIM == 3) v[2] = x[2] - segs[l].fey;
                float ql, a2l;
                centred_norms32<DIM>(I, v, ql, a2l);
                r_in = __builtin_fminf(r_in, __builtin_fmaf(ql - segs[l].fpad0, 0.5f * __builtin_amdgcn_rsqf(a2l),
                                                            -segs[l].fpad1));
            }
            float r_out;
            if constexpr (KIND == kPerfBox) {  // the box's exact radius, as for WOS_BOX
                r_out = __builtin_inff();
#pragma unroll
                for (int a = 0; a < DIM; ++a)
                    r_out = __builtin_fminf(r_out, __builtin_fminf(x[a] - I.pf[a], I.pf[DIM + a] - x[a]) * I.icnf[a]);
            } else {
                float q, a2;
                centred_norms32<DIM>(I, x, q, a2);
                r_out = __builtin_amdgcn_sqrtf(a2 + (I.mbf[0] - q)) - (__builtin_amdgcn_sqrtf(a2) + I.mbf[1]);
            }
            return __builtin_fminf(r_out, __builtin_fmaxf(r_in, d));
        }
    } else if constexpr (mapped_bound_kind(KIND) && RV != 0) {
        if (RV == 1 || I.radius_mode == 2) {
            float q, a2;
            centred_norms32<DIM>(I, x, q, a2);
            const float s = __builtin_amdgcn_sqrtf(a2 + (I.mbf[0] - q));
            if constexpr (KIND == kAnnulus) {
                const float rq = __builtin_amdgcn_rsqf(a2);  // a2 >= (sigma_min R_in)^2 > 0
                const float r_out = s - __builtin_fmaf(a2, rq, I.mbf[1]);
                const float r_in = __builtin_fmaf(q - I.mbf[2], 0.5f * rq, -I.mbf[3]);
                return __builtin_fminf(r_out, __builtin_fmaxf(r_in, d));
            } else {
                return s - (__builtin_amdgcn_sqrtf(a2) + I.mbf[1]);
            }
        }
    }
    if constexpr (KIND == kTriMesh) {
        if (I.radius_mode == 1) {  // mapped triangles, less the FP32 error bound of that distance (mbf[1])
            float y[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                y[k] = __builtin_fmaf(I.Sif3[k * 3 + 2], x[2], __builtin_fmaf(I.Sif3[k * 3 + 1], x[1], I.Sif3[k * 3] * x[0]));
            return mesh_dist32(I, 4, y[0], y[1], y[2], -1).d - I.mbf[1];
        }
    }
    if constexpr (KIND == kBox) {
        if (I.radius_mode == 1) {
            float best = __builtin_inff();
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                // the smaller gap times 1 / |S e_a| (rounding is monotone: the same as the smaller product)
                best = __builtin_fminf(best, __builtin_fminf(x[a] - I.pf[a], I.pf[DIM + a] - x[a]) * I.icnf[a]);
            return best;
        }
    }
    return d;
}

// ------------------------------------------------------------------------------------------
// Cell index of the projection of a stop point onto dD (FP64).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int clamp_index(double v, int n)
{
    const double f = __builtin_floor(v);
    if (!(f >= 0.0)) return 0;  // also catches NaN
    if (f > static_cast<double>(n - 1)) return n - 1;
    return static_cast<int>(f);
}

// Arc of angle theta in (-pi, pi] among n equal arcs counted counter-clockwise from angle 0.
__device__ __forceinline__ int arc_of(double theta, int n)
{
#pragma clang fp contract(off)
    if (theta < 0.0) theta += kTwoPi;
    return clamp_index(theta * static_cast<double>(n) / kTwoPi, n);
}

// Cell index of an FP32 stop position (relative to the centre) on the circles of a disk or an
// annulus, computed in FP32 and returned only where it certainly equals element64's result, else
// -1.  The angle in revolutions, atan2(y, x) / 2 pi, comes from an odd polynomial in
// a = min(|x|, |y|) / max(|x|, |y|) (least-squares fit of atan(a) / 2 pi on [0, 1], evaluated error
// below 2^-24 rev) and three reflections; with the division and the reflections its error stays
// below 2^-21 rev, and t = rev n below n (2^-21 + 2^-24) from the exact value.  The arc floor(t) is
// accepted when t lies farther than n 2^-20 from an integer.  The annulus circle is decided by
// rho^2 against (m -+ w/4)^2 (pf[6], pf[7]; m, w the middle radius and half width); stops lie
// within eps of a circle, w from the middle.
template <int KIND> __device__ __forceinline__ int element32_certified(const DevInst &I, float x, float y)
{
    const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
    const float a = __builtin_fminf(ax, ay) * __builtin_amdgcn_rcpf(__builtin_fmaxf(ax, ay));
    const float z = a * a;
    float p = 0.0010841292096301913f;
    p = __builtin_fmaf(p, z, -0.005348275415599346f);
    p = __builtin_fmaf(p, z, 0.012672500684857368f);
    p = __builtin_fmaf(p, z, -0.021061519160866737f);
    p = __builtin_fmaf(p, z, 0.03152512013912201f);
    p = __builtin_fmaf(p, z, -0.053026240319013596f);
    p = __builtin_fmaf(p, z, 0.15915432572364807f);
    float r = p * a;                 // atan(a) / 2 pi, in [0, 1/8]
    if (ay > ax) r = 0.25f - r;      // angle of (max, min) reflected about the diagonal
    if (x < 0.0f) r = 0.5f - r;
    if (y < 0.0f) r = -r;            // (-1/2, 1/2]
    if (r < 0.0f) r += 1.0f;         // [0, 1]
    int n = I.layout[0], off = 0;
    if constexpr (KIND == kAnnulus) {
        const float rho2 = __builtin_fmaf(x, x, y * y);
        if (rho2 >= I.pf[7]) {
            n = I.layout[0];
        } else if (rho2 <= I.pf[6]) {
            n = I.layout[1];
            off = I.layout[0];
        } else {
            return -1;
        }
    }
    const float nf = static_cast<float>(n);
    const float t = r * nf;
    const float fl = __builtin_floorf(t);
    const float fr = t - fl;
    const float m = nf * 0x1.0p-20f;
    if (!(fr > m && fr < 1.0f - m)) return -1;
    return off + static_cast<int>(fl);
}

// Equal-area cell of a direction v (any length > 0): band of the height v_z / |v| from the top
// (nz bands), then the azimuth sector (nphi sectors from angle 0).
__device__ __forceinline__ int sphere_cell(const double *v, int nz, int nphi)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += v[a] * v[a];
    const double zc = v[2] / __builtin_sqrt(s);
    const int iz = clamp_index((1.0 - zc) * 0.5 * static_cast<double>(nz), nz);
    return iz * nphi + arc_of(atan2(v[1], v[0]), nphi);
}

// Extrinsic Voronoi cell (Appendix Ex. A.2) among the n Bauer nodes R u_k of a sphere, v the point
// relative to the centre: the node nearest v, the lowest index on ties.  Node k has u_k.z = 1 - (2k + 1)/n,
// and |v - R u_k|^2 = (|v| - R)^2 + R |v| |u - u_k|^2 >= (|v| - R)^2 + R |v| (z - u_k.z)^2 (u = v/|v|,
// z = u.z): after a first window of about one turn of the spiral around the node of v's z band, a node
// can only beat the best score s when (z - u_k.z)^2 <= (s - (|v| - R)^2) / (R |v|), an index range that
// the search then completes.  Scores are the plain squared distances, so the cell equals a full scan's.
__device__ __forceinline__ int bauer_cell(const double *v, double R, int n, const PolySeg *u)
{
#pragma clang fp contract(off)
    const double rv = __builtin_sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double z = v[2] / rv;
    auto score = [&](int k) {
        const double t0 = v[0] - R * u[k].ax, t1 = v[1] - R * u[k].ay, t2 = v[2] - R * u[k].ey;
        return t0 * t0 + t1 * t1 + t2 * t2;
    };
    const int k0 = clamp_index((1.0 - z) * 0.5 * static_cast<double>(n), n);
    const int w = static_cast<int>(__builtin_sqrt(static_cast<double>(n) * 3.141592653589793)) + 2;
    const int lo = k0 - w < 0 ? 0 : k0 - w, hi = k0 + w > n - 1 ? n - 1 : k0 + w;
    double best = __builtin_inf();
    int bk = lo;
    for (int k = lo; k <= hi; ++k) {
        const double sc = score(k);
        if (sc < best) {
            best = sc;
            bk = k;
        }
    }
    // the z range that can still hold a better node (1e-12: far above the scores' rounding)
    const double t = (best - (rv - R) * (rv - R)) / (R * rv) + 1e-12;
    const double dz = __builtin_sqrt(t > 0.0 ? t : 0.0);
    const double nn = static_cast<double>(n);
    double flo = __builtin_floor(((1.0 - (z + dz)) * nn - 1.0) * 0.5);
    double fhi = __builtin_ceil(((1.0 - (z - dz)) * nn - 1.0) * 0.5);
    const int klo = !(flo > 0.0) ? 0 : (flo > nn - 1.0 ? n - 1 : static_cast<int>(flo));  // NaN: 0
    const int khi = !(fhi > 0.0) ? 0 : (fhi > nn - 1.0 ? n - 1 : static_cast<int>(fhi));
    for (int k = klo; k < lo; ++k) {
        const double sc = score(k);
        if (sc < best || (sc == best && k < bk)) {
            best = sc;
            bk = k;
        }
    }
    for (int k = hi + 1; k <= khi; ++k) {
        const double sc = score(k);
        if (sc < best) {
            best = sc;
            bk = k;
        }
    }
    return bk;
}

// Cell of a sphere of radius R: layout (n_z, n_phi) gives the equal-area (z band, azimuth) cells,
// (n, 0) the Voronoi cells of n Bauer nodes (table `nodes`, in HBM).
__device__ __forceinline__ int sphere_cell_of(const double *v, int nz, int nphi, double R, const PolySeg *nodes)
{
    return nphi == 0 ? bauer_cell(v, R, nz, nodes) : sphere_cell(v, nz, nphi);
}

// Box: the nearest face (ties: the lowest face index), then the patch of the other coordinates.
template <int DIM> __device__ __forceinline__ int box_cell(const DevInst &I, const double *x)
{
#pragma clang fp contract(off)
    const int n = I.layout[0];
    double best = __builtin_inf();
    int fb = 0;
    for (int f = 0; f < 2 * DIM; ++f) {
        const int a = f >> 1;
        const double df = (f & 1) == 0 ? x[a] - I.p[a] : I.p[DIM + a] - x[a];
        if (df < best) { best = df; fb = f; }
    }
    const int a = fb >> 1;
    int idx = 0;
    for (int b = 0; b < DIM; ++b) {
        if (b == a) continue;
        const double lo = I.p[b], hi = I.p[DIM + b];
        idx = idx * n + clamp_index((x[b] - lo) / (hi - lo) * static_cast<double>(n), n);
    }
    return fb * (DIM == 2 ? n : n * n) + idx;
}

template <int KIND, int DIM> __device__ __forceinline__ int element64(const DevInst &I, const double *x,
                                                                      const PolySeg *segs)
{
#pragma clang fp contract(off)
    if constexpr (KIND == kDisk) {
        return arc_of(atan2(x[1] - I.p[1], x[0] - I.p[0]), I.layout[0]);
    } else if constexpr (KIND == kAnnulus) {
        const double dx = x[0] - I.p[0], dy = x[1] - I.p[1];
        const double rho = __builtin_sqrt(dx * dx + dy * dy);
        const double th = atan2(dy, dx);
        if (I.p[3] - rho <= rho - I.p[2]) return arc_of(th, I.layout[0]);
        return I.layout[0] + arc_of(th, I.layout[1]);
    } else if constexpr (KIND == kEllipse) {
        const double u = (x[0] - I.p[0]) / I.p[2], v = (x[1] - I.p[1]) / I.p[3];
        return arc_of(atan2(v, u), I.layout[0]);
    } else if constexpr (KIND == kPolygon) {
        double best = __builtin_inf(), tb = 0.0;
        int eb = 0;
        for (int e = 0; e < I.n_verts; ++e) {
            double t;
            const double d = __builtin_sqrt(seg_dist_sq<double>(segs[e].ax, segs[e].ay, segs[e].ex,
                                                                segs[e].ey, segs[e].ll, x[0], x[1], &t));
            if (d < best) { best = d; eb = e; tb = t; }
        }
        const double s_at = segs[eb].cum + tb * segs[eb].len;
        return clamp_index(s_at * static_cast<double>(I.layout[0]) / I.perim, I.layout[0]);
    } else if constexpr (KIND == kPerforated || KIND == kPerfBox) {
        // the nearest piece of the boundary (ties: the outer one, then the lowest hole), then the
        // cell of the direction from the piece's centre; outer cells first, then each hole's
        double best = outer_dist64<KIND, DIM>(I, x), v[3] = {0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0};
        int comp = -1;
        for (int l = 0; l < I.n_verts; ++l) {
            const double d = hole_dist64<DIM>(segs[l], x, v);
            if (d < best) {
                best = d;
                comp = l;
#pragma unroll
                for (int a = 0; a < DIM; ++a) vb[a] = v[a];
            }
        }
        int n_out, hc, c;
        const double Rh = comp >= 0 ? segs[comp].ex : 0.0;
        if constexpr (KIND == kPerforated) {
            n_out = DIM == 2 ? I.layout[0] : (I.layout[1] == 0 ? I.layout[0] : I.layout[0] * I.layout[1]);
            hc = DIM == 2 ? I.layout[1] : (I.layout[3] == 0 ? I.layout[2] : I.layout[2] * I.layout[3]);
            if (comp < 0) {
                double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int a = 0; a < DIM; ++a) w[a] = x[a] - I.p[a];
                return DIM == 2 ? arc_of(atan2(w[1], w[0]), I.layout[0])
                                : sphere_cell_of(w, I.layout[0], I.layout[1], I.p[DIM], I.segs + I.node_off[0]);
            }
            c = DIM == 2 ? arc_of(atan2(vb[1], vb[0]), I.layout[1])
                         : sphere_cell_of(vb, I.layout[2], I.layout[3], Rh, I.segs + I.node_off[1]);
        } else {
            n_out = DIM == 2 ? 4 * I.layout[0] : 6 * I.layout[0] * I.layout[0];
            hc = DIM == 2 ? I.layout[1] : (I.layout[2] == 0 ? I.layout[1] : I.layout[1] * I.layout[2]);
            if (comp < 0) return box_cell<DIM>(I, x);
            c = DIM == 2 ? arc_of(atan2(vb[1], vb[0]), I.layout[1])
                         : sphere_cell_of(vb, I.layout[1], I.layout[2], Rh, I.segs + I.node_off[1]);
        }
        return n_out + comp * hc + c;
    } else if constexpr (KIND == kBall) {
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = x[a] - I.p[a];
        return sphere_cell_of(v, I.layout[0], I.layout[1], I.p[3], I.segs + I.node_off[0]);
    } else if constexpr (KIND == kTriMesh) {  // the nearest triangle; layout[0] triangles per element
        return mesh_dist64(I, 0, x[0], x[1], x[2], -1).orig / I.layout[0];
    } else {  // kBox
        return box_cell<DIM>(I, x);
    }
}

// Signed distance of a start point.  For a mesh the unsigned distance gets the sign of the winding-number
// test; all 64 lanes of the wave must call this together (with the same x).
template <int KIND, int DIM> __device__ __forceinline__ double start_dist64(const DevInst &I, const double *x,
                                                                           const PolySeg *segs)
{
    const double d = dist64<KIND, DIM>(I, x, segs);
    if constexpr (KIND == kTriMesh) return mesh_inside_wave(I, x[0], x[1], x[2]) ? d : -d;
    return d;
}

}  // namespace wos
