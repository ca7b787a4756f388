/*
 * wos.h -- C ABI of libwos: walk-on-ellipsoids Monte Carlo estimation of the discretised elliptic
 * measure on one AMD Instinct MI355X (gfx950), and the FP64 truncated-SVD / Tikhonov reconstruction
 * of the inaccessible boundary data that consumes it.
 *
 * The method is that of Cimpean, Grecu and Marin, "Numerical spectral analysis of Cauchy-type
 * inverse problems: a probabilistic approach" (arXiv 2409.03686):
 *   - the walk-on-ellipsoids chain X_{n+1} = X_n + dist(X_n, dD) K^{1/2} U_n with lambda_max(K) = 1
 *     (Section 4.2, eq. "wos chain"), stopped at the first n with dist(X_n, dD) <= eps
 *     (eq. "N epsilon x");
 *   - the Monte Carlo matrix A_{omega,eps,N}[i, j] = (1/N) #{walks from x_i stopping in cell j}
 *     (Section 4.3.1, eq. "WoE_matrix_MC" and its Voronoi counting form; Algorithm "MC-REM");
 *   - the scaled direct operator B = diag(nu) A_{Gamma_1} diag(sigma)^{-1/2}, its SVD, and the
 *     TSVD solution u_1 = diag(sigma)^{-1/2} B_r^+ diag(nu) b, b = u^D - A_{Gamma_0} u^0
 *     (Sections 3 and 5.1, eqs. "SVD", "u1r", "tsvd solution simulations"; Algorithm "Main").
 *
 * Conventions common to every entry point
 *   - Every function returns a wos_status.  On any status other than WOS_OK, wos_last_error()
 *     returns a message for the calling thread.  Argument checks run on the host before any device
 *     work, so WOS_EINVAL never leaves partial device work behind.
 *   - "_dev" pointers are device (HBM) pointers on the context's device; "_host" pointers are host
 *     memory.  The caller owns every buffer it passes in; the library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is enqueued on it and the
 *     call returns without waiting, unless stated otherwise.
 *   - Matrices are row-major unless stated otherwise.  Element (boundary cell) indices follow the
 *     per-kind layout documented at wos_geometry.
 *   - A context is used by one host thread at a time, except the wos_serve* entry points which
 *     synchronise internally.
 */
#ifndef WOS_H
#define WOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WOS_OK = 0,
    WOS_EINVAL = 1,     /* invalid argument (nothing was enqueued) */
    WOS_ENOMEM = 2,     /* device or host allocation failed, or the HBM budget is exceeded */
    WOS_EDEVICE = 3,    /* a HIP call failed; the context is unusable afterwards */
    WOS_EBUSY = 4,      /* the serving queue is full */
    WOS_ETIMEOUT = 5,   /* a serving request exceeded its time limit */
    WOS_ENOTSUP = 6,    /* valid request outside what the library supports */
    WOS_ECANCELLED = 7  /* a serving request was cancelled */
} wos_status;

typedef struct wos_ctx wos_ctx;

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the device memory the
 * library itself allocates (scratch, SVD workspaces, serving slots); 0 = no bound. */
wos_status wos_create(wos_ctx **out, int device, size_t hbm_budget_bytes);
/* Waits for the context's own streams and frees everything it allocated. */
wos_status wos_destroy(wos_ctx *ctx);
/* Message of the last non-OK status returned on this thread ("" if none). */
const char *wos_last_error(void);

/* Two streams of the context's device on disjoint sets of CUs (HIP CU masks): *spectral_stream
 * may use the last spectral_cus CUs, *walk_stream all the others.  With the walk kernel of one
 * instance on the walk stream and the spectral step (assembly, SVD, reconstruction) of the
 * previous instance on the spectral stream, the two overlap: the spectral step is latency-bound
 * on a few workgroups, and its cooperative Jacobi launch does not share CUs with the persistent
 * walk kernel.  Walk grids and cooperative SVD grids are sized for the CUs of the stream they are
 * launched on, so every entry point that takes a stream works on either; results are the same as
 * on an unrestricted stream.  1 <= spectral_cus < number of CUs.  The caller owns the streams and
 * releases them with wos_streams_destroy (after its work on them has finished). */
wos_status wos_streams_create(wos_ctx *ctx, int32_t spectral_cus, void **walk_stream, void **spectral_stream);
wos_status wos_streams_destroy(wos_ctx *ctx, void *walk_stream, void *spectral_stream);

/* ------------------------------------------------------------------------------------------- */
/* Geometry                                                                                      */
/* ------------------------------------------------------------------------------------------- */
/* Domain kinds and their parameters (all coordinates in the original, unmapped frame):
 *   WOS_DISK     dim 2, params (cx, cy, R),           layout (M)            M equal arcs, counter-
 *                clockwise from angle 0; arc j = [2 pi j / M, 2 pi (j+1) / M).
 *   WOS_ANNULUS  dim 2, params (cx, cy, R_in, R_out), layout (M_out, M_in)  outer arcs 0..M_out-1,
 *                then inner arcs; a point is assigned to the nearer circle (ties: outer).
 *   WOS_ELLIPSE  dim 2, params (cx, cy, a, b),        layout (M)            M equal steps of the
 *                eccentric angle t of (cx + a cos t, cy + b sin t).  The walk uses the Lipschitz
 *                lower bound min(a,b) (1 - f(x)) of the distance, f the ellipse gauge (the paper's
 *                remark on Lipschitz replacements of dist), and cells by the eccentric angle.
 *   WOS_POLYGON  dim 2, verts = one counter-clockwise loop of n_verts (x, y) pairs (host), layout
 *                (M): M equal pieces of the perimeter, counted from vertex 0.
 *   WOS_BALL     dim 3, params (cx, cy, cz, R),       layout (n_z, n_phi)   equal-area cells:
 *                band iz over z from the top, sector iphi over the azimuth; j = iz n_phi + iphi.
 *                Every sphere layout may instead be (n, 0), n >= 16: the extrinsic Voronoi cells
 *                (appendix, Ex. A.2) of the n nodes of Bauer's spiral of Section 5.3, polar angle
 *                arccos(1 - (2k - 1)/n) and azimuth sqrt(n pi) times it, k = 1..n (cell k - 1):
 *                the point goes to the nearest node of its sphere, ties to the lower index; cell
 *                measures are the spherical Voronoi areas.
 *   WOS_BOX      dim 2 or 3, params (lo_0..lo_{d-1}, hi_0..hi_{d-1}), layout (n): faces in the
 *                order (x=lo, x=hi, y=lo, y=hi[, z=lo, z=hi]), n^(d-1) patches each, patch
 *                indices along the remaining axes in increasing axis order; j = f n^(d-1) + idx.
 *   WOS_PERFORATED a disc or ball with k disjoint round holes (the paper's Examples 2-4, 6, 7).
 *                params (centre, R) of the outer disc / ball; verts = k holes as (centre, r)
 *                records of dim + 1 numbers (host, n_verts = k).  dim 2: layout (M_out, M_hole, k):
 *                M_out arcs of the outer circle, then M_hole arcs of each hole in hole order, all
 *                counter-clockwise from angle 0 about their own centre.  dim 3: layout (n_z, n_phi,
 *                n_z hole, n_phi hole): the outer sphere's equal-area cells as for WOS_BALL, then
 *                each hole sphere's, about its own centre.  A point goes to the nearest piece
 *                (ties: the outer one, then the lowest hole).  Holes must lie strictly inside the
 *                outer boundary and must not overlap.
 *   WOS_PERFBOX  a box with k disjoint round holes (the paper's Examples 1 and 5).  params and
 *                face patches as WOS_BOX, holes as for WOS_PERFORATED; layout (n, M_hole) in 2D,
 *                (n, n_z hole, n_phi hole) in 3D: the box's patches first, then each hole's cells.
 *   WOS_TRIMESH  dim 3, the interior of a closed surface of triangles (general distance functions are
 *                allowed by the Remark on Algorithm MC-REM, item (ii)).  verts = n_verts triangles
 *                (a, b, c) as 9 numbers each (host, copied during the call), counter-clockwise seen
 *                from outside; 4 <= n_verts <= WOS_MAX_TRIANGLES; degenerate triangles are refused.
 *                layout (g): g consecutive triangles form one cell (g divides n_verts), so M =
 *                n_verts / g.  dist is the distance to the nearest triangle: the plane distance when
 *                the point's projection onto the triangle's plane lies in the triangle, else the
 *                distance to the nearest of its edges.  A stop point goes to the cell of the nearest
 *                triangle (ties: the lowest triangle index).  A start point whose winding number
 *                (the triangles' solid angles seen from it over 4 pi) is below 1/2 is outside: its
 *                walks are escapes.  Step radius r = dist (WOS_RADIUS_WOE_BOUND) or the mapped-exact
 *                radius (WOS_RADIUS_MAPPED_EXACT: the distance from S^{-1} x to the mapped triangles
 *                S^{-1} T, searched in a second hierarchy); WOS_RADIUS_MAPPED_BOUND is refused.  The
 *                triangles are searched through a bounding-volume hierarchy in HBM (256 B per triangle
 *                plus 32 B per node, twice with the mapped-exact radius, rebuilt on the host for each
 *                call).
 * A stop point is assigned to the cell containing its projection onto dD (the intrinsic Voronoi
 * weights of the paper's appendix, Ex. A.3; for Bauer layouts the extrinsic ones of Ex. A.2, taken
 * on the stop point's nearest sphere); ties go to the lowest face/segment index. */
typedef enum {
    WOS_DISK = 0, WOS_ANNULUS = 1, WOS_ELLIPSE = 2, WOS_POLYGON = 3, WOS_BALL = 4, WOS_BOX = 5,
    WOS_PERFORATED = 6, WOS_PERFBOX = 7, WOS_TRIMESH = 8
} wos_geom_kind;

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t kind;         /* wos_geom_kind */
    double params[8];
    int32_t layout[4];
    const double *verts;  /* host; polygon vertices, the holes of a perforated domain or the triangles of a
                             mesh (copied during the call) */
    int32_t n_verts;      /* polygon: 3..WOS_MAX_POLY_VERTS vertices; perforated domains: holes; mesh: triangles */
} wos_geometry;

#define WOS_MAX_POLY_VERTS 64
#define WOS_MAX_HOLES 32
#define WOS_MAX_TRIANGLES (1 << 20)
#define WOS_MAX_ELEMENTS 16384  /* one LDS histogram row must fit in 64 KiB */

/* Number of boundary cells M of a geometry. */
wos_status wos_element_count(const wos_geometry *geom, int32_t *n_elem);
/* sigma_host[M] = surface measure of each cell (the sigma(omega_j) of eq. "boundary_weights"). */
wos_status wos_element_measures(const wos_geometry *geom, double *sigma_host);

/* ------------------------------------------------------------------------------------------- */
/* Measure building (Algorithm MC-REM)                                                           */
/* ------------------------------------------------------------------------------------------- */
typedef enum { WOS_FP64 = 0, WOS_FP32_GEOM_FP64_EXIT = 1 } wos_precision;
/* Step radius r of X + r S U (S = (K / lambda_max)^{1/2}).  The chain of Section 4.2 is the trace
 * of the diffusion on ellipsoids inscribed in D, so any r whose ellipsoid X + r S B(0,1) lies in D
 * gives the same exit law; larger radii give shorter walks.
 *   WOE_BOUND     r = dist(X, dD), the radius of eq. "wos chain" (every domain).
 *   MAPPED_EXACT  the largest inscribed radius, the distance from S^{-1} X to the mapped boundary
 *                 S^{-1} dD (the ellipsoid is the set of z with |S^{-1}(z - X)| <= r): for a box min
 *                 over faces of gap_a / |S e_a|; for a polygon the distance to the mapped edges
 *                 S^{-1}[a, b]; for a mesh the distance to the mapped triangles S^{-1} T; for discs, annuli, balls and discs / balls with holes (FP64 geometry
 *                 only) the distance to the mapped circles / spheres, ellipses / ellipsoids with
 *                 semi-axes R / s_k along the eigenvectors of S (eigenvalues s_k), computed by
 *                 Newton's method on the closest-point equation (§5.1, Remark on Alg. MC-REM,
 *                 item (ii): a distance replaced by another valid one).
 *   MAPPED_BOUND  discs, annuli, balls, ellipses, and discs, balls and boxes with holes
 *                 (WOS_PERFORATED, WOS_PERFBOX): with v = X - c and a = |S v|,
 *                 r = sqrt(a^2 + R^2 - |v|^2) - a for the outer circle or sphere of radius R (for a
 *                 box its exact radius as above); for the inner circle of an annulus, or each hole
 *                 (v and a from its centre), (|v|^2 - R_in^2) / (2 a); r = min(outer, max(smallest
 *                 inner, dist)) (equal to dist when S = I).  Ellipse (semi-axes a, b, A = diag(a, b)):
 *                 with w = A^{-1}(X - c), t = |S A^{-1} w|, g = 1 - |w|^2 and s2 = |A^{-1} S|^2,
 *                 r = max(g / (sqrt(t^2 + s2 g) + t), dist bound).
 * Other combinations return WOS_ENOTSUP. */
typedef enum { WOS_RADIUS_WOE_BOUND = 0, WOS_RADIUS_MAPPED_EXACT = 1, WOS_RADIUS_MAPPED_BOUND = 2 } wos_radius_mode;

typedef struct {
    double K[9];          /* conductivity, row-major, leading dim x dim block; symmetric positive
                             definite; only K / lambda_max(K) enters the walk (Section 4.2) */
    double eps;           /* stopping shell width, > 0; or 0 with WOS_FP64 and max_steps >= 1: the
                             fixed-iteration walk (Remark on Algorithm MC-REM, item (i)), in which
                             every walk makes exactly max_steps steps, stops earlier only on
                             reaching dD (dist <= 0) and is binned at its last point */
    uint64_t walk_begin;  /* walks k in [walk_begin, walk_end) are run for every point; */
    uint64_t walk_end;    /* walk_end <= 2^32, walk_end - walk_begin < 2^32.  Splitting a range and summing is bit-exact. */
    uint64_t seed;        /* Philox key (low word, high word) */
    uint32_t instance;    /* Philox counter word 3: distinguishes instances sharing a seed */
    int32_t precision;    /* wos_precision */
    int32_t radius_mode;  /* wos_radius_mode (MAPPED_EXACT: boxes, polygons, meshes, and in FP64 discs, annuli,
                             balls, perforated discs and balls; MAPPED_BOUND: discs, annuli, balls, ellipses,
                             perforated discs, balls and boxes) */
    uint32_t max_steps;   /* step cap S_max (0 -> 10000, must be < 2^31); capped walks are binned where they are */
} wos_walk_params;

/* Random numbers: Philox4x32-10 (Salmon et al., SC'11), key (seed lo, seed hi), counter
 * (block b, walk k, point i, instance).  FP64: the q-th uniform of a walk is the top 53 bits of
 * words (2(q&1), 2(q&1)+1) of block q>>1, u = m 2^-53 + 2^-54; step s uses q = s in 2D (angle
 * 2 pi u) and q = 2s, 2s+1 in 3D (z = 1 - 2u, azimuth 2 pi u).  FP32 geometry: the q-th uniform
 * is the top 24 bits of word q&3 of block q>>2, u = m 2^-24 + 2^-25, same q per step. */

/* Statistics words accumulated into stats_dev (uint64[WOS_STATS_WORDS]). */
enum {
    WOS_STAT_WALKS = 0, WOS_STAT_STEPS = 1, WOS_STAT_MAX_STEPS = 2, WOS_STAT_CAP_HITS = 3,
    WOS_STAT_ESCAPES = 4, WOS_STAT_FP64_EVALS = 5, WOS_STAT_LANE_SLOTS = 6, WOS_STATS_WORDS = 8
};

/* Runs walks [walk_begin, walk_end) from each of the n_obs points and ACCUMULATES
 *   counts_dev[i * M + j] += #{walks from point i stopping in cell j}
 * (uint32, row-major n_obs x M, caller-zeroed), so sub-ranges, resumed runs and shards sum
 * bit-exactly.  x_obs_dev: double[n_obs * dim] row-major.  stats_dev (optional): accumulated
 * statistics (walks, sphere steps, max steps (a maximum), cap hits, escapes = stop points with a
 * negative distance, FP64 shell evaluations, lane-step slots issued).  trace_dev (optional):
 * int32[n_obs * (walk_end - walk_begin) * 2] receiving (cell, steps) of every walk, for tests.
 * Points outside D stop with zero steps and count as escapes.  Every row sums to exactly
 * walk_end - walk_begin.  Asynchronous on `stream`. */
wos_status wos_build_measure(wos_ctx *ctx, const wos_geometry *geom, const wos_walk_params *walk,
                             const double *x_obs_dev, int32_t n_obs, uint32_t *counts_dev,
                             uint64_t *stats_dev, int32_t *trace_dev, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): wos_build_measure with the same arguments, results and errors, whose
 * scratch (the instance descriptor with its geometry records, at most 64 KiB, and the work cursors,
 * at most 2^18 + 2 words: 2^18 points in point mode) lives in a static device array of 1.06 MiB
 * that each GPU holds until the process ends.  The call allocates no device or pinned memory: the
 * descriptor reaches the array through the arguments of small kernels (so a captured graph holds
 * the bytes), the cursors are cleared by a kernel.  Larger descriptors or cursor counts return
 * WOS_EINVAL before anything is enqueued.  Every call on a GPU shares that GPU's array, which keeps
 * the last call's contents: calls that overlap on one GPU (different streams, threads or contexts)
 * race and must be serialised by the caller. */
wos_status wos_build_measure_noalloc(wos_ctx *ctx, const wos_geometry *geom, const wos_walk_params *walk,
                                     const double *x_obs_dev, int32_t n_obs, uint32_t *counts_dev,
                                     uint64_t *stats_dev, int32_t *trace_dev, void *stream);

/* One instance of a batched build. */
typedef struct {
    wos_geometry geom;
    wos_walk_params walk;
    const double *x_obs_dev;
    int32_t n_obs;
    uint32_t *counts_dev;
    uint64_t *stats_dev;   /* optional, per instance */
    int32_t *trace_dev;    /* optional, per instance */
} wos_measure_job;

/* Builds the measures of n_jobs heterogeneous instances with persistent kernels that pull
 * (instance, point, walk-chunk) work items from one global queue per (precision, dimension)
 * group; results are identical to n_jobs separate wos_build_measure calls. */
wos_status wos_build_measure_batch(wos_ctx *ctx, const wos_measure_job *jobs, int32_t n_jobs,
                                   void *stream);

/* Launch shape of the walk kernel: threads per block, walks per lane per work item, and who owns the
 * work.  WOS_ITEMS_BLOCK: the waves of a block share an item (point, walk range) and drain together
 * at its end.  WOS_ITEMS_WAVE: every wave owns its items and starts the walks of its next item while
 * the last walks of the previous one still run (two histogram rows per wave in LDS): fewer idle
 * lanes, more instructions per step.  WOS_ITEMS_POINT: a block owns a point and its waves reserve
 * the point's walks walks_per_lane per lane at a time until none are left; blocks without a point
 * join points that still have walks, so lanes drain only when a point runs out.  WOS_ITEMS_AUTO is
 * the point mode for WOS_FP64 walks and the block mode otherwise (the faster ones measured); the
 * autotuner times all three.  A mode that does not apply falls back to the
 * block mode (wave mode above 64 KiB of LDS per block, point mode above 2^30 walks per point).
 * The counts never depend on these choices. */
typedef enum { WOS_ITEMS_AUTO = 0, WOS_ITEMS_BLOCK = 1, WOS_ITEMS_WAVE = 2, WOS_ITEMS_POINT = 3 } wos_item_mode;
typedef struct {
    int32_t block;          /* 64, 128, 256, 512 or 1024 */
    int32_t walks_per_lane; /* >= 1 */
    int32_t items;          /* wos_item_mode */
} wos_tuning;

/* Sets the launch shape used for (dim, kind, precision) from now on (kind < 0: all kinds). */
wos_status wos_set_tuning(wos_ctx *ctx, int32_t dim, int32_t kind, int32_t precision,
                          const wos_tuning *t);
/* Times every candidate launch shape on a walk sub-range of `job` (results discarded), stores the
 * fastest for the job's (dim, kind, precision) and returns it.  Blocking. */
wos_status wos_autotune(wos_ctx *ctx, const wos_measure_job *job, uint64_t sample_walks,
                        wos_tuning *best, void *stream);

/* ------------------------------------------------------------------------------------------- */
/* Spectral step: B = diag(nu) (counts / N)[:, Gamma_1] diag(sigma_1)^{-1/2} = U diag(s) V^T      */
/* ------------------------------------------------------------------------------------------- */
typedef struct wos_svd_t wos_svd_t;

/* Allocates the device workspace of an SVD of an n_obs x n_elem count matrix.  gamma1_mask_host
 * (uint8[n_elem], 1 = Gamma_1), sigma_host (double[n_elem]) and nu_host (double[n_obs] or NULL
 * for 1/sqrt(n_obs)) are copied.  Sizes: m = n_obs, n = |Gamma_1|, k = min(m, n). */
wos_status wos_svd_create(wos_ctx *ctx, int32_t n_obs, int32_t n_elem,
                          const uint8_t *gamma1_mask_host, const double *sigma_host,
                          const double *nu_host, wos_svd_t **out);
wos_status wos_svd_destroy(wos_ctx *ctx, wos_svd_t *h);

/* Assembles B from counts_dev (n_walks walks per row) and computes its thin SVD in FP64 on the
 * device (paper eq. "SVD").  Results stay in the handle:
 *   U: double[m * k] column-major, s: double[k] descending, V: double[n * k] column-major.
 * s^2 are the eigenvalues of Lambda^nu = B B^T (the spectrum the paper studies).
 * Method: with A = B (or B^T when m < n) and c = min(m, n) <= 2048, first the Gram path:
 * G = A^T A, a factor X with X X^T = G (c <= 192: pivoted elimination in one workgroup; wider: a
 * blocked Cholesky factorisation with diagonal pivoting), one-sided Jacobi on X (right vectors and
 * s; c > 192: spread over the device, which needs c / 16 (rounded up to a multiple of 4) resident
 * workgroups of 256 threads on the stream's CUs, else the Gram path is skipped, and followed by a
 * first-order correction of the right vectors), left vectors u_j = A v_j / s_j.  Its result is kept
 * only if the left vectors pass the check max_ij |u_i.u_j - delta_ij| s_i s_j <= max(2^-40,
 * 16 c' 2^-52) s_1^2 (c' = c rounded up to 64), every s_j is positive and the residual certificate
 * |A^T u_j - s_j v_j| + s_j | |u_j|^2 - 1 | <= 2^-35 s_1 holds for every j (it bounds the distance
 * from s_j to a singular value of A); otherwise (and for c > 2048) one-sided Jacobi (Hestenes) on
 * A itself computes the result. */
wos_status wos_svd(wos_ctx *ctx, wos_svd_t *h, const uint32_t *counts_dev, uint64_t n_walks,
                   void *stream);
/* Device pointers and sizes of the factors (valid until the handle is destroyed). */
wos_status wos_svd_factors(const wos_svd_t *h, const double **U_dev, const double **s_dev,
                           const double **V_dev, int32_t *m, int32_t *n, int32_t *k);
typedef enum { WOS_SVD_HESTENES = 0, WOS_SVD_GRAM = 1 } wos_svd_method;
/* Of the last completed wos_svd: Jacobi sweeps and error flags (0 = converged; 1 grid barrier time-
 * out, 2 sweep limit) of the method whose result the handle holds, and that method (any of the
 * out-pointers may be NULL).  Synchronises `stream`. */
wos_status wos_svd_info(const wos_svd_t *h, int32_t *sweeps, int32_t *error_flag, int32_t *method,
                        void *stream);
/* Diagnostics of the Gram path of the last completed wos_svd: its Jacobi sweeps and error flags
 * (as in wos_svd_info; both 0 when the path did not run), its orthogonality statistic
 * max_ij |u_i.u_j - delta_ij| s_i s_j / s_1^2 and its residual certificate
 * max_j |A^T u_j - s_j v_j| + s_j | |u_j|^2 - 1 | (absolute).  Any out-pointer may be NULL.
 * Synchronises `stream`. */
wos_status wos_svd_gram_check(const wos_svd_t *h, int32_t *gram_sweeps, int32_t *gram_error_flag,
                              double *check, double *residual, void *stream);
/* Device time of the last wos_svd called outside stream capture (HIP events on its stream): the
 * Gram path's Jacobi kernel (0 if it did not run) and the whole call, in milliseconds, and the
 * plane rotations the device-wide Jacobi applied (0 for the one-workgroup Jacobi).  Waits for that
 * call to finish.  WOS_EINVAL if no such call has run on the handle. */
wos_status wos_svd_timing(const wos_svd_t *h, float *jacobi_ms, float *total_ms, uint64_t *rotations);

/* ------------------------------------------------------------------------------------------- */
/* Reconstruction (Algorithm Main)                                                               */
/* ------------------------------------------------------------------------------------------- */
typedef enum { WOS_TSVD_RANK = 0, WOS_TSVD_DISCREPANCY = 1, WOS_TIKHONOV = 2 } wos_reg;

typedef struct {
    int32_t kind;        /* wos_reg */
    int32_t rank;        /* WOS_TSVD_RANK: truncation r (clamped to the numerical rank) */
    double alpha;        /* WOS_TIKHONOV: alpha > 0, or 0 to choose it by the discrepancy rule */
    double noise_delta;  /* discrepancy rules: expected |nu * noise(b)| */
    double tau;          /* discrepancy rules: safety factor (e.g. 1.1) */
} wos_reg_params;

/* With q = diag(nu) (uD - (counts/N)[:, Gamma_0] u0) and the factors of h:
 *   u1 = diag(sigma_1)^{-1/2} V diag(phi) U^T q,  phi_i = 1/s_i (i <= r, TSVD) or
 *        s_i / (s_i^2 + alpha^2) (Tikhonov),
 *   pred = (counts/N)[:, Gamma_1] u1 + (counts/N)[:, Gamma_0] u0   (data predicted at x^D).
 * Discrepancy rules: r = smallest r with |q - B w_r| <= tau delta; alpha solves
 * |q - B w_alpha| = tau delta.  uD_dev: double[m]; u0_dev: double[|Gamma_0|] in cell order (may be
 * NULL when Gamma_0 is empty); u1_dev: double[n]; pred_dev (optional): double[m];
 * rank_used_dev (optional, int32), alpha_used_dev (optional, double). */
wos_status wos_reconstruct(wos_ctx *ctx, const wos_svd_t *h, const uint32_t *counts_dev,
                           uint64_t n_walks, const double *uD_dev, const double *u0_dev,
                           const wos_reg_params *reg, double *u1_dev, double *pred_dev,
                           int32_t *rank_used_dev, double *alpha_used_dev, void *stream);

/* ------------------------------------------------------------------------------------------- */
/* Products of the estimated measure (Section 5.2, items (i)-(iv))                               */
/* ------------------------------------------------------------------------------------------- */
/* The truncation sweep of Section 5.2, items (iii) and (iv): for every r = 1..r_max the r-TSVD
 * solution (eq. u1r with the same numerical-rank rule as wos_reconstruct), the data it predicts at
 * the points and the residual norm:
 *   u1_dev[(r-1) n + j]   = (diag(sigma_1)^{-1/2} V_r S_r^{-1} U_r^T q)_j      (n x r_max, column-major),
 *   pred_dev[(r-1) m + i] = ((counts/N)[:, Gamma_1] u1^(r) + (counts/N)[:, Gamma_0] u0)_i, formed as
 *                           (counts/N)[:, Gamma_0] u0 + (U_r U_r^T q)_i / nu_i  (m x r_max; optional),
 *   resid_dev[r]          = |q - B w_r| for r = 0..r_max (r_max + 1 values; optional),
 * with q = diag(nu) (uD - (counts/N)[:, Gamma_0] u0).  Column r - 1 of u1 equals wos_reconstruct with
 * WOS_TSVD_RANK and rank r bit for bit.  1 <= r_max <= k (the triplets the handle holds); pred needs
 * every nu_i != 0.  Uses the handle's work matrix as scratch (the factors stay valid).  Arguments
 * as for wos_reconstruct; asynchronous on `stream`. */
wos_status wos_reconstruct_sweep(wos_ctx *ctx, const wos_svd_t *h, const uint32_t *counts_dev,
                                 uint64_t n_walks, const double *uD_dev, const double *u0_dev,
                                 int32_t r_max, double *u1_dev, double *pred_dev, double *resid_dev,
                                 void *stream);

/* Eigenvalues of Lambda^nu (eq. Lambda_tilde_nu), lambda_f = s_f^2, and the eigenfunction estimators
 * of eq. eigenfunctions_MC on the Gamma_1 cells, for f = 0..n_fun-1:
 *   ef_dev[f n + l] = lambda_f^{-1/2} sum_i nu_i [u_f]_i rho_i(l) = V[l, f] / sqrt(sigma_l),
 * u_f the f-th left singular vector of B (an orthonormal eigenvector of Lambda^nu); the right-hand
 * form is the one evaluated.  Each estimator is orthonormal in L^2(Gamma_1) (sum_l sigma_l ef_f ef_g
 * = delta_fg); its sign is that of the handle's singular pair.  Meaningful for s_f above the
 * numerical rank.  0 <= n_fun <= k; lambda_dev: double[n_fun] (optional), ef_dev: double[n x n_fun]
 * (optional), device.  Asynchronous on `stream`. */
wos_status wos_eigenfunctions(wos_ctx *ctx, const wos_svd_t *h, int32_t n_fun, double *lambda_dev,
                              double *ef_dev, void *stream);

/* Density estimator of the elliptic measure on every boundary cell (eq. rho omega1 MC with the
 * cells as weight functions, Section 5.2 item (i)) and its average over the points:
 *   rho_dev[i n_elem + j] = (counts[i n_elem + j] / n_walks) / sigma_j   (n_obs x n_elem, row-major),
 *   mean_dev[j]           = (1 / n_obs) sum_i rho[i, j].
 * sigma_dev: double[n_elem] cell measures (device); either output may be NULL, not both.  Needs no
 * SVD.  Asynchronous on `stream`. */
wos_status wos_density(wos_ctx *ctx, const uint32_t *counts_dev, int32_t n_obs, int32_t n_elem,
                       uint64_t n_walks, const double *sigma_dev, double *rho_dev, double *mean_dev,
                       void *stream);

/* ------------------------------------------------------------------------------------------- */
/* Captured pipeline: the whole path of one instance as one HIP graph                            */
/* ------------------------------------------------------------------------------------------- */
typedef struct wos_plan wos_plan;

/* Records zero-fill of counts, the walk kernel(s), the SVD and the reconstruction of one
 * instance into a HIP graph.  All pointers are captured and must stay valid while the plan
 * lives; svd and the reconstruction arguments may be NULL for a measure-only plan. */
wos_status wos_plan_create(wos_ctx *ctx, const wos_measure_job *job, wos_svd_t *svd,
                           const double *uD_dev, const double *u0_dev, const wos_reg_params *reg,
                           double *u1_dev, double *pred_dev, int32_t *rank_used_dev,
                           double *alpha_used_dev, wos_plan **out);
/* Records a batch of measure jobs (as wos_build_measure_batch: one persistent walk launch per
 * (precision, dimension) group, mixed kinds and conductivities inside a group; eq. "H_MC" of §4.2
 * for each instance) into a HIP graph: zero-fill of every job's counts and statistics, then the
 * launches.  The jobs' device pointers are captured and must stay valid while the plan lives; each
 * launch of the plan recomputes the counts from zero.  The launch shapes are those of the tuning in
 * force at creation (wos_set_tuning / wos_autotune).  Errors: WOS_EINVAL for an empty batch or an
 * invalid job (nothing is recorded), WOS_ENOMEM, WOS_EDEVICE. */
wos_status wos_plan_create_batch(wos_ctx *ctx, const wos_measure_job *jobs, int32_t n_jobs, wos_plan **out);
wos_status wos_plan_launch(wos_plan *plan, void *stream);
wos_status wos_plan_destroy(wos_plan *plan);

/* ------------------------------------------------------------------------------------------- */
/* Serving: continuous batching of build + SVD + reconstruct requests                            */
/* ------------------------------------------------------------------------------------------- */
typedef struct {
    wos_geometry geom;
    wos_walk_params walk;          /* walk_begin/walk_end: the walk budget N = end - begin */
    const double *x_obs_host;      /* double[n_obs * dim] */
    int32_t n_obs;
    const uint8_t *gamma1_mask_host;
    const double *uD_host;         /* double[n_obs] */
    const double *u0_host;         /* double[|Gamma_0|] */
    wos_reg_params reg;
    double arrival_s;              /* offset from the start of wos_serve (open-loop replay) */
} wos_request;

typedef struct {
    double *u1_host;               /* caller-allocated double[|Gamma_1|] */
    double *pred_host;             /* caller-allocated double[n_obs] or NULL */
    double *s_host;                /* caller-allocated double[min(n_obs, |Gamma_1|)] or NULL */
    int32_t rank_used;
    double alpha_used;
    int32_t status;                /* wos_status of this request */
    double t_arrive, t_admit, t_done;  /* seconds since the start of wos_serve */
    uint64_t walks, steps;
    int32_t svd_fallback;          /* 1: svd_mode 2 could not serve the request from its trusted
                                    * triplets, so it was served by the full SVD (walks run again) */
} wos_result;

typedef struct {
    size_t hbm_budget_bytes;       /* admission bound on the device memory of in-flight requests */
    int32_t max_inflight;          /* concurrent requests on the device (streams) */
    double timeout_s;              /* per request, from arrival; 0 = none */
    int32_t svd_mode;              /* 0: full SVD of each request (the cooperative Jacobi kernels
                                    * of wos_svd, which run one at a time on the device);
                                    * 1: truncated SVD from plain kernels, so requests overlap:
                                    * the leading min(k, kt) triplets, kt = 64 when min(m, n) <= 64
                                    * else 128 (a random range sketch of kt columns first when
                                    * min(m, n) > kt); components below 1e-5 s_1 are not used by
                                    * the reconstruction, and s_host receives min(k, kt) values
                                    * followed by zeros.
                                    * 2: as 1, certified: only the leading triplets whose residual
                                    * |A v - s u| is at most 2^-35 s_1 (the full SVD's bound) are
                                    * used; a TSVD rank (given, or chosen by the discrepancy rule)
                                    * that needs more sends the request to the full SVD
                                    * (svd_fallback = 1), so every result has the full SVD's
                                    * accuracy.  Tikhonov requests use every triplet kept. */
} wos_serve_opts;

/* Blocking driver: replays the requests at their arrival times (open loop), admits each when a
 * slot and enough HBM budget are free, runs admitted requests concurrently on separate streams
 * (their walk kernels overlap on the device), and fills results[i].  Returns WOS_OK if the loop
 * ran; per-request status is in results[i].status. */
wos_status wos_serve(wos_ctx *ctx, const wos_request *reqs, int32_t n, wos_result *results,
                     const wos_serve_opts *opts);

/* Live form of the same engine: a serving thread owned by the context.
 *   wos_serve_start  starts it with the given options (WOS_EBUSY if one is running);
 *   wos_serve_submit validates a request, copies its host inputs (the caller may reuse them at
 *                    once; arrival_s is ignored, the arrival is the submission time) and returns
 *                    a ticket;
 *   wos_serve_poll   waits up to wait_ms (0: no wait, < 0: until done) for the ticket; when done
 *                    it copies u1 / pred / s into the buffers out points to (u1_host is required,
 *                    pred_host and s_host may be NULL), fills the rest of *out, releases the
 *                    ticket and returns WOS_OK (the request's own status is out->status);
 *                    WOS_EBUSY if still running, WOS_EINVAL for an unknown ticket;
 *   wos_serve_stop   finishes the requests in flight, then stops the thread (wos_destroy does
 *                    this too).  Tickets not polled are released.
 * These four entry points may be called from any host thread. */
wos_status wos_serve_start(wos_ctx *ctx, const wos_serve_opts *opts);
wos_status wos_serve_submit(wos_ctx *ctx, const wos_request *req, uint64_t *ticket);
wos_status wos_serve_poll(wos_ctx *ctx, uint64_t ticket, wos_result *out, int32_t wait_ms);
wos_status wos_serve_stop(wos_ctx *ctx);

/* ------------------------------------------------------------------------------------------- */
/* Diagnostics                                                                                    */
/* ------------------------------------------------------------------------------------------- */
/* The hardware sine and cosine (arguments in revolutions: cos(2 pi x), sin(2 pi x)) that the FP32
 * walk directions use (§4.2 eq. "wos chain": the uniform direction U), evaluated on the inputs they
 * take: cos_dev[i], sin_dev[i] at x_i = fma(i, 2^-24, offset) rounded once to FP32, i < n.  The
 * FP32 step's radius shrink assumes each within 2^-20 of the exact value; this lets a test check
 * that on every input.  cos_dev and sin_dev are device float[n] owned by the caller; n <= 2^24
 * (else WOS_EINVAL); enqueued on `stream`. */
wos_status wos_diag_trig32(float offset, uint32_t n, float *cos_dev, float *sin_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WOS_H */
