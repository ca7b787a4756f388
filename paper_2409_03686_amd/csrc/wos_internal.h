// wos_internal.h -- declarations shared by the libwos host runtime and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wos_device.hpp"

namespace wos {

constexpr int kMaxSweeps = 60;

// View of an SVD workspace passed by value to the linear-algebra kernels.
// Largest column count (after transposing wide blocks) of the one-workgroup Gram path: its
// factorisation keeps the whole Gram matrix in the registers of one 1024-thread workgroup.
constexpr int kGramMaxCols = 192;
// Largest column count of the device-wide Gram path (blocked Cholesky factor, Jacobi with the
// factor's rows in the registers of 256-thread workgroups, at most 8 rows per thread).
constexpr int kGramGridMaxCols = 2048;
// Round flags of the device-wide Jacobi (one per workgroup: kGramGridMaxCols / 16 workgroups).
constexpr int kGridFlags = 128;
// Control words of the device-wide Jacobi: flags, rotations and large rotations per sweep, a grid
// barrier counter and an error word.
constexpr int kGridCtlWords = kGridFlags + 2 * kMaxSweeps + 2;

// Control words of an SVD (device, zeroed by the assemble kernel).
enum SvdCtrl : int {
    kCtrlBarrier = 0,    // grid barrier counter, Hestenes path
    kCtrlError = 1,      // barrier time-out, Hestenes path
    kCtrlGramOk = 2,     // 1: the Gram path's result was accepted, the Hestenes path is skipped
    kCtrlTrusted = 3,    // truncated path: leading triplets whose residual certificate holds
    kCtrlUnresolved = 4, // truncated path: the regularisation needs triplets beyond the trusted ones
    kCtrlWords = 8
};
// info words: [0] sweeps, [1] error flags of the result returned; [2], [3] the same for the
// Gram path's Jacobi stage; [4] 1 if the result came from the Gram path.
constexpr int kInfoWords = 8;

struct SvdDevView {
    int m, n, k;            // B is m x n (m = points, n = |Gamma_1|), k = min(m, n)
    int rows, cols, colsp;  // work matrix A (rows x colsp, column-major): B, or B^T when m < n
    int trans;
    int n_elem, n0;         // cells of the count matrix, |Gamma_0|
    double tol;             // Jacobi rotation threshold on |a_p.a_q| / (|a_p| |a_q|)
    double *A, *W;          // work matrix, accumulated rotations (colsp x colsp)
    double *s, *U, *V;      // outputs
    double *nu, *isig1;     // nu (m), sigma_1^{-1/2} (n)
    int32_t *g1idx, *g0idx; // Gamma_1 / Gamma_0 cell indices
    int32_t *emap;          // cell -> Gamma_1 index (>= 0) or -(Gamma_0 index) - 1
    double *work;           // cols + 1
    double *q, *cvec, *phic;
    uint32_t *rot;          // rotations per sweep: [0, kMaxSweeps) Hestenes, [kMaxSweeps, 2 kMaxSweeps) Gram
    uint32_t *ctrl;         // SvdCtrl words
    int32_t *info;          // kInfoWords
    // Gram path (np = 0: not used for this shape)
    int np;                 // order of the padded Gram matrix, a multiple of 64, >= cols
    double *G;              // np x np Gram matrix A^T A
    double *L;              // np x np factor X with X X^T = G, then its Jacobi-rotated columns
    double *zs;             // np column norms of the rotated factor
    double *gnrm;           // np squared norms in flight (device-wide Jacobi; null otherwise)
    uint32_t *gctl;         // kGridCtlWords control words (device-wide Jacobi; null otherwise)
    int32_t *gpiv;          // 3 np row states of the pivoted blocked Cholesky, then 1024 words of candidates
    unsigned long long *crit;  // [0] orthogonality check, [1] residual certificate (bit patterns)
    // Truncated path (serving; tk = 0: not used): the kt leading singular triplets from a range
    // sketch of kt columns (cols > kt) or from the Gram path of A itself (cols <= kt), with
    // single-workgroup kernels only.
    int tk;                 // kt, a multiple of 64 (at most 128)
    int certified;          // 1: certify each triplet; the rank may use only the trusted ones
    double rank_cut;        // components with s <= rank_cut s_1 are left out of reconstructions
    double *Om, *Y, *Q;     // cols x kt sketch, rows x kt range, rows x kt orthonormal basis
    double *Cm, *Gt, *Lt, *zt;  // kt x cols projection, kt x kt Gram and factor, kt norms
    int32_t *perm;          // kt: factor column of each rank
};

struct RegDev {
    int kind, rank;
    double alpha, delta, tau;
};

// Walk launch modes: who owns the work.  0: a block owns an item (point, walk range); 1: a wave owns
// an item and overlaps it with its next one (two histogram rows, the segments and a stop queue per
// wave in LDS); 2: a block owns a point and reserves its walks chunk by chunk from the point's walk
// cursor, blocks that run out of points join points with walks left.
size_t walk_lds_bytes(int precision, int dim, int block, int hist_words, int seg_bytes, int mode);
// 32-bit words of the launch's cursors (zeroed by launch_walks): the item / point cursor, a spare
// word, and in point mode one walk cursor per point.
size_t walk_cursor_words(int mode, uint64_t total_items);
// kind_sel: the domain kind shared by all instances of the launch (plus kRadiusVariant when they all
// use the mapped-bound radius), or -1 when they differ
const void *walk_kernel_ptr(int precision, int dim, int kind_sel, int mode);
hipError_t launch_walks(int precision, int dim, int kind_sel, int mode, const DevInst *insts, int n_inst,
                        uint64_t total_items, uint32_t *cursor, int hist_words, int seg_bytes, int block, int grid,
                        hipStream_t stream);

// Events recorded around the Gram path's Jacobi kernel and around the whole SVD (eager calls only).
struct SvdEvents {
    hipEvent_t jac0, jac1, all0, all1;
    bool jac_recorded;  // set by svd_launch when the Jacobi ran between jac0 and jac1
};
// n_cu: CUs the stream may use (cooperative grids are sized for them); ev: null, or events to record
hipError_t svd_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, int coop_grid, int n_cu,
                      hipStream_t stream, SvdEvents *ev = nullptr);
int svd_coop_grid(int rows, int colsp, int n_cu);
int gram_order(int cols);  // np of the Gram path for this column count, 0 if it does not apply
// truncated SVD of the assembled work matrix (serving): non-cooperative kernels only
hipError_t tsvd_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, uint64_t seed,
                       hipStream_t stream);
constexpr int kTruncRank = 128;
hipError_t recon_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, const double *uD,
                        const double *u0, const RegDev &reg, double *u1, double *pred, int32_t *rank_out,
                        double *alpha_out, hipStream_t stream);
hipError_t density_launch(const uint32_t *counts, int m, int n_elem, uint64_t n_walks, const double *sigma,
                          double *rho, double *mean, hipStream_t stream);
hipError_t eigfun_launch(const SvdDevView &v, int n_fun, double *lam, double *ef, hipStream_t stream);
size_t sweep_part_words(const SvdDevView &v, int r_max);  // doubles of residual partials (in v.A)
hipError_t sweep_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, const double *uD,
                        const double *u0, int r_max, double *u1, double *pred, double *resid, hipStream_t stream);
hipError_t fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t stream);

}  // namespace wos
