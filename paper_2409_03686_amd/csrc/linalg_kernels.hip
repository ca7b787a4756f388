// linalg_kernels.hip -- FP64 spectral end of the path on gfx950.
//
//   assemble:    B = diag(nu) (counts / N)[:, Gamma_1] diag(sigma_1)^{-1/2}  (column-major work copy,
//                B^T when there are fewer points than Gamma_1 cells, so the work matrix is tall)
//   Gram path:   G = A^T A on MFMA, a factor X with X X^T = G, one-sided Jacobi on X, U = A V / s on
//                MFMA, an a-posteriori check (the default path; up to 2048 columns):
//                  <= 192 columns: pivoted elimination and Jacobi each in one workgroup;
//                  wider: blocked Cholesky (MFMA trailing updates) and a Jacobi over the device
//                  with the factor's rows in registers and blocks passed between workgroups.
//   Hestenes:    one-sided Jacobi on A itself with accumulated rotations, all column pairs of a
//                round in parallel, a cooperative grid with a device-wide barrier between rounds
//                (runs when the Gram result is rejected or the block is wider than 2048 columns)
//   truncated:   the leading singular triplets from a range sketch (serving), plain kernels only
//   reconstruct: q = nu (u^D - H_0 u^0), c = U^T q, filter factors phi (TSVD rank, discrepancy rule
//                or Tikhonov), u_1 = sigma^{-1/2} V (phi c), predicted data H_1 u_1 + H_0 u^0.
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>

#include "wos_internal.h"

namespace wos {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the block (blockDim a multiple of 64, at most 1024); every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double *scratch)
{
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += scratch[i];  // fixed order: deterministic
    return t;
}

__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *scratch)
{
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) {
        scratch[3 * w] = a;
        scratch[3 * w + 1] = b;
        scratch[3 * w + 2] = c;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0, tc = 0.0;
    for (int i = 0; i < nw; ++i) {
        ta += scratch[3 * i];
        tb += scratch[3 * i + 1];
        tc += scratch[3 * i + 2];
    }
    a = ta;
    b = tb;
    c = tc;
}

// ---------------------------------------------------------------------------------------------
__global__ void assemble_kernel(SvdDevView v, const uint32_t *__restrict__ counts, double inv_n)
{
    const size_t total = static_cast<size_t>(v.rows) * v.colsp;
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int r = static_cast<int>(e % v.rows);
        const int c = static_cast<int>(e / v.rows);
        double val = 0.0;
        if (c < v.cols) {
            const int i = v.trans ? c : r;   // observation point
            const int l = v.trans ? r : c;   // Gamma_1 column
            val = v.nu[i] * (static_cast<double>(counts[static_cast<size_t>(i) * v.n_elem + v.g1idx[l]]) * inv_n)
                  * v.isig1[l];
        }
        v.A[e] = val;
    }
    const size_t wtot = v.tk ? 0 : static_cast<size_t>(v.colsp) * v.colsp;  // no W on the truncated path
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < wtot;
         e += static_cast<size_t>(gridDim.x) * blockDim.x)
        v.W[e] = (e % v.colsp) == (e / v.colsp) ? 1.0 : 0.0;
    if (blockIdx.x == 0) {  // rotation counters, control words, info, acceptance statistic
        for (int t = threadIdx.x; t < 2 * kMaxSweeps; t += blockDim.x) v.rot[t] = 0u;
        if (threadIdx.x < kCtrlWords) v.ctrl[threadIdx.x] = 0u;
        if (threadIdx.x < kInfoWords) v.info[threadIdx.x] = 0;
        if (threadIdx.x < 2) v.crit[threadIdx.x] = 0ull;
        if (v.gctl)
            for (int t = threadIdx.x; t < kGridCtlWords; t += blockDim.x) v.gctl[t] = 0u;
    }
}

// Device-wide barrier for a cooperative grid: arrival counter with a generation target and a
// bounded spin (an expired spin sets the error flag instead of hanging).  One release fence before
// the arrival and one acquire fence after the wait; the polls themselves are relaxed (an acquire
// load per poll would invalidate the L2 of the polling XCD every time).
__device__ __forceinline__ void grid_barrier(uint32_t *counter, uint32_t *err, uint32_t nblocks,
                                             uint32_t &gen)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        gen += 1;
        const uint32_t target = gen * nblocks;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(4);
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            if (++spins > (1u << 26)) {
                atomicExch(err, 1u);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Round-robin ("circle") ordering: in round t of n - 1 rounds, slot i of n / 2 pairs element a with
// element b; over a sweep every unordered pair meets exactly once.
__device__ __forceinline__ void pair_of(int t, int i, int n, int &p, int &q)
{
    const int m1 = n - 1;
    const int a = i == 0 ? 0 : ((i - 1 + t) % m1) + 1;
    const int b = ((n - 2 - i + t) % m1) + 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// Pair K of round IR of the circle ordering of N elements, as compile-time constants.
template <int N, int IR, int K> struct PairC {
    static constexpr int a = K == 0 ? 0 : ((K - 1 + IR) % (N - 1)) + 1;
    static constexpr int b = ((N - 2 - K + IR) % (N - 1)) + 1;
    static constexpr int p = a < b ? a : b;
    static constexpr int q = a < b ? b : a;
};

template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// DPP move of a double (both 32-bit halves); lanes outside row_mask receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes with VALU data movement only: quad permutes, half-row and row mirrors,
// then row broadcasts 15 and 31 accumulate rows into row 3; lane 63 holds the totals.  The NV
// reductions advance step by step together, so their DPP latencies overlap.
template <int NV>
__device__ __forceinline__ void wave_totals(double (&v)[NV])
{
    static_for<0, NV>([&](auto e) { v[e] += dpp64<0xB1>(v[e]); });        // quad_perm (1, 0, 3, 2)
    static_for<0, NV>([&](auto e) { v[e] += dpp64<0x4E>(v[e]); });        // quad_perm (2, 3, 0, 1)
    static_for<0, NV>([&](auto e) { v[e] += dpp64<0x141>(v[e]); });       // row_half_mirror
    static_for<0, NV>([&](auto e) { v[e] += dpp64<0x140>(v[e]); });       // row_mirror
    static_for<0, NV>([&](auto e) { v[e] += dpp64<0x142, 0xA>(v[e]); });  // row_bcast15 into rows 1, 3
    static_for<0, NV>([&](auto e) { v[e] += dpp64<0x143, 0xC>(v[e]); });  // row_bcast31 into rows 2, 3
    static_for<0, NV>([&](auto e) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v[e]), 63);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v[e]), 63);
        v[e] = __hiloint2double(hi, lo);
    });
}

// Maximum over the 64 lanes of non-negative doubles (which order as their bit patterns), with the
// same DPP steps as wave_totals; lanes outside a step's row mask contribute 0.
__device__ __forceinline__ double wave_max_pos(double v)
{
    v = __builtin_fmax(v, dpp64<0xB1>(v));
    v = __builtin_fmax(v, dpp64<0x4E>(v));
    v = __builtin_fmax(v, dpp64<0x141>(v));
    v = __builtin_fmax(v, dpp64<0x140>(v));
    v = __builtin_fmax(v, dpp64<0x142, 0xA>(v));
    v = __builtin_fmax(v, dpp64<0x143, 0xC>(v));
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// FP64 inverse square root: the hardware estimate refined by two Newton steps (each step squares
// the relative error of the estimate).
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-x * y, y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-x * y, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

// One Newton step on the hardware estimates: enough where only the rotation angle depends on the
// value (any angle near the optimal one reduces the off-diagonal; the test uses fresh products).
__device__ __forceinline__ double rcp64_1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsq64_1(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
}

// Plane rotation that zeroes g = x_p . x_q for the squared norms a = |x_p|^2, b = |x_q|^2
// (Rutishauser's form): zeta = (b - a) / 2g, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = c t.  zeta and t only choose the angle and take one Newton step
// each; |zeta| is capped at 2^500 (the angle is below rounding long before, and zeta^2 must not
// overflow).  c comes from a twice-refined inverse square root, so c^2 + s^2 = 1 to a few ulps,
// which keeps the rotation orthogonal.  Requires g != 0.
__device__ __forceinline__ void rot_params(double a, double b, double g, double &c, double &s, double &t)
{
    const double zeta = (b - a) * rcp64_1(2.0 * g);
    const double az = __builtin_fmin(__builtin_fabs(zeta), 0x1.0p500);
    const double z2 = __builtin_fma(az, az, 1.0);
    const double tt = rcp64_1(__builtin_fma(z2, rsq64_1(z2), az));
    t = zeta >= 0.0 ? tt : -tt;
    c = rsq64(__builtin_fma(t, t, 1.0));
    s = c * t;
}

// Sums NV per-wave values over the NW waves of the block: lane 0 of each wave writes its totals,
// one barrier, then every thread adds the wave totals in a fixed order (identical in all waves).
template <int NV, int NW>
__device__ __forceinline__ void block_totals(double (&val)[NV], double (*buf)[16])
{
    wave_totals<NV>(val);
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) static_for<0, NV>([&](auto e) { buf[wid][e] = val[e]; });
        __syncthreads();
        static_for<0, NV>([&](auto e) {
            double acc = 0.0;
            for (int w2 = 0; w2 < NW; ++w2) acc += buf[w2][e];
            val[e] = acc;
        });
    }
}

// One round IR of the cyclic sweep over the N columns held in registers: the N/2 dot products
// g = x_p . x_q of disjoint pairs (their reductions interleaved), block totals, then for each pair
// with g^2 > tol^2 |x_p|^2 |x_q|^2 the rotation parameters from the tracked norms and two-term
// updates of the rows of the work matrix (and of the accumulated rotations when RW > 0).  The
// decisions are uniform, so a pair that is already orthogonal costs only its dot product.
template <int N, int IR, int R, int RW, int NW>
__device__ __forceinline__ void inner_round(double (&x)[R][N], double (&w)[RW > 0 ? RW : 1][N], double (&n2)[N],
                                            double (*part)[16][16], int &nrot, double tol2)
{
    constexpr int NPR = N / 2;
    double g[NPR];
    static_for<0, NPR>([&](auto kk) {
        constexpr int p = PairC<N, IR, decltype(kk)::value>::p, q = PairC<N, IR, decltype(kk)::value>::q;
        double sg = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) sg = __builtin_fma(x[i][p], x[i][q], sg);
        g[kk] = sg;
    });
    block_totals<NPR, NW>(g, part[IR & 1]);
    static_for<0, NPR>([&](auto kk) {
        constexpr int p = PairC<N, IR, decltype(kk)::value>::p, q = PairC<N, IR, decltype(kk)::value>::q;
        const double a = n2[p], b = n2[q], gg = g[kk];
        if (gg != 0.0 && gg * gg > tol2 * a * b) {
            double c, sn, t;
            rot_params(a, b, gg, c, sn, t);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const double xp = x[i][p], xq = x[i][q];
                x[i][p] = c * xp - sn * xq;
                x[i][q] = sn * xp + c * xq;
            }
            if constexpr (RW > 0) {
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const double wp = w[i][p], wq = w[i][q];
                    w[i][p] = c * wp - sn * wq;
                    w[i][q] = sn * wp + c * wq;
                }
            }
            // column norms after the rotation that zeroes g (Hestenes): |x_p|^2 - t g, |x_q|^2 + t g
            n2[p] = a - t * gg;
            n2[q] = b + t * gg;
            ++nrot;
        }
    });
}

template <int N, int R, int RW, int NW, int... IR>
__device__ __forceinline__ void inner_sweep(double (&x)[R][N], double (&w)[RW > 0 ? RW : 1][N], double (&n2)[N],
                                            double (*part)[16][16], int &nrot, double tol2,
                                            std::integer_sequence<int, IR...>)
{
    (inner_round<N, IR, R, RW, NW>(x, w, n2, part, nrot, tol2), ...);
}

// Arguments of one blocked one-sided Jacobi run.
struct JacobiArgs {
    double *X;             // rows x colsp work matrix, column-major, leading dimension ldx
    double *W;             // colsp x colsp accumulated rotations (leading dimension colsp), or null
    int rows, ldx, colsp;
    double tol;            // rotate while g^2 > tol^2 |x_p|^2 |x_q|^2
    uint32_t *rot;         // kMaxSweeps rotation counters
    uint32_t *bar, *err;   // grid barrier counter, barrier time-out flag
    int32_t *info;         // [0] sweeps, [1] error flags (1 barrier time-out, 2 not converged)
    const uint32_t *skip;  // when non-null and *skip != 0 the kernel returns at once
};

// Blocked one-sided Jacobi (Hestenes) with register-resident block pairs.
//
// Columns are grouped in blocks of BW; the blocks meet pairwise in round-robin order, one block
// pair per group of T threads per round, with a device-wide barrier between rounds.  A group loads
// the 2 BW columns of its pair, rows of X and (if kept) rows of W alike, into registers (thread t
// of the group holds rows t, t + T, ...), computes their norms, then runs one cyclic sweep over
// them: in each of 2 BW - 1 rounds, BW disjoint pairs get g = x_p . x_q from a DPP (+ LDS when
// T > 64) reduction and a pair with g^2 > tol^2 |x_p|^2 |x_q|^2 is rotated by the plane rotation
// that zeroes g, applied as two-term updates to its rows; the norms follow the rotation
// analytically and are recomputed from the columns at the next load.  Fresh dot products and
// two-term updates keep small columns accurate relative to their own size.  All waves of a group
// compute the same sums in the same order, so they take the same decisions.  A sweep without
// rotations ends the iteration.  A workgroup holds GPB independent one-wave groups when T = 64
// (fewer workgroups meet at the barrier), or one group of T threads.
template <int R, int RW, int T, int BW, int GPB = 1>
__global__ __launch_bounds__(T *GPB) void jacobi_kernel(JacobiArgs J)
{
    static_assert(GPB == 1 || T == 64, "several groups per workgroup need one-wave groups");
    constexpr int N = 2 * BW;
    constexpr int NW = T / 64;
    __shared__ double part[2][16][16];
    __shared__ int cols_s[GPB][N];
    if (J.skip && *J.skip != 0u) return;  // uniform over the grid: written by an earlier kernel
    const int grp = GPB > 1 ? static_cast<int>(threadIdx.x) / T : 0;
    const int lt = GPB > 1 ? static_cast<int>(threadIdx.x) % T : static_cast<int>(threadIdx.x);
    int *cols = cols_s[grp];
    auto group_sync = [] {
        if constexpr (GPB == 1) __syncthreads();
        else __builtin_amdgcn_wave_barrier();
    };
    const int nblk = J.colsp / BW;
    const int npairs = nblk / 2;
    const int ld = J.ldx;
    const int ldw = J.colsp;
    const double tol2 = J.tol * J.tol;
    uint32_t gen = 0;
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        for (int t = 0; t < nblk - 1; ++t) {
            for (int pi = blockIdx.x * GPB + grp; pi < npairs; pi += gridDim.x * GPB) {
                int P, Qb;
                pair_of(t, pi, nblk, P, Qb);
                if (lt < N) cols[lt] = lt < BW ? P * BW + lt : Qb * BW + lt - BW;
                group_sync();
                double x[R][N], w[RW > 0 ? RW : 1][N];
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const double *ca = J.X + static_cast<size_t>(cols[j]) * ld;
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const int r = lt + i * T;
                        x[i][j] = r < J.rows ? ca[r] : 0.0;
                    }
                    if constexpr (RW > 0) {
                        const double *cw = J.W + static_cast<size_t>(cols[j]) * ldw;
#pragma unroll
                        for (int i = 0; i < RW; ++i) {
                            const int r = lt + i * T;
                            w[i][j] = r < ldw ? cw[r] : 0.0;
                        }
                    }
                }
                double n2[N];
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < R; ++i) acc = __builtin_fma(x[i][j], x[i][j], acc);
                    n2[j] = acc;
                }
                block_totals<N, NW>(n2, part[1]);
                int nrot = 0;
                inner_sweep<N, R, RW, NW>(x, w, n2, part, nrot, tol2, std::make_integer_sequence<int, N - 1>{});
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    double *ca = J.X + static_cast<size_t>(cols[j]) * ld;
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const int r = lt + i * T;
                        if (r < J.rows) ca[r] = x[i][j];
                    }
                    if constexpr (RW > 0) {
                        double *cw = J.W + static_cast<size_t>(cols[j]) * ldw;
#pragma unroll
                        for (int i = 0; i < RW; ++i) {
                            const int r = lt + i * T;
                            if (r < ldw) cw[r] = w[i][j];
                        }
                    }
                }
                if (lt == 0 && nrot) atomicAdd(&J.rot[sweep], static_cast<uint32_t>(nrot));
                group_sync();
            }
            grid_barrier(J.bar, J.err, gridDim.x, gen);
        }
        const uint32_t rotated = __hip_atomic_load(&J.rot[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t failed = __hip_atomic_load(J.err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (rotated == 0u || failed) {
            ++sweep;
            break;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.info[0] = sweep;
        J.info[1] = static_cast<int32_t>(__hip_atomic_load(J.err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) |
                    (sweep >= kMaxSweeps && J.rot[kMaxSweeps - 1] != 0u ? 2 : 0);
    }
}

// Launch shape by the size of the work matrix: T threads, R rows of X and RW rows of W each.
struct JacobiShape {
    const void *fn;
    int threads;  // per workgroup
    int bw;       // columns per block
    int gpb;      // block pairs per workgroup
};
#define WOS_BJ(R, RW, T) JacobiShape{reinterpret_cast<const void *>(&jacobi_kernel<R, RW, T, 4>), T, 4, 1}
static JacobiShape jacobi_shape(int rows, int colsp)
{
    // one workgroup per CU: 256 threads (one wave per SIMD, up to 512 VGPRs) with R rows each
    if (rows <= 256) return WOS_BJ(1, 1, 256);
    if (rows <= 1024) return colsp <= 256 ? WOS_BJ(4, 1, 256) : WOS_BJ(4, 4, 256);
    if (rows <= 2048) return colsp <= 512 ? WOS_BJ(8, 2, 256) : WOS_BJ(8, 8, 256);
    if (rows <= 4096) {
        if (colsp <= 1024) return WOS_BJ(16, 4, 256);
        if (colsp <= 2048) return WOS_BJ(16, 8, 256);
        return WOS_BJ(8, 8, 512);
    }
    if (rows <= 8192) return WOS_BJ(8, 8, 1024);
    return {nullptr, 0, 4, 1};
}
#undef WOS_BJ

// Column norms out[c] = |X[:, c]| for c < ncols (one block per column).
__global__ void colnorm_kernel(const double *__restrict__ X, int rows, int ld, int ncols, double *__restrict__ out,
                               const uint32_t *skip)
{
    __shared__ double scratch[16];
    if (skip && *skip != 0u) return;
    for (int c = blockIdx.x; c < ncols; c += gridDim.x) {
        const double *a = X + static_cast<size_t>(c) * ld;
        double acc = 0.0;
        for (int r = threadIdx.x; r < rows; r += blockDim.x) acc = __builtin_fma(a[r], a[r], acc);
        acc = block_sum(acc, scratch);
        if (threadIdx.x == 0) out[c] = __builtin_sqrt(acc);
        __syncthreads();
    }
}

__global__ void scatter_kernel(SvdDevView v, const uint32_t *skip)
{
    if (skip && *skip != 0u) return;
    for (int c = blockIdx.x; c < v.cols; c += gridDim.x) {
        const double sc = v.work[c];
        int rank = 0;
        for (int o = 0; o < v.cols; ++o) {
            const double so = v.work[o];
            rank += (so > sc || (so == sc && o < c)) ? 1 : 0;
        }
        if (threadIdx.x == 0) v.s[rank] = sc;
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        const double *a = v.A + static_cast<size_t>(c) * v.rows;
        const double *w = v.W + static_cast<size_t>(c) * v.colsp;
        if (!v.trans) {
            double *u = v.U + static_cast<size_t>(rank) * v.m;
            for (int r = threadIdx.x; r < v.m; r += blockDim.x) u[r] = a[r] * inv;
            double *vv = v.V + static_cast<size_t>(rank) * v.n;
            for (int r = threadIdx.x; r < v.n; r += blockDim.x) vv[r] = w[r];
        } else {
            double *u = v.U + static_cast<size_t>(rank) * v.m;
            for (int r = threadIdx.x; r < v.m; r += blockDim.x) u[r] = w[r];
            double *vv = v.V + static_cast<size_t>(rank) * v.n;
            for (int r = threadIdx.x; r < v.n; r += blockDim.x) vv[r] = a[r] * inv;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Gram path (cols <= kGramGridMaxCols)
//
//   G = A^T A (MFMA), a factor X with X X^T = G, one-sided Jacobi on X: X W = Z with orthogonal
//   columns, so G = Z Z^T and the right singular vectors of A are Z's columns over their norms s;
//   the left ones are A v / s (MFMA).  Up to kGramMaxCols columns the factor comes from an
//   outer-product elimination with diagonal pivoting and the Jacobi runs in one workgroup; wider
//   blocks take the device-wide kernels further down.  The result is accepted when (i) the computed
//   left vectors pass max_ij |u_i.u_j - delta_ij| s_i s_j <= max(2^-40, 16 np 2^-52) s_1^2 (so
//   V^T A^T A V = diag(s^2) holds to that level entrywise: a consistency check of the factor and the
//   iteration, whose stopping rule leaves cosines up to np 2^-52 between the columns) and (ii) the
//   residual certificate (gram_resid_kernel) bounds the error of every singular value by 2^-35 s_1;
//   otherwise the Hestenes path on A runs.  Rounding in G is proportional to the column norms it
//   combines, so singular values whose vectors are localised (small columns, as on Monte Carlo
//   blocks with s_min / s_1 = 1e-6) stay accurate to a few 1e-13 s_1, while values below ~sqrt(u) s_1
//   that arise from cancellation cannot be resolved from G at all: the certificate tells the two
//   apart.
// ---------------------------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

// One 16 x 16 tile of G = A^T A per wave: v_mfma_f64_16x16x4f64 over the rows, 4 at a time.
// Lane l supplies A-operand (i = l % 16, k = l / 16) and B-operand (k = l / 16, j = l % 16); it
// receives D[4 v + l / 16][l % 16] in accumulator element v.
__global__ __launch_bounds__(256) void gram_kernel(SvdDevView v)
{
    const int np = v.np, nt = np / 16;
    const int wave = static_cast<int>((blockIdx.x * 256u + threadIdx.x) >> 6);
    if (wave >= nt * nt) return;  // whole waves
    const int i0 = (wave % nt) * 16, j0 = (wave / nt) * 16;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const bool va = i0 + li < v.colsp, vb = j0 + li < v.colsp;
    const double *ca = v.A + static_cast<size_t>(va ? i0 + li : 0) * v.rows;
    const double *cb = v.A + static_cast<size_t>(vb ? j0 + li : 0) * v.rows;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < v.rows; r0 += 4) {
        const int r = r0 + lk;
        const double a = (va && r < v.rows) ? ca[r] : 0.0;
        const double b = (vb && r < v.rows) ? cb[r] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) v.G[static_cast<size_t>(j0 + li) * np + i0 + 4 * e + lk] = acc[e];
}

__device__ __forceinline__ double readlane64(double x, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Outer-product elimination with diagonal pivoting, G = sum_k l_k l_k^T: step k takes the column
// j of the remaining Schur complement with the largest diagonal d, l_k = S[:, j] / sqrt(d) (zero on
// eliminated rows), S -= l_k l_k^T.  One workgroup of 1024 threads; S stays in registers (wave w
// holds columns CPW w .. CPW w + CPW - 1, lane l rows l + 64 i); wave 0 keeps the diagonal and
// picks the pivots.  Stops when no diagonal exceeds np 2^-52 times the first pivot; the remaining
// columns of X are zero.
template <int RPL>
__global__ __launch_bounds__(1024) void gram_chol_kernel(SvdDevView v)
{
    constexpr int NPD = 64 * RPL, CPW = 4 * RPL;
    __shared__ double lcol[NPD];
    __shared__ double piv_d;
    __shared__ int piv_j;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double x[RPL][CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int i = 0; i < RPL; ++i) x[i][c] = v.G[static_cast<size_t>(w * CPW + c) * NPD + lane + 64 * i];
    uint32_t live_cols = (1u << CPW) - 1u;  // wave-uniform
    uint32_t live_rows = (1u << RPL) - 1u;  // per lane
    double dg[RPL];                          // wave 0: Schur diagonal of index lane + 64 i (-1: eliminated)
    auto pick = [&]() {
        double bv = -1.0;
        int bi = NPD;
#pragma unroll
        for (int i = 0; i < RPL; ++i)
            if (dg[i] > bv) {
                bv = dg[i];
                bi = lane + 64 * i;
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            piv_d = bv;
            piv_j = bi;
        }
    };
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int j = lane + 64 * i;
            dg[i] = v.G[static_cast<size_t>(j) * NPD + j];
        }
        pick();
    }
    __syncthreads();
    const double thresh = static_cast<double>(NPD) * 0x1.0p-52 * piv_d;
    int k = 0;
    for (; k < NPD; ++k) {
        const double d = piv_d;
        const int jp = piv_j;
        if (!(d > thresh) || jp >= NPD) break;  // uniform
        const int wp = jp / CPW, cp = jp - wp * CPW;
        if (w == wp) {
            const double inv = rsq64(d);
            static_for<0, CPW>([&](auto cc) {
                if (decltype(cc)::value == cp) {
#pragma unroll
                    for (int i = 0; i < RPL; ++i) {
                        const int r = lane + 64 * i;
                        const double val = ((live_rows >> i) & 1u) ? x[i][decltype(cc)::value] * inv : 0.0;
                        lcol[r] = val;
                        v.L[static_cast<size_t>(k) * NPD + r] = val;
                    }
                }
            });
            live_cols &= ~(1u << cp);
        }
        __syncthreads();
        if (lane == (jp & 63)) live_rows &= ~(1u << (jp >> 6));
        double lr[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) lr[i] = lcol[lane + 64 * i];
        static_for<0, CPW>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if (live_cols & (1u << c)) {
                const double lj = lcol[w * CPW + c];
#pragma unroll
                for (int i = 0; i < RPL; ++i) x[i][c] = __builtin_fma(-lr[i], lj, x[i][c]);
            }
        });
        if (w == 0) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int j = lane + 64 * i;
                dg[i] = j == jp ? -1.0 : (dg[i] < 0.0 ? dg[i] : __builtin_fma(-lr[i], lr[i], dg[i]));
            }
            pick();
        }
        __syncthreads();
    }
    for (size_t e = static_cast<size_t>(k) * NPD + threadIdx.x; e < static_cast<size_t>(NPD) * NPD; e += 1024)
        v.L[e] = 0.0;
}

// Singular values in descending order and the eigenvector side: one block per factor column c;
// s[rank] = zs[c], Vs[:, rank] = Z[:, c] / zs[c] (Vs = V, or U when the work matrix is B^T).
__global__ void gram_vside_kernel(SvdDevView v)
{
    double *vs = v.trans ? v.U : v.V;
    for (int c = blockIdx.x; c < v.np; c += gridDim.x) {
        const double sc = v.zs[c];
        int rank = 0;
        for (int o = 0; o < v.np; ++o) {
            const double so = v.zs[o];
            rank += (so > sc || (so == sc && o < c)) ? 1 : 0;
        }
        if (rank >= v.k) continue;
        if (threadIdx.x == 0) v.s[rank] = sc;
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        for (int r = threadIdx.x; r < v.cols; r += blockDim.x)
            vs[static_cast<size_t>(rank) * v.cols + r] = v.L[static_cast<size_t>(c) * v.np + r] * inv;
    }
}

// The other side: Y = A Vs diag(1/s), rows x k, one 16 x 16 tile per wave (MFMA over the columns).
__global__ __launch_bounds__(256) void gram_yside_kernel(SvdDevView v)
{
    const double *vs = v.trans ? v.U : v.V;
    double *ys = v.trans ? v.V : v.U;
    const int tr = (v.rows + 15) / 16, tk = (v.k + 15) / 16;
    const int wave = static_cast<int>((blockIdx.x * 256u + threadIdx.x) >> 6);
    if (wave >= tr * tk) return;
    const int r0 = (wave % tr) * 16, l0 = (wave / tr) * 16;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int r = r0 + li, l = l0 + li;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < v.cols; c0 += 4) {
        const int c = c0 + lk;
        const double a = (r < v.rows && c < v.cols) ? v.A[static_cast<size_t>(c) * v.rows + r] : 0.0;
        const double b = (l < v.k && c < v.cols) ? vs[static_cast<size_t>(l) * v.cols + c] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (l < v.k) {
        const double sl = v.s[l];
        const double inv = sl > 0.0 ? 1.0 / sl : 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int rr = r0 + 4 * e + lk;
            if (rr < v.rows) ys[static_cast<size_t>(l) * v.rows + rr] = acc[e] * inv;
        }
    }
}

// Certificate of the singular values: with u_j = A v_j / s_j (so A v_j = s_j u_j exactly), the
// residual of the other side, e_j = |A^T u_j - s_j v_j| + s_j | |u_j|^2 - 1 |, bounds the distance
// from s_j to a singular value of A (the symmetric matrix [[0, A], [A^T, 0]] has the residual
// (0, A^T u - s v) / sqrt 2 at (u, v) / sqrt 2, after u is normalised).  C = A^T Ys (cols x k) is in
// Cm; one block per column j folds e_j into crit[1] (bit pattern, atomic max).
__global__ __launch_bounds__(256) void gram_resid_kernel(SvdDevView v, const double *__restrict__ Cm)
{
    __shared__ double scratch[16];
    const double *vs = v.trans ? v.U : v.V;
    const double *ys = v.trans ? v.V : v.U;
    for (int j = blockIdx.x; j < v.k; j += gridDim.x) {
        const double sj = v.s[j];
        double r2 = 0.0, u2 = 0.0;
        for (int i = threadIdx.x; i < v.cols; i += 256) {
            const double d = Cm[static_cast<size_t>(j) * v.cols + i] - sj * vs[static_cast<size_t>(j) * v.cols + i];
            r2 = __builtin_fma(d, d, r2);
        }
        for (int i = threadIdx.x; i < v.rows; i += 256) {
            const double y = ys[static_cast<size_t>(j) * v.rows + i];
            u2 = __builtin_fma(y, y, u2);
        }
        r2 = block_sum(r2, scratch);
        u2 = block_sum(u2, scratch);
        const double ej = __builtin_sqrt(r2) + sj * __builtin_fabs(u2 - 1.0);
        if (threadIdx.x == 0)
            atomicMax(v.crit + 1, static_cast<unsigned long long>(__double_as_longlong(ej != ej ? __builtin_inf() : ej)));
        __syncthreads();
    }
}

// Accepts the Gram path's result when the iteration ended without error, the left vectors pass the
// orthogonality check, every singular value is positive (a zero one would leave its eigenvector
// column empty: V = Z / s; the Hestenes path gives it a basis vector of the null space) and the
// residual certificate bounds every singular value's error by 2^-35 s_1.
__global__ void gram_accept_kernel(SvdDevView v)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double s0 = v.s[0], sk = v.s[v.k - 1];
    const double crit = __longlong_as_double(static_cast<long long>(v.crit[0]));
    const double resid = __longlong_as_double(static_cast<long long>(v.crit[1]));
    // the Jacobi leaves |z_p.z_q| <= np 2^-52 |z_p| |z_q|, so the check's floor grows with np
    const double limit = __builtin_fmax(0x1.0p-40, 16.0 * v.np * 0x1.0p-52);
    const bool ok = v.info[3] == 0 && s0 > 0.0 && sk > 0.0 && crit <= limit && resid <= 0x1.0p-35 * s0;
    v.ctrl[kCtrlGramOk] = ok ? 1u : 0u;
    if (ok) {
        v.info[0] = v.info[2];
        v.info[1] = 0;
        v.info[4] = 1;
    }
}

// First-order correction of the eigenvector side Vs (device-wide path).  The rotated factor's
// columns are orthogonal only up to cosines of np 2^-52 relative to their own norms, so
// F = Vs^T A^T A Vs - diag(s^2) = diag(s) (Ys^T Ys - I) diag(s) keeps entries of that size times
// s_i^2 + s_j^2, which for a large and a small singular value is large next to the small one's
// square (regularised solutions, which act like (A^T A + alpha^2)^{-1}, amplify it by
// (s_1 / alpha)^2).  Perturbation theory of the symmetric eigenproblem gives the correction
// Vs <- Vs (I + K), K_ij = F_ij / (s_j^2 - s_i^2), taken only where |F_ij| <= |s_j^2 - s_i^2| / 10 (a
// pair that close stays as it is; filters hardly tell its members apart).  C = Ys^T Ys is in Cm; the
// kernel writes I + K (k x k, column-major) to Km and clears the acceptance statistic for the
// check that follows the correction.
__global__ void gram_fix_kernel(SvdDevView v, const double *__restrict__ Cm, double *__restrict__ Km)
{
    const size_t kk = static_cast<size_t>(v.k) * v.k;
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < kk;
         e += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(e % v.k), j = static_cast<int>(e / v.k);
        double val = i == j ? 1.0 : 0.0;
        if (i != j) {
            const double si = v.s[i], sj = v.s[j];
            const double f = si * Cm[e] * sj;
            const double d2 = (sj - si) * (sj + si);
            if (d2 != 0.0 && __builtin_fabs(f) <= 0.1 * __builtin_fabs(d2)) val = f / d2;
        }
        Km[e] = val;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) v.crit[0] = 0ull;
}

__global__ void copy_f64_kernel(double *__restrict__ dst, const double *__restrict__ src, size_t n)
{
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * blockDim.x)
        dst[e] = src[e];
}

// ---------------------------------------------------------------------------------------------
// Truncated path (serving): the leading kt singular triplets with single-workgroup and plain
// kernels only, so that requests on different streams overlap on the device.
//   cols <= kt: the Gram path of A itself with the Jacobi of one workgroup (gram_jacobi1_kernel).
//   cols >  kt: a range sketch Y = A Om (Om a +-1 matrix from Philox) and an orthonormal basis
//               Q = Y E diag(1/lambda) from the eigenvectors E, eigenvalues lambda^2 of Y^T Y (Gram
//               path); one subspace iteration Y = A A^T Q, re-orthonormalised the same way
//               (without it the leading singular values come out only to ~1e-3 when the spectrum
//               has a Monte Carlo noise floor; with one the TSVD solutions stay within ~4e-5 of the
//               full SVD's, with two within ~1e-7 at one more one-workgroup Jacobi run per
//               request); then C = Q^T A, the Gram path of C^T, U = Q E_C, V = C^T E_C / s.
// Components with s <= rank_cut s_1 (1e-5) are left out of the reconstruction: below that the
// Gram path's squaring of the condition number makes them inaccurate.
// ---------------------------------------------------------------------------------------------

// ---------------------------------------------------------------------------------------------
// One-workgroup Jacobi of the Gram path's factor (np = 64 R <= 192 columns).
//
// X stays in registers: 32 blocks of BW = 2 R columns, wave w (of 16) holding block w ("top") and
// block 31 - w ("bottom"), lane l rows l + 64 i.  A sweep rotates the pairs inside each block, then
// lets the blocks meet in round-robin order (circle method: block 0 fixed, the other 31 move one
// position per round, so every two blocks meet once and the arrangement is back at the start after
// 31 rounds); a meeting sweeps the BW x BW cross pairs of the wave's two blocks in BW rounds of BW
// disjoint pairs.  Blocks move between waves through LDS (16 one-block slots).  In a round the BW
// dot products are reduced together (split_totals leaves pair j's total in lane j), lane j computes
// pair j's rotation from the tracked squared norms (LDS), and the rotations are applied with
// broadcast parameters.  Norms are recomputed from the columns at the start of every sweep.  No
// grid-wide synchronisation: the kernel runs beside other work on a few CUs.
// ---------------------------------------------------------------------------------------------

// x from lane (lane ^ M), M = 1, 2, 4, 8, 16, 32.
template <int M> __device__ __forceinline__ double xor_lane(double x)
{
    if constexpr (M == 1) return dpp64<0xB1>(x);        // quad_perm (1, 0, 3, 2)
    else if constexpr (M == 2) return dpp64<0x4E>(x);   // quad_perm (2, 3, 0, 1)
    else if constexpr (M == 8) return dpp64<0x128>(x);  // row_ror 8 within rows of 16
    else if constexpr (M == 32) {
        const int lo = __shfl_xor(__double2loint(x), 32), hi = __shfl_xor(__double2hiint(x), 32);
        return __hiloint2double(hi, lo);
    } else {  // 4, 16: swizzle in bit-mask mode within groups of 32 lanes, lane' = lane ^ M
        const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), 0x1F | (M << 10));
        const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), 0x1F | (M << 10));
        return __hiloint2double(hi, lo);
    }
}

// Wave sums of P values (P = 2, 4, 8); lane l receives the sum of value l % P.  Stage k halves the
// list: with b = bit k of the lane, a lane keeps the values whose index has bit k equal to b and
// adds its partner's (lane ^ 2^k) copies of them; the one value left is summed over the other
// lane bits.
template <int P> __device__ __forceinline__ double split_totals(double (&v)[P], int lane)
{
    static_for<0, (P == 2 ? 1 : (P == 4 ? 2 : 3))>([&](auto st) {
        constexpr int k = decltype(st)::value, M = 1 << k, N = P >> k;
        const bool b = (lane & M) != 0;
        static_for<0, N / 2>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const double keep = b ? v[2 * i + 1] : v[2 * i];
            const double send = b ? v[2 * i] : v[2 * i + 1];
            v[i] = keep + xor_lane<M>(send);
        });
    });
    double t = v[0];
    if constexpr (P <= 2) t += xor_lane<2>(t);
    if constexpr (P <= 4) t += xor_lane<4>(t);
    t += xor_lane<8>(t);
    t += xor_lane<16>(t);
    t += xor_lane<32>(t);
    return t;
}

// Pair J of round RI: CROSS = 0, the circle ordering inside the top block (J < BW / 2) or the
// bottom block; CROSS = 1, top column J with bottom column (J + RI) mod BW.
template <int BW, int CROSS, int RI, int J> struct WjPair {
    static constexpr int k = J < BW / 2 ? J : J - BW / 2;
    static constexpr int off = J < BW / 2 ? 0 : BW;
    static constexpr int p = CROSS ? J : PairC<BW, RI, k>::p + off;
    static constexpr int q = CROSS ? BW + (J + RI) % BW : PairC<BW, RI, k>::q + off;
};

template <int R, int CROSS, int RI>
__device__ __forceinline__ void wj_round(double (&x)[R][4 * R], double *nrm_w, int lane, uint32_t &nrot, double tol2,
                                         bool &big)
{
    constexpr int BW = 2 * R, P = BW <= 2 ? 2 : (BW <= 4 ? 4 : 8);
    double g[P];
    static_for<0, P>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        if constexpr (j < BW) {
            constexpr int p = WjPair<BW, CROSS, RI, j>::p, q = WjPair<BW, CROSS, RI, j>::q;
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < R; ++i) acc = __builtin_fma(x[i][p], x[i][q], acc);
            g[j] = acc;
        } else {
            g[j] = 0.0;
        }
    });
    const double gj = split_totals<P>(g, lane);
    double c = 1.0, sn = 0.0;
    bool act = false;
    // an opaque copy of the lane index: the per-round norm addresses are then formed in the round
    // instead of being hoisted out of the sweep loop for all rounds at once (registers)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    if (ln < BW) {
        int p, q;
        if constexpr (CROSS) {
            p = ln;
            q = BW + (ln + RI) % BW;
        } else {
            const int k = ln < BW / 2 ? ln : ln - BW / 2, off = ln < BW / 2 ? 0 : BW;
            pair_of(RI, k, BW, p, q);
            p += off;
            q += off;
        }
        const double a = nrm_w[p], b = nrm_w[q];
        act = gj != 0.0 && gj * gj > tol2 * a * b;
        if (act) {
            double t;
            big = big || gj * gj >= 1e-16 * (a * b);  // a rotated cosine of 1e-8 or more
            rot_params(a, b, gj, c, sn, t);
            nrm_w[p] = a - t * gj;
            nrm_w[q] = b + t * gj;
        }
    }
    const uint64_t rm = __ballot(act);
    nrot += static_cast<uint32_t>(__popcll(rm));
    static_for<0, BW>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int p = WjPair<BW, CROSS, RI, j>::p, q = WjPair<BW, CROSS, RI, j>::q;
        if (rm & (1ull << j)) {  // uniform
            const double cj = readlane64(c, j), sj = readlane64(sn, j);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const double xp = x[i][p], xq = x[i][q];
                x[i][p] = cj * xp - sj * xq;
                x[i][q] = sj * xp + cj * xq;
            }
        }
    });
}

// One move of the circle method: tops shift up one wave (wave 0 keeps its top, wave 0's bottom
// becomes wave 1's top), bottoms shift down one wave (wave 15's top becomes its bottom).  The
// squared norms travel with their columns.
template <int R>
__device__ __forceinline__ void wj_exchange(double (&x)[R][4 * R], double *stage, double (*nrm)[4 * R],
                                            double (*nst)[2 * R], int lane, int w)
{
    constexpr int BW = 2 * R, NPD = 64 * R;
    auto put = [&](int slot, auto off_tag) {
        constexpr int off = decltype(off_tag)::value;
        double *d = stage + static_cast<size_t>(slot) * BW * NPD;
        static_for<0, BW>([&](auto cc) {
#pragma unroll
            for (int i = 0; i < R; ++i) d[decltype(cc)::value * NPD + lane + 64 * i] = x[i][off + decltype(cc)::value];
        });
        if (lane < BW) nst[slot][lane] = nrm[w][off + lane];
    };
    auto get = [&](int slot, auto off_tag) {
        constexpr int off = decltype(off_tag)::value;
        const double *d = stage + static_cast<size_t>(slot) * BW * NPD;
        static_for<0, BW>([&](auto cc) {
#pragma unroll
            for (int i = 0; i < R; ++i) x[i][off + decltype(cc)::value] = d[decltype(cc)::value * NPD + lane + 64 * i];
        });
        if (lane < BW) nrm[w][off + lane] = nst[slot][lane];
    };
    using Top = std::integral_constant<int, 0>;
    using Bot = std::integral_constant<int, BW>;
    __syncthreads();  // the previous move's reads are done
    if (w >= 1) put(w, Top{});
    else put(0, Bot{});
    __syncthreads();
    if (w >= 2) get(w - 1, Top{});
    else if (w == 1) get(0, Top{});
    __syncthreads();
    if (w >= 1) put(w - 1, Bot{});  // slots 0..14; slot 15 still holds wave 15's old top
    __syncthreads();
    get(w <= 14 ? w : 15, Bot{});
}

template <int R>
__global__ __launch_bounds__(1024) void gram_jacobi1_kernel(double *__restrict__ X, double *__restrict__ zs,
                                                            int32_t *info)
{
    constexpr int NPD = 64 * R, BW = 2 * R, NC = 4 * R;
    extern __shared__ double stage[];  // 16 slots of BW x NPD
    __shared__ double nrm[16][NC];
    __shared__ double nst[16][BW];
    __shared__ uint32_t nrot_sh;
    __shared__ uint32_t big_sh;  // some rotation of the sweep had a cosine of 1e-8 or more
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tb = w, bb = 31 - w;
    double x[R][NC];
    static_for<0, BW>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            x[i][c] = X[static_cast<size_t>(tb * BW + c) * NPD + lane + 64 * i];
            x[i][BW + c] = X[static_cast<size_t>(bb * BW + c) * NPD + lane + 64 * i];
        }
    });
    const double tol = static_cast<double>(NPD) * 0x1.0p-52;
    const double tol2 = tol * tol;
    double *nrm_w = nrm[w];
    // squared column norms, one wave reduction at a time (keeps the register footprint small)
    auto norms = [&](double (&n2)[NC]) {
        static_for<0, NC>([&](auto cc) {
            double acc[1] = {0.0};
#pragma unroll
            for (int i = 0; i < R; ++i) acc[0] = __builtin_fma(x[i][decltype(cc)::value], x[i][decltype(cc)::value], acc[0]);
            wave_totals<1>(acc);
            n2[decltype(cc)::value] = acc[0];
        });
    };
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        {
            double n2[NC];
            norms(n2);
            if (lane == 0) static_for<0, NC>([&](auto cc) { nrm_w[decltype(cc)::value] = n2[decltype(cc)::value]; });
        }
        if (threadIdx.x == 0) {
            nrot_sh = 0u;
            big_sh = 0u;
        }
        __syncthreads();
        uint32_t nrot = 0;
        bool big = false;
        static_for<0, BW - 1>([&](auto ri) { wj_round<R, 0, decltype(ri)::value>(x, nrm_w, lane, nrot, tol2, big); });
        for (int r = 0; r < 31; ++r) {
            static_for<0, BW>([&](auto ri) { wj_round<R, 1, decltype(ri)::value>(x, nrm_w, lane, nrot, tol2, big); });
            wj_exchange<R>(x, stage, nrm, nst, lane, w);
        }
        if (lane == 0 && nrot) atomicAdd(&nrot_sh, nrot);
        if (__any(big) && lane == 0) atomicOr(&big_sh, 1u);
        __syncthreads();
        // Done after a sweep without rotations, or after one whose largest rotated cosine was
        // below 1e-8: convergence is quadratic by then, so a further sweep would only meet cosines
        // of order 1e-16, below the tolerance (the Gram path's a-posteriori check guards the result).
        const bool done = nrot_sh == 0u || big_sh == 0u;
        __syncthreads();
        if (done) {
            ++sweep;
            break;
        }
    }
    // after whole sweeps every block is back in its home wave
    double n2[NC];
    norms(n2);
    static_for<0, BW>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            X[static_cast<size_t>(tb * BW + c) * NPD + lane + 64 * i] = x[i][c];
            X[static_cast<size_t>(bb * BW + c) * NPD + lane + 64 * i] = x[i][BW + c];
        }
        if (lane == 0) {
            zs[tb * BW + c] = __builtin_sqrt(n2[c]);
            zs[bb * BW + c] = __builtin_sqrt(n2[BW + c]);
        }
    });
    if (threadIdx.x == 0 && info) {
        info[0] = sweep;
        info[1] = sweep >= kMaxSweeps ? 2 : 0;
    }
}

template <int R> static hipError_t launch_gram_jacobi1(double *X, double *zs, int32_t *info, hipStream_t stream)
{
    constexpr size_t lds = static_cast<size_t>(16) * (2 * R) * (64 * R) * sizeof(double);
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&gram_jacobi1_kernel<R>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    });
    gram_jacobi1_kernel<R><<<1, 1024, lds, stream>>>(X, zs, info);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Gram path for wide work matrices (kGramMaxCols < cols <= kGramGridMaxCols)
//
//   G = A^T A (gram_kernel), then a factor X with X X^T = G by a blocked Cholesky factorisation with
//   diagonal pivoting, then one-sided Jacobi on X spread over the device (gram_jacobi_grid_kernel).
//   Panel k takes 64 pivots: its candidates are the 128 remaining rows with the largest Schur
//   diagonal; one workgroup factors their 128 x 128 Schur block with greedy diagonal pivoting
//   (64 steps, each taking the candidate with the largest updated diagonal), which gives the
//   panel's pivot rows and the factor's rows at the candidates; the other rows come from forward
//   substitution against the pivots' 64 x 64 triangle, and the Schur complement is updated on MFMA.
//   Rows stay in their original order (X is lower triangular in pivot order).  The pivoting makes
//   the columns of X graded, which is what makes one-sided Jacobi on X converge fast (on the cube's
//   4096 x 1728 block 11 sweeps against 25 without pivoting).  A candidate whose Schur diagonal is at
//   or below np 2^-52 G_jj (numerically dependent on the pivots before it) is not taken while another
//   qualifies; a step without a qualifying candidate eliminates one with a zero factor column.
// ---------------------------------------------------------------------------------------------
constexpr int kCholNb = 64;     // pivots per panel
constexpr int kCholCand = 128;  // candidates per panel
// sort keys and rows of the candidate selection (np <= 2048 rounded up to a power of two)
constexpr size_t kCholLds = static_cast<size_t>(2048) * (sizeof(double) + sizeof(int));

// Row state of the pivoted factorisation (int32 arrays of np in SvdDevView::gpiv):
//   rs[r]  -1 while row r remains, else the panel that eliminated it
//   cp[r]  the last panel that had row r among its candidates (-1 none)
//   piv[k] the row of pivot step k
struct CholState {
    int32_t *rs, *cp, *piv;
};

// (key, row) a precedes (key, row) b: larger key first, then lower row
__device__ __forceinline__ bool chol_before(double ka, int ia, double kb, int ib)
{
    return ka > kb || (ka == kb && ia < ib);
}

// Panel k0, part 1: candidate selection, a bitonic sort of the remaining rows by their Schur diagonal
// (larger first, then lower row) in LDS; writes the kCholCand candidates (rows, diagonals,
// dependence thresholds np 2^-52 G_jj) to cand and marks them in the row states.  Panel 0 first
// copies the diagonal of G to dg and initialises the row states.
struct CholCand {
    int32_t row[kCholCand];
    double d[kCholCand], th[kCholCand];
};

__global__ __launch_bounds__(1024) void chol_select_kernel(const double *__restrict__ S, int np, int k0,
                                                           double *__restrict__ dg, CholState cs,
                                                           CholCand *__restrict__ cand)
{
    extern __shared__ double lds[];  // n2 sort keys, then n2 rows
    const int tid = threadIdx.x;
    const int panel = k0 / kCholNb;
    if (k0 == 0) {
        for (int j = tid; j < np; j += 1024) {
            dg[j] = S[static_cast<size_t>(j) * np + j];
            cs.rs[j] = -1;
            cs.cp[j] = -1;
        }
        __syncthreads();
    }
    int n2 = 64;
    while (n2 < np) n2 <<= 1;
    double *key = lds;
    int *row = reinterpret_cast<int *>(lds + n2);
    for (int j = tid; j < n2; j += 1024) {
        key[j] = (j < np && cs.rs[j] < 0) ? S[static_cast<size_t>(j) * np + j] : -__builtin_inf();
        row[j] = j;
    }
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < n2 / 2; i += 1024) {
                const int a = (i / j) * 2 * j + (i % j), b = a + j;
                const bool up = (a & k) == 0;
                const double ka = key[a], kb = key[b];
                const int ia = row[a], ib = row[b];
                if (up ? chol_before(kb, ib, ka, ia) : chol_before(ka, ia, kb, ib)) {
                    key[a] = kb;
                    key[b] = ka;
                    row[a] = ib;
                    row[b] = ia;
                }
            }
            __syncthreads();
        }
    }
    const int nrem = np - k0;  // every panel eliminates kCholNb rows
    const int nc = nrem < kCholCand ? nrem : kCholCand;
    if (tid < kCholCand) {
        const int r = tid < nc ? row[tid] : -1;
        cand->row[tid] = r;
        cand->d[tid] = tid < nc ? key[tid] : -__builtin_inf();
        cand->th[tid] = tid < nc ? static_cast<double>(np) * 0x1.0p-52 * dg[r] : 0.0;
        if (tid < nc) cs.cp[r] = panel;
    }
}

// Panel k0, part 2: the 64 greedy pivot steps, one wave.  The candidates' Schur block M (lower
// triangle) is gathered into LDS once; lane l keeps the factor rows of candidates l and l + 64 in
// registers.  Step s takes the candidate with the largest updated diagonal (among those above their
// dependence threshold; none: the first remaining one, with a zero column), its owner publishes its
// factor row in LDS, and every candidate a forms l_a = (M[a, p] - L[a, 0:s] L[p, 0:s]^T) / sqrt(d_p)
// and d_a -= l_a^2 (left-looking, so no block update).  The steps are unrolled at compile time (the
// factor rows stay in registers).  Writes the factor's columns k0 .. k0 + 63 at the candidate rows,
// the pivots and the row states.
__global__ __launch_bounds__(256) void chol_steps_kernel(const double *__restrict__ S, double *__restrict__ X, int np,
                                                         int k0, CholState cs, const CholCand *__restrict__ cand)
{
    constexpr int kTri = kCholCand * (kCholCand + 1) / 2;
    __shared__ double M[kTri];         // M[a (a + 1) / 2 + b], b <= a
    __shared__ double Lc[kCholCand][kCholNb + 1];  // factor rows of the candidates, as computed
    __shared__ int rowc[kCholCand];
    const int tid = threadIdx.x, lane = tid & 63;
    const int panel = k0 / kCholNb;
    const int nrem = np - k0;
    const int nc = nrem < kCholCand ? nrem : kCholCand;
    if (tid < kCholCand) rowc[tid] = cand->row[tid];
    __syncthreads();
    // gather by the whole workgroup, 8 independent loads in flight per thread
    for (int e0 = tid; e0 < kTri; e0 += 256 * 8) {
        double val[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u;
            val[u] = 0.0;
            if (e < kTri) {
                int a = static_cast<int>((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
                while ((a + 1) * (a + 2) / 2 <= e) ++a;
                while (a * (a + 1) / 2 > e) --a;
                const int b = e - a * (a + 1) / 2;
                if (a < nc) val[u] = S[static_cast<size_t>(rowc[b]) * np + rowc[a]];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e0 + 256 * u < kTri) M[e0 + 256 * u] = val[u];
    }
    __syncthreads();
    if (tid >= 64) return;
    double Lr[2][kCholNb];
    bool taken[2];
    double d[2], th[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int a = lane + 64 * h;
        taken[h] = a >= nc;
        d[h] = cand->d[a];
        th[h] = cand->th[a];
#pragma unroll
        for (int t = 0; t < kCholNb; ++t) Lr[h][t] = 0.0;
    }
    static_for<0, kCholNb>([&](auto ss) {
        constexpr int st = decltype(ss)::value;
        // argmax of the qualifying diagonals: positive doubles order as their bit patterns, so the
        // low 7 mantissa bits carry 127 - a (equal truncated values: the lower candidate wins)
        double key = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int a = lane + 64 * h;
            if (!taken[h] && d[h] > th[h]) {
                const double k = __longlong_as_double(
                    static_cast<long long>((static_cast<unsigned long long>(__double_as_longlong(d[h])) & ~0x7Full) |
                                           static_cast<unsigned long long>(127 - a)));
                key = key > k ? key : k;
            }
        }
        key = wave_max_pos(key);
        const bool qual = key > 0.0;  // uniform
        int p;
        double best = 0.0;
        if (qual) {
            p = 127 - static_cast<int>(static_cast<unsigned long long>(__double_as_longlong(key)) & 0x7Full);
            const double dp = (p >> 6) ? d[1] : d[0];
            best = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(dp), p & 63),
                                    __builtin_amdgcn_readlane(__double2loint(dp), p & 63));
        } else {  // none above its threshold: the first remaining candidate, with a zero column
            const uint64_t m0 = __ballot(!taken[0]), m1 = __ballot(!taken[1]);
            p = m0 ? __builtin_ctzll(m0) : 64 + __builtin_ctzll(m1);
        }
        const double inv = qual ? rsq64(best) : 0.0;
        const double *lp = Lc[p];  // the pivot's factor row (uniform address: broadcast reads)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int a = lane + 64 * h;
            double acc0 = a >= p ? M[a * (a + 1) / 2 + p] : M[p * (p + 1) / 2 + a], acc1 = 0.0;
#pragma unroll
            for (int t = 0; t + 1 < st; t += 2) {
                acc0 = __builtin_fma(-Lr[h][t], lp[t], acc0);
                acc1 = __builtin_fma(-Lr[h][t + 1], lp[t + 1], acc1);
            }
            if constexpr (st & 1) acc0 = __builtin_fma(-Lr[h][st - 1], lp[st - 1], acc0);
            // sqrt(d_p) at the pivot; rows already taken (or absent) keep zeros
            const double l = taken[h] ? 0.0 : (a == p ? best * inv : (acc0 + acc1) * inv);
            if (a == p) taken[h] = true;
            Lr[h][st] = l;
            Lc[a][st] = l;
            d[h] = __builtin_fma(-l, l, d[h]);
        }
        if (lane == 0) {
            const int rp = rowc[p];
            cs.piv[k0 + st] = rp;
            cs.rs[rp] = panel;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // column st is read by the next steps
    });
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int a = lane + 64 * h;
        if (a < nc) {
            const int r = rowc[a];
#pragma unroll
            for (int t = 0; t < kCholNb; ++t) X[static_cast<size_t>(k0 + t) * np + r] = Lr[h][t];
        }
    }
}

// Rows of panel k0 that were not its candidates: rows eliminated by earlier panels get zeros, the
// others solve L_PP l_r = S[r, P] by forward substitution (one thread per row), L_PP the pivots'
// lower triangle (rows of X at the pivots) in LDS; a zero pivot leaves its entry zero.
__global__ __launch_bounds__(256) void chol_rows_kernel(const double *__restrict__ S, double *__restrict__ X, int np,
                                                        int k0, CholState cs)
{
    __shared__ double L[kCholNb][kCholNb + 1];  // L[c][t] = factor column k0 + t at pivot row c
    __shared__ double inv[kCholNb];
    __shared__ int P[kCholNb];
    const int panel = k0 / kCholNb;
    if (threadIdx.x < kCholNb) P[threadIdx.x] = cs.piv[k0 + threadIdx.x];
    __syncthreads();
    for (int e = threadIdx.x; e < kCholNb * kCholNb; e += 256) {
        const int c = e % kCholNb, t = e / kCholNb;
        L[c][t] = X[static_cast<size_t>(k0 + t) * np + P[c]];
    }
    __syncthreads();
    if (threadIdx.x < kCholNb) {
        const double d = L[threadIdx.x][threadIdx.x];
        inv[threadIdx.x] = d > 0.0 ? 1.0 / d : 0.0;
    }
    __syncthreads();
    const int r = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
    if (r >= np || cs.cp[r] == panel) return;
    const int st = cs.rs[r];
    if (st >= 0 && st < panel) {
#pragma unroll
        for (int c = 0; c < kCholNb; ++c) X[static_cast<size_t>(k0 + c) * np + r] = 0.0;
        return;
    }
    double x[kCholNb];
#pragma unroll
    for (int c = 0; c < kCholNb; ++c) x[c] = S[static_cast<size_t>(P[c]) * np + r];
    static_for<0, kCholNb>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        double acc = x[c];
#pragma unroll
        for (int t = 0; t < c; ++t) acc = __builtin_fma(-x[t], L[c][t], acc);
        x[c] = acc * inv[c];
    });
#pragma unroll
    for (int c = 0; c < kCholNb; ++c) X[static_cast<size_t>(k0 + c) * np + r] = x[c];
}

// Schur complement update of panel k0 over the whole np x np matrix (rows eliminated before have
// zero factor entries): S_ij -= sum_c X_i,k0+c X_j,k0+c, one 16 x 16 tile per wave (MFMA).
__global__ __launch_bounds__(256) void chol_syrk_kernel(double *__restrict__ S, const double *__restrict__ X, int np,
                                                        int k0)
{
    const int T = np / 16;
    const int wave = static_cast<int>((blockIdx.x * 256u + threadIdx.x) >> 6);
    if (wave >= T * T) return;  // whole waves
    const int i0 = 16 * (wave % T), j0 = 16 * (wave / T);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c0 = 0; c0 < kCholNb; c0 += 4) {
        const double *xc = X + static_cast<size_t>(k0 + c0 + lk) * np;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xc[i0 + li], xc[j0 + li], acc, 0, 0, 0);
    }
    double *sc = S + static_cast<size_t>(j0 + li) * np + i0 + lk;
#pragma unroll
    for (int e = 0; e < 4; ++e) sc[4 * e] -= acc[e];
}

static hipError_t chol_pivoted(const SvdDevView &v, hipStream_t stream)
{
    const CholState cs{reinterpret_cast<int32_t *>(v.gpiv), reinterpret_cast<int32_t *>(v.gpiv) + v.np,
                       reinterpret_cast<int32_t *>(v.gpiv) + 2 * v.np};
    CholCand *cand = reinterpret_cast<CholCand *>(v.gpiv + 3 * static_cast<size_t>(v.np));
    const int T = v.np / 16;
    for (int k0 = 0; k0 < v.np; k0 += kCholNb) {
        chol_select_kernel<<<1, 1024, kCholLds, stream>>>(v.G, v.np, k0, v.zs, cs, cand);
        chol_steps_kernel<<<1, 256, 0, stream>>>(v.G, v.L, v.np, k0, cs, cand);
        chol_rows_kernel<<<(v.np + 255) / 256, 256, 0, stream>>>(v.G, v.L, v.np, k0, cs);
        if (k0 + kCholNb < v.np) chol_syrk_kernel<<<(T * T + 3) / 4, 256, 0, stream>>>(v.G, v.L, v.np, k0);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// One-sided Jacobi of the Gram path's factor X (np x np) spread over the device.
//
// The columns form nblk = np / BW blocks.  Workgroup w of P = nblk / 2 holds, in round t of the
// circle ordering, block top(t, w) = 0 (w = 0) or ((w - 1 + t) mod (nblk - 1)) + 1 and block
// bot(t, w) = ((nblk - 2 - w + t) mod (nblk - 1)) + 1 in registers (thread t holds rows t + 256 i,
// i < R).  A sweep rotates the pairs inside each block, then runs nblk - 1 rounds in which the two
// blocks of every workgroup meet (BW sub-rounds of BW disjoint cross pairs).  After a round the
// blocks move: tops go from workgroup w to w - 1 (workgroup 1's top becomes workgroup 0's bottom;
// block 0 stays with workgroup 0), bottoms from w to w + 1 (workgroup P - 1's bottom becomes its own
// top).  A moving block is written to its home columns of X, the writer publishes the round number
// in its flag (release), and the receiver waits for that flag (acquire) before loading; a block has
// one holder at a time, so its home columns serve as its mailbox.  The squared norms travel through
// nrm.  Dot products: per-thread partials, a wave reduction that leaves pair j's sum in lane j, then
// the four waves' sums added in a fixed order from LDS, so every wave takes the same decisions.
// After nblk - 1 moves every block is home again.  Each sweep ends with device-wide counts of its
// rotations and of rotations with a cosine >= 1e-7; the iteration stops after a sweep without the
// latter: convergence is quadratic by then, so what is left is of order 1e-14, which the first-order
// eigenvector correction that follows this kernel reduces to rounding.  Every wait is bounded: an expired wait sets the error
// word and the workgroups leave, the result is then rejected.  When the stream's CUs cannot hold P
// workgroups, G < P workgroups take P / G positions each per round through memory, with a device-wide
// barrier between rounds (same arithmetic per meeting, so the same result bit for bit).
// ---------------------------------------------------------------------------------------------
struct GridJacobiArgs {
    double *X;       // np x np factor, column-major, rotated in place
    double *zs;      // np column norms of the result
    double *nrm;     // np squared norms of the blocks in flight
    uint32_t *ctl;   // kGridFlags round flags, then the counters of GridCtl (zeroed before the launch)
    int32_t *info;   // [0] sweeps, [1] error flags (1 wait expired, 2 not converged)
    int np;
    int P;           // block pairs (np / (2 BW)); the grid has P workgroups or fewer
};

// Relaxed polls of a round flag (the caller issues one acquire fence after all its waits).
__device__ __forceinline__ bool spin_until(const uint32_t *word, uint32_t target, uint32_t *err)
{
    uint32_t spins = 0;
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
        if (++spins > (1u << 26)) {
            atomicExch(err, 1u);
            return false;
        }
    }
    return true;
}

// One sub-round: BW disjoint pairs (WjPair<BW, CROSS, RI, j>) of the workgroup's 2 BW columns.
template <int R, int BW, int NW, int CROSS, int RI>
__device__ __forceinline__ void gj_round(double (&x)[R][2 * BW], double *nrm_w, double (*part)[NW][8], int &ph,
                                         int lane, int wv, uint32_t &nrot, bool &big, double tol2)
{
    constexpr int P8 = BW <= 2 ? 2 : (BW <= 4 ? 4 : 8);
    double g[P8];
    static_for<0, P8>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        if constexpr (j < BW) {
            constexpr int p = WjPair<BW, CROSS, RI, j>::p, q = WjPair<BW, CROSS, RI, j>::q;
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < R; ++i) acc = __builtin_fma(x[i][p], x[i][q], acc);
            g[j] = acc;
        } else {
            g[j] = 0.0;
        }
    });
    const double gw = split_totals<P8>(g, lane);
    if (lane < BW) part[ph][wv][lane] = gw;
    __syncthreads();
    const int ls = lane & 7;
    double gj = part[ph][0][ls];
#pragma unroll
    for (int w2 = 1; w2 < NW; ++w2) gj += part[ph][w2][ls];
    ph ^= 1;
    double c = 1.0, sn = 0.0;
    bool act = false;
    int ln = lane;
    asm volatile("" : "+v"(ln));
    if (ln < BW) {
        int p, q;
        if constexpr (CROSS) {
            p = ln;
            q = BW + (ln + RI) % BW;
        } else {
            const int k = ln < BW / 2 ? ln : ln - BW / 2, off = ln < BW / 2 ? 0 : BW;
            pair_of(RI, k, BW, p, q);
            p += off;
            q += off;
        }
        const double a = nrm_w[p], b = nrm_w[q];
        act = gj != 0.0 && gj * gj > tol2 * a * b;
        if (act) {
            double t;
            big = big || gj * gj >= 1e-14 * (a * b);  // a rotated cosine of 1e-7 or more
            rot_params(a, b, gj, c, sn, t);
            nrm_w[p] = a - t * gj;
            nrm_w[q] = b + t * gj;
        }
    }
    const uint64_t rm = __ballot(act);
    nrot += static_cast<uint32_t>(__popcll(rm));
    static_for<0, BW>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int p = WjPair<BW, CROSS, RI, j>::p, q = WjPair<BW, CROSS, RI, j>::q;
        if (rm & (1ull << j)) {  // uniform
            const double cj = readlane64(c, j), sj = readlane64(sn, j);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const double xp = x[i][p], xq = x[i][q];
                x[i][p] = cj * xp - sj * xq;
                x[i][q] = sj * xp + cj * xq;
            }
        }
    });
}

template <int R, int BW, int NT>
__global__ __launch_bounds__(NT) void gram_jacobi_grid_kernel(GridJacobiArgs J)
{
    constexpr int NW = NT / 64;
    __shared__ double part[2][NW][8];
    __shared__ double nrm_s[NW][2 * BW];
    __shared__ uint32_t stop_sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int G = gridDim.x, P = J.P, nblk = 2 * P, m1 = nblk - 1, np = J.np;
    // Ring position of this workgroup.  Workgroups are dispatched to the 8 XCDs round-robin, so
    // consecutive positions (the neighbours that exchange blocks every round) are given to
    // workgroups of the same XCD, and only 8 of the ring's links cross XCDs.
    const int bx = blockIdx.x, xq = G / 8, xr = G % 8, xx = bx % 8;
    const int w = G < P ? bx : xx * xq + (xx < xr ? xx : xr) + bx / 8;
    uint32_t *flag = J.ctl;
    uint32_t *rot = J.ctl + kGridFlags;
    uint32_t *bigc = rot + kMaxSweeps;
    uint32_t *bar = bigc + kMaxSweeps;
    uint32_t *err = bar + 1;
    double *nrm_w = nrm_s[wv];
    auto top_of = [&](int t, int ww) { return ww == 0 ? 0 : ((ww - 1 + t) % m1) + 1; };
    auto bot_of = [&](int t, int ww) { return ((nblk - 2 - ww + t) % m1) + 1; };
    double x[R][2 * BW];
    // Blocks move between workgroups through their home columns of X as agent-scope relaxed atomic
    // stores and loads: they are written through to the device's coherent level, so the release
    // fence of a round finds no dirty L2 lines of them to write back.
    auto load = [&](int blk, int off) {
        const double *src = J.X + static_cast<size_t>(blk) * BW * np;
#pragma unroll
        for (int c = 0; c < BW; ++c)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = tid + NT * i;
                x[i][off + c] = r < np ? __hip_atomic_load(src + static_cast<size_t>(c) * np + r, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                                       : 0.0;
            }
        if (lane < BW) nrm_w[off + lane] = __hip_atomic_load(J.nrm + blk * BW + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto store = [&](int blk, int off, bool with_norms) {
        double *dst = J.X + static_cast<size_t>(blk) * BW * np;
#pragma unroll
        for (int c = 0; c < BW; ++c)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = tid + NT * i;
                if (r < np)
                    __hip_atomic_store(dst + static_cast<size_t>(c) * np + r, x[i][off + c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        if (with_norms && wv == 0 && lane < BW)
            __hip_atomic_store(J.nrm + blk * BW + lane, nrm_w[off + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // squared norms of the 2 BW columns, fresh from the registers (all waves get the same values)
    auto norms = [&]() {
        static_for<0, 2 * BW>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            double acc[1] = {0.0};
#pragma unroll
            for (int i = 0; i < R; ++i) acc[0] = __builtin_fma(x[i][c], x[i][c], acc[0]);
            wave_totals<1>(acc);
            if (lane == 0) part[0][wv][c & 7] = acc[0];
            __syncthreads();
            if (lane == 0) {
                double t = part[0][0][c & 7];
#pragma unroll
                for (int w2 = 1; w2 < NW; ++w2) t += part[0][w2][c & 7];
                nrm_w[c] = t;
            }
            __syncthreads();
        });
    };
    const double tol = static_cast<double>(np) * 0x1.0p-52;
    const double tol2 = tol * tol;
    uint32_t gen = 0, rho = 0;
    int ph = 0, sweep = 0;
    bool failed = false;
    auto intra = [&](uint32_t &nrot, bool &big) {
        static_for<0, BW - 1>([&](auto ri) {
            gj_round<R, BW, NW, 0, decltype(ri)::value>(x, nrm_w, part, ph, lane, wv, nrot, big, tol2);
        });
    };
    auto meet = [&](uint32_t &nrot, bool &big) {
        static_for<0, BW>([&](auto ri) {
            gj_round<R, BW, NW, 1, decltype(ri)::value>(x, nrm_w, part, ph, lane, wv, nrot, big, tol2);
        });
    };
    // sweep totals: a device-wide barrier, then every workgroup reads the same counts
    auto sweep_done = [&](uint32_t nrot, bool big) {
        if (tid == 0) {
            if (nrot) atomicAdd(&rot[sweep], nrot);
            if (big) atomicAdd(&bigc[sweep], 1u);
        }
        grid_barrier(bar, err, static_cast<uint32_t>(G), gen);
        const uint32_t nr = __hip_atomic_load(&rot[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t nb = __hip_atomic_load(&bigc[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        failed = __hip_atomic_load(err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        return nr == 0u || nb == 0u;
    };
    if (G < P) {
        // Fewer workgroups than block pairs (the stream's CUs cannot hold P): workgroup w takes the
        // positions w, w + G, ... of every round, loading both blocks from their home columns and
        // storing them back, with a device-wide barrier between rounds.  Each meeting runs the
        // same code on the same data as in the resident mode below, so the result is the same bit
        // for bit whatever the number of workgroups.
        for (; sweep < kMaxSweeps && !failed; ++sweep) {
            uint32_t nrot = 0;
            bool big = false;
            for (int t = 0; t < m1 && !failed; ++t) {
                for (int pos = w; pos < P; pos += G) {
                    load(top_of(t, pos), 0);
                    load(bot_of(t, pos), BW);
                    __syncthreads();
                    if (t == 0) {  // home blocks: fresh norms, the pairs inside each block
                        norms();
                        intra(nrot, big);
                    }
                    meet(nrot, big);
                    store(top_of(t, pos), 0, true);
                    store(bot_of(t, pos), BW, true);
                    __syncthreads();
                }
                if (t + 1 < m1) {
                    grid_barrier(bar, err, static_cast<uint32_t>(G), gen);
                    failed = __hip_atomic_load(err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u;
                }
            }
            if (failed) break;
            if (sweep_done(nrot, big)) {
                ++sweep;
                break;
            }
        }
        for (int pos = w; pos < P; pos += G) {
            load(pos, 0);
            load(nblk - 1 - pos, BW);
            __syncthreads();
            norms();
            if (wv == 0 && lane < 2 * BW) {
                const int col = lane < BW ? pos * BW + lane : (nblk - 1 - pos) * BW + lane - BW;
                J.zs[col] = __builtin_sqrt(nrm_w[lane]);
            }
            __syncthreads();
        }
        if (w == 0 && tid == 0) {
            J.info[0] = sweep;
            J.info[1] = (failed || __hip_atomic_load(err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u ? 1 : 0) |
                        (sweep >= kMaxSweeps ? 2 : 0);
        }
        return;
    }
    load(w, 0);
    load(nblk - 1 - w, BW);
    __syncthreads();
    for (; sweep < kMaxSweeps && !failed; ++sweep) {
        norms();
        uint32_t nrot = 0;
        bool big = false;
        intra(nrot, big);
        for (int t = 0; t < m1 && !failed; ++t) {
            meet(nrot, big);
            if (P == 1) continue;  // two blocks: nothing moves
            // outgoing: the top to w - 1 (w >= 1), the bottom to w + 1 (w <= P - 2)
            if (w >= 1) store(top_of(t, w), 0, true);
            if (w <= P - 2) store(bot_of(t, w), BW, true);
            __syncthreads();
            if (tid == 0) {  // the barrier above ordered the workgroup's stores before this release
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(&flag[w], rho + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (w == P - 1) {  // the bottom becomes the top
#pragma unroll
                for (int c = 0; c < BW; ++c)
#pragma unroll
                    for (int i = 0; i < R; ++i) x[i][c] = x[i][BW + c];
                if (lane < BW) nrm_w[lane] = nrm_w[BW + lane];
            }
            if (tid == 0) {
                bool ok = true;
                if (w <= P - 2) ok = spin_until(&flag[w + 1], rho + 1, err);
                if (ok && w >= 1) ok = spin_until(&flag[w - 1], rho + 1, err);
                stop_sh = ok ? 0u : 1u;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            failed = stop_sh != 0u;
            if (failed) break;
            if (w == 0) load(top_of(t, 1), BW);
            else {
                if (w <= P - 2) load(top_of(t, w + 1), 0);
                load(bot_of(t, w - 1), BW);
            }
            ++rho;
            __syncthreads();
        }
        if (failed) break;
        if (sweep_done(nrot, big)) {
            ++sweep;
            break;
        }
    }
    // home again after whole sweeps (or garbage after a failed wait, which the acceptance rejects)
    norms();
    store(w, 0, false);
    store(nblk - 1 - w, BW, false);
    if (wv == 0 && lane < 2 * BW) {
        const int col = lane < BW ? w * BW + lane : (nblk - 1 - w) * BW + lane - BW;
        J.zs[col] = __builtin_sqrt(nrm_w[lane]);
    }
    if (w == 0 && tid == 0) {
        J.info[0] = sweep;
        J.info[1] = (failed || __hip_atomic_load(err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u ? 1 : 0) |
                    (sweep >= kMaxSweeps ? 2 : 0);
    }
}

constexpr int kGridBW = 8;

// The device-wide Jacobi: 256 threads per workgroup (one wave per SIMD) and R = np / 256 rounded up
// rows per thread.  (512 or 1024 threads with fewer rows each measured slower: more waves meet at
// every sub-round's barrier, and the larger variants spill.)
constexpr int kGridThreads = 256;

template <int R> static const void *grid_fn()
{
    return reinterpret_cast<const void *>(&gram_jacobi_grid_kernel<R, kGridBW, kGridThreads>);
}

static const void *grid_jacobi_fn(int np)
{
    switch ((np + kGridThreads - 1) / kGridThreads) {
    case 1: return grid_fn<1>();
    case 2: return grid_fn<2>();
    case 3: return grid_fn<3>();
    case 4: return grid_fn<4>();
    case 5: return grid_fn<5>();
    case 6: return grid_fn<6>();
    case 7: return grid_fn<7>();
    case 8: return grid_fn<8>();
    }
    return nullptr;
}

// C(i, j) = scale_j sum_k opA(i, k) opB(k, j), opA(i, k) = A[i sai + k sak],
// opB(k, j) = B[k sbk + col(j) sbj] with col(j) = bcol ? bcol[j] : j, and scale_j from z[col(j)]:
// mode 0: 1, mode 1: 1 / z^2, mode 2: 1 / z (0 where z <= 1e-7 max z), mode 3: 1 / z (0 where
// z = 0).  C column-major with leading dimension ldc; rows m .. mo - 1 and columns n .. no - 1 of C
// (mo, no: 0 for m, n) are written as zeros.
struct GemmArgs {
    const double *A;
    long sai, sak;
    const double *B;
    long sbk, sbj;
    const int32_t *bcol;
    double *C;
    long ldc;
    int m, n, kd;
    const double *z;
    int zn, mode;
    int mo = 0, no = 0;
};

__device__ __forceinline__ double gemm_scale(const GemmArgs &g, int cj)
{
    if (g.mode == 0) return 1.0;
    const double zc = g.z[cj];
    if (g.mode == 3) return zc > 0.0 ? 1.0 / zc : 0.0;
    double zmax = 0.0;
    for (int e = 0; e < g.zn; ++e) zmax = g.z[e] > zmax ? g.z[e] : zmax;
    return zc > 1e-7 * zmax ? (g.mode == 1 ? 1.0 / (zc * zc) : 1.0 / zc) : 0.0;
}

// The GEMM in 64 x 64 tiles of C per 256-thread workgroup: K in chunks of 16 staged through LDS
// (the A chunk 64 x 16 and the B chunk 16 x 64, both stored k-major), each wave computing a 32 x 32
// quarter as 2 x 2 v_mfma_f64_16x16x4f64 tiles, so every operand fetched from L2 feeds 32 MFMA
// products instead of one.  Chunks are loaded along the operand's unit stride (coalesced), and the
// next chunk is fetched into registers while the current one is multiplied from the other of two
// LDS buffers (one barrier per chunk).
constexpr int kTM = 64, kTK = 16;
__global__ __launch_bounds__(256) void gemm_tile_kernel(GemmArgs g)
{
    __shared__ double As[2][kTK][kTM + 1];  // As[buf][k][i]
    __shared__ double Bs[2][kTK][kTM + 1];  // Bs[buf][k][j]
    __shared__ int cols[kTM];
    const int mo = g.mo > g.m ? g.mo : g.m, no = g.no > g.n ? g.no : g.n;
    const int tm = (mo + kTM - 1) / kTM;
    const int i0 = static_cast<int>(blockIdx.x % tm) * kTM, j0 = static_cast<int>(blockIdx.x / tm) * kTM;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wi = (wv & 1) * 32, wj = (wv >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    if (tid < kTM) {
        const int j = j0 + tid;
        cols[tid] = j < g.n ? (g.bcol ? g.bcol[j] : j) : -1;
    }
    __syncthreads();
    d4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    const bool a_rows = g.sai == 1;  // A contiguous along i, else along k
    const bool b_ks = g.sbk == 1;    // B contiguous along k, else along j
    // this thread's four elements of each chunk: (k, i) of A and (k, j) of B
    int ak[4], ai[4], bk[4], bj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ai[q] = a_rows ? (tid & 63) : (tid >> 4) + 16 * q;
        ak[q] = a_rows ? (tid >> 6) + 4 * q : (tid & 15);
        bj[q] = b_ks ? (tid >> 4) + 16 * q : (tid & 63);
        bk[q] = b_ks ? (tid & 15) : (tid >> 6) + 4 * q;
    }
    double ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gi = i0 + ai[q], gk = k0 + ak[q];
            ra[q] = (gi < g.m && gk < g.kd) ? g.A[gi * g.sai + gk * g.sak] : 0.0;
            const int cj = cols[bj[q]], gkb = k0 + bk[q];
            rb[q] = (cj >= 0 && gkb < g.kd) ? g.B[gkb * g.sbk + cj * g.sbj] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][ak[q]][ai[q]] = ra[q];
            Bs[buf][bk[q]][bj[q]] = rb[q];
        }
    };
    const int nch = (g.kd + kTK - 1) / kTK;
    if (nch > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) fetch((c + 1) * kTK);  // in flight during the products below
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 4) {
            const double a0 = As[buf][kk + lk][wi + li], a1 = As[buf][kk + lk][wi + 16 + li];
            const double b0 = Bs[buf][kk + lk][wj + li], b1 = Bs[buf][kk + lk][wj + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        // the other buffer was last read in chunk c - 1, before the previous barrier
        if (c + 1 < nch) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        const int jl = wj + 16 * y + li, j = j0 + jl;
        if (j >= no) continue;
        const double scale = j < g.n ? gemm_scale(g, cols[jl]) : 0.0;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = i0 + wi + 16 * x + 4 * e + lk;
                if (i < mo) g.C[i + static_cast<long>(j) * g.ldc] = (i < g.m && j < g.n) ? acc[x][y][e] * scale : 0.0;
            }
    }
}

// Om (rows x cols, column-major) = +-1 from the top bit of Philox4x32-10 words, keyed by the
// request's seed; counter (row / 4, column, 0x534b4554, 0).
__global__ void sketch_kernel(double *Om, int rows, int cols, uint32_t k0, uint32_t k1)
{
    const size_t total = static_cast<size_t>(rows) * cols;
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int r = static_cast<int>(e % rows), c = static_cast<int>(e / rows);
        uint32_t c0 = static_cast<uint32_t>(r >> 2), c1 = static_cast<uint32_t>(c), c2 = 0x534b4554u, c3 = 0u;
        philox4x32_10(c0, c1, c2, c3, k0, k1);
        const uint32_t wsel = (r & 3) == 0 ? c0 : (r & 3) == 1 ? c1 : (r & 3) == 2 ? c2 : c3;
        Om[e] = (wsel >> 31) ? 1.0 : -1.0;
    }
}

// s[rank] = z[c], perm[rank] = c for the k largest of z[0..n) (descending, ties by index).
__global__ void rank_kernel(const double *__restrict__ z, int n, int k, double *__restrict__ s_out,
                            int32_t *__restrict__ perm)
{
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const double zc = z[c];
        int rank = 0;
        for (int o = 0; o < n; ++o) rank += (z[o] > zc || (z[o] == zc && o < c)) ? 1 : 0;
        if (rank < k) {
            s_out[rank] = zc;
            perm[rank] = c;
        }
    }
}

constexpr int kPowerIters = 1;

static hipError_t gemm(const GemmArgs &g, hipStream_t stream)
{
    const int mo = g.mo > g.m ? g.mo : g.m, no = g.no > g.n ? g.no : g.n;
    const int tiles = ((mo + kTM - 1) / kTM) * ((no + kTM - 1) / kTM);
    if (tiles > 0) gemm_tile_kernel<<<tiles, 256, 0, stream>>>(g);
    return hipGetLastError();
}

// Acceptance statistic from C = Ys^T Ys (k x k, column-major): max_ij |C_ij - delta_ij| s_i s_j / s_1^2
// folded into crit[0] (atomic max on the bit pattern).
__global__ void gram_crit_kernel(SvdDevView v, const double *__restrict__ Cm)
{
    const size_t kk = static_cast<size_t>(v.k) * v.k;
    const double s0 = v.s[0];
    const double inv2 = s0 > 0.0 ? 1.0 / (s0 * s0) : 0.0;
    double dev = 0.0;
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < kk;
         e += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(e % v.k), j = static_cast<int>(e / v.k);
        const double d = __builtin_fabs(Cm[e] - (i == j ? 1.0 : 0.0)) * v.s[i] * v.s[j] * inv2;
        dev = (d > dev || d != d) ? d : dev;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double od = __shfl_xor(dev, o);
        dev = (od > dev || od != od) ? od : dev;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(v.crit, static_cast<unsigned long long>(__double_as_longlong(dev)));
}

// ---------------------------------------------------------------------------------------------
// Reconstruction
// ---------------------------------------------------------------------------------------------
__global__ void recon_q_kernel(SvdDevView v, const uint32_t *__restrict__ counts, double inv_n,
                               const double *__restrict__ uD, const double *__restrict__ u0)
{
    __shared__ double scratch[16];
    for (int i = blockIdx.x; i < v.m; i += gridDim.x) {
        double acc = 0.0;
        const uint32_t *row = counts + static_cast<size_t>(i) * v.n_elem;
        for (int l = threadIdx.x; l < v.n0; l += blockDim.x)
            acc = __builtin_fma(static_cast<double>(row[v.g0idx[l]]) * inv_n, u0[l], acc);
        acc = block_sum(acc, scratch);
        if (threadIdx.x == 0) v.q[i] = v.nu[i] * (uD[i] - acc);
        __syncthreads();
    }
}

__global__ void recon_c_kernel(SvdDevView v)
{
    __shared__ double scratch[16];
    for (int l = blockIdx.x; l < v.k; l += gridDim.x) {
        const double *u = v.U + static_cast<size_t>(l) * v.m;
        double acc = 0.0;
        for (int i = threadIdx.x; i < v.m; i += blockDim.x) acc = __builtin_fma(u[i], v.q[i], acc);
        acc = block_sum(acc, scratch);
        if (threadIdx.x == 0) v.cvec[l] = acc;
        __syncthreads();
    }
    if (blockIdx.x == 0) {  // |q|^2
        double acc = 0.0;
        for (int i = threadIdx.x; i < v.m; i += blockDim.x) acc = __builtin_fma(v.q[i], v.q[i], acc);
        acc = block_sum(acc, scratch);
        if (threadIdx.x == 0) v.work[v.cols] = acc;
    }
}

// Components with s_l at or below this level are left out of every solution: the numerical rank
// (max(m, n) u s_1), or the cut of the truncated path when that is larger.
__device__ __forceinline__ double rank_level(const SvdDevView &v)
{
    const double s0 = v.k > 0 ? v.s[0] : 0.0;
    const double t = static_cast<double>(v.m > v.n ? v.m : v.n) * 0x1.0p-52 * s0;
    return v.rank_cut * s0 > t ? v.rank_cut * s0 : t;
}

// Single block: filter factors phi and the regularisation actually used.
__global__ void recon_select_kernel(SvdDevView v, RegDev reg, int32_t *rank_out, double *alpha_out)
{
    __shared__ double scratch[16];
    __shared__ double sh_alpha;
    __shared__ int sh_rank;
    const int k = v.k;
    const double s0 = k > 0 ? v.s[0] : 0.0;
    const double rank_tol = rank_level(v);
    if (threadIdx.x == 0) {
        int kpos = 0;
        for (int l = 0; l < k; ++l) kpos += v.s[l] > rank_tol ? 1 : 0;
        // certified truncated path: only the trusted triplets may be used; a rank that needs more
        // is flagged (the serving engine then solves the request with the full SVD)
        const int kuse = v.tk && v.certified
                             ? (kpos < static_cast<int>(v.ctrl[kCtrlTrusted]) ? kpos : static_cast<int>(v.ctrl[kCtrlTrusted]))
                             : kpos;
        bool unresolved = false;
        int r = 0;
        double alpha = 0.0;
        if (reg.kind == 0) {
            const int want = reg.rank < 0 ? 0 : (reg.rank > kpos ? kpos : reg.rank);
            r = want > kuse ? kuse : want;
            unresolved = want > kuse;
        } else if (reg.kind == 1) {
            const double target = reg.tau * reg.delta;
            double res2 = v.work[v.cols];
            r = kpos;
            bool met = false;
            for (int l = 0; l < kuse; ++l) {
                res2 -= v.cvec[l] * v.cvec[l];
                const double res = __builtin_sqrt(res2 > 0.0 ? res2 : 0.0);
                if (res <= target) {
                    r = l + 1;
                    met = true;
                    break;
                }
            }
            if (!met && kuse < kpos) {
                r = kuse;
                unresolved = true;
            }
        }
        if (v.tk && v.certified) v.ctrl[kCtrlUnresolved] = unresolved ? 1u : 0u;
        sh_rank = r;
        sh_alpha = alpha;
    }
    __syncthreads();
    if (reg.kind == 2) {
        double alpha = reg.alpha;
        if (!(alpha > 0.0)) {
            // residual^2(alpha) = sum_l (alpha^2 / (s_l^2 + alpha^2))^2 c_l^2 + |q_perp|^2
            double cc = 0.0;
            for (int l = threadIdx.x; l < k; l += blockDim.x) cc = __builtin_fma(v.cvec[l], v.cvec[l], cc);
            cc = block_sum(cc, scratch);
            double qperp2 = v.work[v.cols] - cc;
            qperp2 = qperp2 > 0.0 ? qperp2 : 0.0;
            const double target2 = (reg.tau * reg.delta) * (reg.tau * reg.delta);
            double lo = log(s0 * 1e-16), hi = log(s0 * 1e4);
            auto f = [&](double la) {
                const double a2 = exp(2.0 * la);
                double acc = 0.0;
                for (int l = threadIdx.x; l < k; l += blockDim.x) {
                    const double g = a2 / (v.s[l] * v.s[l] + a2);
                    acc = __builtin_fma(g * g, v.cvec[l] * v.cvec[l], acc);
                }
                return block_sum(acc, scratch) + qperp2 - target2;
            };
            if (f(lo) >= 0.0) {
                alpha = exp(lo);
            } else if (f(hi) <= 0.0) {
                alpha = exp(hi);
            } else {
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (mid <= lo || mid >= hi) break;
                    if (f(mid) > 0.0) hi = mid; else lo = mid;
                }
                alpha = exp(0.5 * (lo + hi));
            }
        }
        if (threadIdx.x == 0) sh_alpha = alpha;
        __syncthreads();
    }
    const int r = sh_rank;
    const double alpha = sh_alpha;
    for (int l = threadIdx.x; l < k; l += blockDim.x) {
        double phi = 0.0;
        if (reg.kind == 2) {
            const double sl = v.s[l];
            phi = sl / (sl * sl + alpha * alpha);
        } else if (l < r) {
            phi = 1.0 / v.s[l];
        }
        v.phic[l] = phi * v.cvec[l];
    }
    if (threadIdx.x == 0) {
        if (rank_out) *rank_out = reg.kind == 2 ? 0 : r;
        if (alpha_out) *alpha_out = reg.kind == 2 ? alpha : 0.0;
    }
}

__global__ void recon_u1_kernel(SvdDevView v, double *__restrict__ u1)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < v.n; j += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int l = 0; l < v.k; ++l) acc = __builtin_fma(v.V[static_cast<size_t>(l) * v.n + j], v.phic[l], acc);
        u1[j] = acc * v.isig1[j];
    }
}

__global__ void recon_pred_kernel(SvdDevView v, const uint32_t *__restrict__ counts, double inv_n,
                                  const double *__restrict__ u1, const double *__restrict__ u0,
                                  double *__restrict__ pred)
{
    __shared__ double scratch[16];
    for (int i = blockIdx.x; i < v.m; i += gridDim.x) {
        const uint32_t *row = counts + static_cast<size_t>(i) * v.n_elem;
        double acc = 0.0;
        for (int j = threadIdx.x; j < v.n_elem; j += blockDim.x) {
            const int e = v.emap[j];
            const double uj = e >= 0 ? u1[e] : (u0 ? u0[-e - 1] : 0.0);
            acc = __builtin_fma(static_cast<double>(row[j]) * inv_n, uj, acc);
        }
        acc = block_sum(acc, scratch);
        if (threadIdx.x == 0) pred[i] = acc;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Products of the estimated measure (Section 5.2, items (i)-(iv))
// ---------------------------------------------------------------------------------------------
// Density estimator on the boundary cells (eq. rho omega1 MC with the cell indicators as weight
// functions): rho[i, j] = (counts[i, j] / N) / sigma_j, divided in that order.
__global__ void density_kernel(const uint32_t *__restrict__ counts, int m, int n_elem, double n_walks,
                               const double *__restrict__ sigma, double *__restrict__ rho)
{
    for (int i = blockIdx.y; i < m; i += gridDim.y) {
        const size_t base = static_cast<size_t>(i) * n_elem;
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_elem; j += gridDim.x * blockDim.x)
            rho[base + j] = static_cast<double>(counts[base + j]) / n_walks / sigma[j];
    }
}

// Average of the density over the points: one block per 64 cells, its 16 waves take every 16th
// row, then a fixed-order sum of the 16 partials.
__global__ __launch_bounds__(1024) void density_mean_kernel(const uint32_t *__restrict__ counts, int m, int n_elem,
                                                            double n_walks, const double *__restrict__ sigma,
                                                            double *__restrict__ mean)
{
    __shared__ double part[16][kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int j = blockIdx.x * kWave + lane;
    double acc = 0.0;
    if (j < n_elem) {
        const double sj = sigma[j];
        for (int i = w; i < m; i += 16)
            acc += static_cast<double>(counts[static_cast<size_t>(i) * n_elem + j]) / n_walks / sj;
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && j < n_elem) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += part[q][lane];
        mean[j] = t / static_cast<double>(m);
    }
}

// Eigenvalues lambda_f = s_f^2 of Lambda^nu = B B^T and the eigenfunction estimators on the Gamma_1
// cells.  The estimator of eq. eigenfunctions_MC, lambda_f^{-1/2} sum_i nu_i [u_f]_i rho_i, equals
// lambda_f^{-1/2} diag(sigma_1)^{-1/2} B^T u_f = diag(sigma_1)^{-1/2} v_f, which is what is formed here
// (no division by s_f).
__global__ void eigfun_kernel(SvdDevView v, int n_fun, double *__restrict__ lam, double *__restrict__ ef)
{
    for (int f = blockIdx.y; f < n_fun; f += gridDim.y) {
        if (lam && blockIdx.x == 0 && threadIdx.x == 0) lam[f] = v.s[f] * v.s[f];
        if (!ef) continue;
        const double *vf = v.V + static_cast<size_t>(f) * v.n;
        for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < v.n; l += gridDim.x * blockDim.x)
            ef[static_cast<size_t>(f) * v.n + l] = vf[l] * v.isig1[l];
    }
}

// u1 of every truncation r = 1..r_max (column r - 1).  Same filter factors and accumulation order
// as recon_select_kernel / recon_u1_kernel, so column r - 1 equals the rank-r reconstruction bit for
// bit.
__global__ void sweep_u1_kernel(SvdDevView v, int r_max, double *__restrict__ u1)
{
    const double lev = rank_level(v);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < v.n; j += gridDim.x * blockDim.x) {
        const double is = v.isig1[j];
        double acc = 0.0;
        for (int l = 0; l < r_max; ++l) {
            const double sl = v.s[l];
            if (sl > lev) acc = __builtin_fma(v.V[static_cast<size_t>(l) * v.n + j], (1.0 / sl) * v.cvec[l], acc);
            u1[static_cast<size_t>(l) * v.n + j] = acc * is;
        }
    }
}

// Rows of the sweep, 256 per block.  Per row: g0 = (counts/N)[:, Gamma_0] u0 (one wave per row),
// then for r = 0..r_max the projection p_r = U_r c_r, the data predicted at the point,
// g0 + p_r / nu (because (counts/N)[:, Gamma_1] u1^(r) = diag(nu)^{-1} B w_r = diag(nu)^{-1} U_r c_r),
// and the block's share of |q - p_r|^2, written to part[r * gridDim.x + block].
__global__ __launch_bounds__(256) void sweep_rows_kernel(SvdDevView v, const uint32_t *__restrict__ counts,
                                                         double inv_n, const double *__restrict__ u0, int r_max,
                                                         double *__restrict__ pred, double *__restrict__ part)
{
    __shared__ double g0s[256];
    __shared__ double red[4][kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int row0 = blockIdx.x * 256;
    for (int t = w; t < 256; t += 4) {
        const int i = row0 + t;
        double acc = 0.0;
        if (i < v.m && u0) {
            const uint32_t *row = counts + static_cast<size_t>(i) * v.n_elem;
            for (int l = lane; l < v.n0; l += kWave)
                acc = __builtin_fma(static_cast<double>(row[v.g0idx[l]]) * inv_n, u0[l], acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) g0s[t] = acc;
    }
    __syncthreads();
    const int i = row0 + static_cast<int>(threadIdx.x);
    const bool live = i < v.m;
    const double lev = rank_level(v);
    const double qi = live ? v.q[i] : 0.0, nui = live ? v.nu[i] : 1.0, g0 = g0s[threadIdx.x];
    double p = 0.0;
    for (int r = 0; r <= r_max; ++r) {
        if (r > 0) {
            const int l = r - 1;
            if (live && v.s[l] > lev) p = __builtin_fma(v.U[static_cast<size_t>(l) * v.m + i], v.cvec[l], p);
            if (live && pred) pred[static_cast<size_t>(l) * v.m + i] = g0 + p / nui;
        }
        const double e = live ? qi - p : 0.0;
        const double e2 = wave_sum(e * e);
        if (lane == 0) red[w][r & (kWave - 1)] = e2;
        if ((r & (kWave - 1)) == kWave - 1 || r == r_max) {  // uniform over the block
            __syncthreads();
            const int t = static_cast<int>(threadIdx.x);
            if (t <= (r & (kWave - 1)))
                part[static_cast<size_t>((r & ~(kWave - 1)) + t) * gridDim.x + blockIdx.x] =
                    ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
            __syncthreads();
        }
    }
}

__global__ void sweep_resid_kernel(const double *__restrict__ part, int nb, int r_max, double *__restrict__ resid)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r <= r_max; r += gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += part[static_cast<size_t>(r) * nb + b];
        resid[r] = __builtin_sqrt(t);
    }
}

}  // namespace

int gram_order(int cols)
{
    if (cols < 1 || cols > kGramGridMaxCols) return 0;
    if (cols > kGramMaxCols) return (cols + 63) & ~63;  // device-wide path
    return cols <= 64 ? 64 : (cols <= 128 ? 128 : 192);
}

static int coop_blocks(const JacobiShape &sh, int npairs, int n_cu)
{
    int per_cu = 0;
    if (!sh.fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sh.fn, sh.threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int maxres = per_cu * n_cu;
    npairs = npairs < 1 ? 1 : npairs;
    return npairs < maxres ? npairs : maxres;
}

int svd_coop_grid(int rows, int colsp, int n_cu)
{
    const JacobiShape sh = jacobi_shape(rows, colsp);
    return coop_blocks(sh, (colsp / (2 * sh.bw) + sh.gpb - 1) / sh.gpb, n_cu);
}

// assemble -> [Gram path: G, factor, Jacobi on the factor, norms, V side, U side, check, accept]
// -> Hestenes path on A (skipped when the Gram result was accepted) -> norms -> scatter.
hipError_t svd_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, int coop_grid, int n_cu,
                      hipStream_t stream, SvdEvents *ev)
{
    if (ev) {
        ev->jac_recorded = false;
        (void)hipEventRecord(ev->all0, stream);
    }
    const size_t total = static_cast<size_t>(v.rows) * v.colsp;
    int g = static_cast<int>((total + 255) / 256);
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    assemble_kernel<<<g, 256, 0, stream>>>(v, counts, inv_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t *skip = nullptr;
    const bool grid = v.np > kGramMaxCols;
    // the device-wide Jacobi needs all of its P = np / 16 workgroups resident on the stream's CUs
    bool gram = v.np > 0;
    int grid_wgs = 0;  // workgroups of the device-wide Jacobi: all P block pairs resident, or fewer
    if (grid) {
        int per_cu = 0;
        const void *fn = grid_jacobi_fn(v.np);
        if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kGridThreads, 0) != hipSuccess ||
            per_cu < 1)
            gram = false;
        grid_wgs = std::min(v.np / (2 * kGridBW), per_cu * std::max(n_cu, 1));
    }
    if (gram) {
        const long rl = v.rows, cl = v.cols, kl = v.k, npl = v.np;
        double *vs = v.trans ? v.U : v.V;        // the eigenvector side (cols x k)
        double *ys = v.trans ? v.V : v.U;        // the other side (rows x k)
        // G = A^T A (np x np; the columns past colsp are zero)
        if ((e = gemm({v.A, rl, 1, v.A, 1, rl, nullptr, v.G, npl, v.colsp, v.colsp, v.rows, nullptr, 0, 0, v.np, v.np},
                      stream)) != hipSuccess)
            return e;
        if (grid) {
            if ((e = chol_pivoted(v, stream)) != hipSuccess) return e;
            if ((e = hipGetLastError()) != hipSuccess) return e;
            GridJacobiArgs J{v.L, v.zs, v.gnrm, v.gctl, v.info + 2, v.np, v.np / (2 * kGridBW)};
            void *args[] = {&J};
            if (ev) (void)hipEventRecord(ev->jac0, stream);
            e = hipLaunchCooperativeKernel(grid_jacobi_fn(v.np), dim3(grid_wgs), dim3(kGridThreads), args, 0, stream);
            if (e != hipSuccess) return e;
            if (ev) {
                (void)hipEventRecord(ev->jac1, stream);
                ev->jac_recorded = true;
            }
        } else {
            if (v.np == 64) gram_chol_kernel<1><<<1, 1024, 0, stream>>>(v);
            else if (v.np == 128) gram_chol_kernel<2><<<1, 1024, 0, stream>>>(v);
            else gram_chol_kernel<3><<<1, 1024, 0, stream>>>(v);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            // the factor's Jacobi in one workgroup (zs = the rotated columns' norms)
            if (ev) (void)hipEventRecord(ev->jac0, stream);
            if (v.np == 64) e = launch_gram_jacobi1<1>(v.L, v.zs, v.info + 2, stream);
            else if (v.np == 128) e = launch_gram_jacobi1<2>(v.L, v.zs, v.info + 2, stream);
            else e = launch_gram_jacobi1<3>(v.L, v.zs, v.info + 2, stream);
            if (e != hipSuccess) return e;
            if (ev) {
                (void)hipEventRecord(ev->jac1, stream);
                ev->jac_recorded = true;
            }
        }
        gram_vside_kernel<<<v.np, 64, 0, stream>>>(v);
        // Ys = A Vs diag(1 / s) and C = Ys^T Ys (k x k, in G)
        const GemmArgs yside{v.A, 1, rl, vs, 1, cl, nullptr, ys, rl, v.rows, v.k, v.cols, v.s, v.k, 3};
        const GemmArgs cross{ys, rl, 1, ys, 1, rl, nullptr, v.G, kl, v.k, v.k, v.rows, nullptr, 0, 0};
        if ((e = gemm(yside, stream)) != hipSuccess) return e;
        const size_t kk = static_cast<size_t>(v.k) * v.k;
        const int gk = static_cast<int>(std::min<size_t>(4096, (kk + 255) / 256));
        if (grid) {  // first-order correction of the eigenvector side, then the other side again
            if ((e = gemm(cross, stream)) != hipSuccess) return e;
            const size_t nk = static_cast<size_t>(v.cols) * v.k;
            gram_fix_kernel<<<gk, 256, 0, stream>>>(v, v.G, v.L);
            if ((e = gemm({vs, 1, cl, v.L, 1, kl, nullptr, v.G, cl, v.cols, v.k, v.k, nullptr, 0, 0}, stream)) != hipSuccess)
                return e;
            copy_f64_kernel<<<static_cast<int>(std::min<size_t>(4096, (nk + 255) / 256)), 256, 0, stream>>>(vs, v.G, nk);
            if ((e = gemm(yside, stream)) != hipSuccess) return e;
        }
        if ((e = gemm(cross, stream)) != hipSuccess) return e;
        gram_crit_kernel<<<gk, 256, 0, stream>>>(v, v.G);
        // residual certificate: C = A^T Ys (cols x k) in G
        if ((e = gemm({v.A, rl, 1, ys, 1, rl, nullptr, v.G, cl, v.cols, v.k, v.rows, nullptr, 0, 0}, stream)) != hipSuccess)
            return e;
        gram_resid_kernel<<<std::min(v.k, 2048), 256, 0, stream>>>(v, v.G);
        gram_accept_kernel<<<1, 64, 0, stream>>>(v);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        skip = v.ctrl + kCtrlGramOk;
    }
    {
        const JacobiShape sh = jacobi_shape(v.rows, v.colsp);
        if (!sh.fn) return hipErrorInvalidValue;
        JacobiArgs J{v.A, v.W, v.rows, v.rows, v.colsp, v.tol, v.rot, v.ctrl + kCtrlBarrier, v.ctrl + kCtrlError,
                     v.info, skip};
        void *args[] = {&J};
        e = hipLaunchCooperativeKernel(sh.fn, dim3(coop_grid), dim3(sh.threads), args, 0, stream);
        if (e != hipSuccess) return e;
    }
    const int gc = v.cols < 1 ? 1 : (v.cols > 2048 ? 2048 : v.cols);
    colnorm_kernel<<<gc, 256, 0, stream>>>(v.A, v.rows, v.rows, v.cols, v.work, skip);
    scatter_kernel<<<gc, 256, 0, stream>>>(v, skip);
    if (ev) (void)hipEventRecord(ev->all1, stream);
    return hipGetLastError();
}

// Residual of each computed triplet of the truncated path, |A v_l - s_l u_l| (W = A V, rows x k),
// into zt[l]; one block per triplet.
__global__ void trip_resid_kernel(SvdDevView v, const double *__restrict__ W)
{
    __shared__ double scratch[16];
    const int l = blockIdx.x;
    if (l >= v.k) return;
    const double *u = (v.trans ? v.V : v.U) + static_cast<size_t>(l) * v.rows;
    const double *w = W + static_cast<size_t>(l) * v.rows;
    const double sl = v.s[l];
    double acc = 0.0;
    for (int r = threadIdx.x; r < v.rows; r += blockDim.x) {
        const double d = w[r] - sl * u[r];
        acc = __builtin_fma(d, d, acc);
    }
    acc = block_sum(acc, scratch);
    if (threadIdx.x == 0) v.zt[l] = __builtin_sqrt(acc);
}

// The trusted prefix: the leading triplets whose residual is at most 2^-35 s_1 (the bound the full
// SVD's acceptance uses), stopping at the first that misses it.
__global__ void trust_kernel(SvdDevView v)
{
    if (threadIdx.x != 0) return;
    const double lim = 0x1.0p-35 * (v.k > 0 ? v.s[0] : 0.0);
    int t = 0;
    while (t < v.k && v.zt[t] <= lim) ++t;
    v.ctrl[kCtrlTrusted] = static_cast<uint32_t>(t);
}

hipError_t tsvd_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, uint64_t seed, hipStream_t stream)
{
    if (v.tk != 64 && v.tk != 128) return hipErrorInvalidValue;
    const size_t total = static_cast<size_t>(v.rows) * v.colsp;
    int g = static_cast<int>((total + 255) / 256);
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    assemble_kernel<<<g, 256, 0, stream>>>(v, counts, inv_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int K = v.tk;
    auto chol = [&](double *G, double *L) {
        SvdDevView w = v;
        w.G = G;
        w.L = L;
        if (K == 64) gram_chol_kernel<1><<<1, 1024, 0, stream>>>(w);
        else gram_chol_kernel<2><<<1, 1024, 0, stream>>>(w);
    };
    auto jac = [&](double *X, double *z) {
        if (K == 64) (void)launch_gram_jacobi1<1>(X, z, v.info, stream);
        else (void)launch_gram_jacobi1<2>(X, z, v.info, stream);
    };
    // certified mode: the residual of every computed triplet (W = A V_A in Y, which is free by then)
    // and the trusted prefix
    auto certify = [&]() -> hipError_t {
        if (!v.certified) return hipGetLastError();
        const double *colside = v.trans ? v.U : v.V;
        hipError_t e2 = gemm({v.A, 1, static_cast<long>(v.rows), colside, 1, static_cast<long>(v.cols), nullptr, v.Y,
                              static_cast<long>(v.rows), v.rows, v.k, v.cols, nullptr, 0, 0},
                             stream);
        if (e2 != hipSuccess) return e2;
        trip_resid_kernel<<<v.k, 256, 0, stream>>>(v, v.Y);
        trust_kernel<<<1, 64, 0, stream>>>(v);
        return hipGetLastError();
    };
    if (v.cols <= K) {  // the Gram path of A with the one-workgroup Jacobi
        const int nt = K / 16;
        gram_kernel<<<(nt * nt + 3) / 4, 256, 0, stream>>>(v);
        chol(v.G, v.L);
        jac(v.L, v.zs);
        gram_vside_kernel<<<K, 64, 0, stream>>>(v);
        const int ty = ((v.rows + 15) / 16) * ((v.k + 15) / 16);
        gram_yside_kernel<<<(ty + 3) / 4, 256, 0, stream>>>(v);
        return certify();
    }
    const long R = v.rows, Cc = v.cols, Kl = K;
    const int sg = static_cast<int>(std::min<size_t>(4096, (static_cast<size_t>(Cc) * K + 255) / 256));
    sketch_kernel<<<sg, 256, 0, stream>>>(v.Om, v.cols, K, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    // Y = A Om
    if ((e = gemm({v.A, 1, R, v.Om, 1, Cc, nullptr, v.Y, R, v.rows, K, v.cols, nullptr, 0, 0}, stream)) != hipSuccess) return e;
    // Orthonormal basis of range(Y): Y^T Y = Lt Lt^T, Jacobi -> eigenvectors Lt / zt and eigenvalues
    // zt^2, Q = Y Lt diag(1 / zt^2) (columns with zt <= 1e-7 max zt dropped)
    auto orth = [&]() -> hipError_t {
        hipError_t e2 = gemm({v.Y, R, 1, v.Y, 1, R, nullptr, v.Gt, Kl, K, K, v.rows, nullptr, 0, 0}, stream);
        if (e2 != hipSuccess) return e2;
        chol(v.Gt, v.Lt);
        jac(v.Lt, v.zt);
        return gemm({v.Y, 1, R, v.Lt, 1, Kl, nullptr, v.Q, R, v.rows, K, K, v.zt, K, 1}, stream);
    };
    if ((e = orth()) != hipSuccess) return e;
    // kPowerIters subspace iterations Y = A (A^T Q), each followed by orth (Om holds A^T Q)
    for (int it = 0; it < kPowerIters; ++it) {
        if ((e = gemm({v.A, R, 1, v.Q, 1, R, nullptr, v.Om, Cc, v.cols, K, v.rows, nullptr, 0, 0}, stream)) != hipSuccess) return e;
        if ((e = gemm({v.A, 1, R, v.Om, 1, Cc, nullptr, v.Y, R, v.rows, K, v.cols, nullptr, 0, 0}, stream)) != hipSuccess) return e;
        if ((e = orth()) != hipSuccess) return e;
    }
    // C = Q^T A, then the Gram path of C^T: G = C C^T, factor, Jacobi
    if ((e = gemm({v.Q, R, 1, v.A, 1, R, nullptr, v.Cm, Kl, K, v.cols, v.rows, nullptr, 0, 0}, stream)) != hipSuccess) return e;
    if ((e = gemm({v.Cm, 1, Kl, v.Cm, Kl, 1, nullptr, v.G, Kl, K, K, v.cols, nullptr, 0, 0}, stream)) != hipSuccess) return e;
    chol(v.G, v.L);
    jac(v.L, v.zs);
    rank_kernel<<<1, 256, 0, stream>>>(v.zs, K, v.k, v.s, v.perm);
    double *rowside = v.trans ? v.V : v.U;  // rows x k
    double *colside = v.trans ? v.U : v.V;  // cols x k
    // U_A = Q E / s (E = L[:, perm] / zs[perm]), V_A = C^T E / s = C^T L[:, perm] / zs^2
    if ((e = gemm({v.Q, 1, R, v.L, 1, Kl, v.perm, rowside, R, v.rows, v.k, K, v.zs, K, 2}, stream)) != hipSuccess) return e;
    if ((e = gemm({v.Cm, Kl, 1, v.L, 1, Kl, v.perm, colside, Cc, v.cols, v.k, K, v.zs, K, 1}, stream)) != hipSuccess) return e;
    return certify();
}

hipError_t recon_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, const double *uD,
                        const double *u0, const RegDev &reg, double *u1, double *pred, int32_t *rank_out,
                        double *alpha_out, hipStream_t stream)
{
    const int gm = v.m < 1 ? 1 : (v.m > 2048 ? 2048 : v.m);
    const int gk = v.k < 1 ? 1 : (v.k > 2048 ? 2048 : v.k);
    recon_q_kernel<<<gm, 256, 0, stream>>>(v, counts, inv_n, uD, u0);
    recon_c_kernel<<<gk, 256, 0, stream>>>(v);
    recon_select_kernel<<<1, 256, 0, stream>>>(v, reg, rank_out, alpha_out);
    const int gn = (v.n + 255) / 256 < 1 ? 1 : (v.n + 255) / 256;
    recon_u1_kernel<<<gn, 256, 0, stream>>>(v, u1);
    if (pred) recon_pred_kernel<<<gm, 256, 0, stream>>>(v, counts, inv_n, u1, u0, pred);
    return hipGetLastError();
}

hipError_t density_launch(const uint32_t *counts, int m, int n_elem, uint64_t n_walks, const double *sigma,
                          double *rho, double *mean, hipStream_t stream)
{
    const double n = static_cast<double>(n_walks);
    if (rho) {
        const dim3 grid((n_elem + 255) / 256 > 64 ? 64 : (n_elem + 255) / 256, m > 32768 ? 32768 : m);
        density_kernel<<<grid, 256, 0, stream>>>(counts, m, n_elem, n, sigma, rho);
    }
    if (mean) density_mean_kernel<<<(n_elem + kWave - 1) / kWave, 1024, 0, stream>>>(counts, m, n_elem, n, sigma, mean);
    return hipGetLastError();
}

hipError_t eigfun_launch(const SvdDevView &v, int n_fun, double *lam, double *ef, hipStream_t stream)
{
    if (n_fun <= 0) return hipSuccess;
    const dim3 grid((v.n + 255) / 256 > 64 ? 64 : (v.n + 255) / 256, n_fun > 32768 ? 32768 : n_fun);
    eigfun_kernel<<<grid, 256, 0, stream>>>(v, n_fun, lam, ef);
    return hipGetLastError();
}

size_t sweep_part_words(const SvdDevView &v, int r_max)
{
    return static_cast<size_t>((v.m + 255) / 256) * static_cast<size_t>(r_max + 1);
}

hipError_t sweep_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, const double *uD,
                        const double *u0, int r_max, double *u1, double *pred, double *resid, hipStream_t stream)
{
    const int gm = v.m < 1 ? 1 : (v.m > 2048 ? 2048 : v.m);
    const int gk = v.k < 1 ? 1 : (v.k > 2048 ? 2048 : v.k);
    recon_q_kernel<<<gm, 256, 0, stream>>>(v, counts, inv_n, uD, u0);
    recon_c_kernel<<<gk, 256, 0, stream>>>(v);
    const int gn = (v.n + 255) / 256 < 1 ? 1 : (v.n + 255) / 256;
    sweep_u1_kernel<<<gn, 256, 0, stream>>>(v, r_max, u1);
    if (pred || resid) {
        // the block partials of the residual norms go to the work matrix, free once the factors exist
        const int nb = (v.m + 255) / 256;
        sweep_rows_kernel<<<nb, 256, 0, stream>>>(v, counts, inv_n, u0, r_max, pred, v.A);
        if (resid) sweep_resid_kernel<<<(r_max + 256) / 256, 256, 0, stream>>>(v.A, nb, r_max, resid);
    }
    return hipGetLastError();
}

}  // namespace wos
