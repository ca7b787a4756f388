// linalg_kernels.hip -- FP64 spectral end of the path on gfx950.
//
//   assemble:    B = diag(nu) (counts / N)[:, Gamma_1] diag(sigma_1)^{-1/2}  (column-major work copy)
//   jacobi:      one-sided (Hestenes) Jacobi SVD of the work copy, all column pairs of a round in
//                parallel (round-robin ordering), one cooperative grid with a device-wide barrier
//                between rounds and a convergence test at the end of every sweep
//   finalize:    column norms -> singular values, descending order, U and V scattered
//   reconstruct: q = nu (u^D - H_0 u^0), c = U^T q, filter factors phi (TSVD rank, discrepancy rule
//                or Tikhonov), u_1 = sigma^{-1/2} V (phi c), predicted data H_1 u_1 + H_0 u^0.
// Matrix work is small next to the walks (a 1024 x 192 B at the annulus workload), so every kernel
// is written for latency: few launches, wave-level shuffles, no host round trips.
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
    const size_t wtot = static_cast<size_t>(v.colsp) * v.colsp;
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < wtot;
         e += static_cast<size_t>(gridDim.x) * blockDim.x)
        v.W[e] = (e % v.colsp) == (e / v.colsp) ? 1.0 : 0.0;
    if (blockIdx.x == 0 && threadIdx.x < kMaxSweeps + 2) {
        if (threadIdx.x < kMaxSweeps) v.rot[threadIdx.x] = 0u;
        else v.ctrl[threadIdx.x - kMaxSweeps] = 0u;  // barrier counter, error flag
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) v.info[0] = 0;
}

// Device-wide barrier for a cooperative grid: arrival counter with a generation target and a
// bounded spin (an expired spin sets the error flag instead of hanging).
__device__ __forceinline__ void grid_barrier(uint32_t *counter, uint32_t *err, uint32_t nblocks,
                                             uint32_t &gen)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        gen += 1;
        const uint32_t target = gen * nblocks;
        __threadfence();
        atomicAdd(counter, 1u);
        uint32_t spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(4);
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            if (++spins > (1u << 26)) {
                atomicExch(err, 1u);
                break;
            }
        }
        __threadfence();
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


// Round-robin pair K of inner round IR of an 8-column block pair, as compile-time constants.
template <int IR, int K> struct P8 {
    static constexpr int a = K == 0 ? 0 : ((K - 1 + IR) % 7) + 1;
    static constexpr int b = ((6 - K + IR) % 7) + 1;
    static constexpr int p = a < b ? a : b;
    static constexpr int q = a < b ? b : a;
};

// DPP move of a double (both 32-bit halves); lanes outside row_mask receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes with VALU data movement only: quad permutes, half-row and row mirrors,
// then row broadcasts 15 and 31 accumulate rows into row 3; lane 63 holds the total.
__device__ __forceinline__ double wave_total(double v)
{
    v += dpp64<0xB1>(v);        // quad_perm (1, 0, 3, 2)
    v += dpp64<0x4E>(v);        // quad_perm (2, 3, 0, 1)
    v += dpp64<0x141>(v);       // row_half_mirror
    v += dpp64<0x140>(v);       // row_mirror
    v += dpp64<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
    v += dpp64<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

template <int IR, int K, int R>
__device__ __forceinline__ double pair_dot(const double (&x)[R][8])
{
    constexpr int p = P8<IR, K>::p, q = P8<IR, K>::q;
    double sg = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) sg = __builtin_fma(x[i][p], x[i][q], sg);
    return sg;
}

template <int IR, int K, int R, int RW>
__device__ __forceinline__ void pair_rotate(double (&x)[R][8], double (&w)[RW][8], double (&n2)[8], double c,
                                            double sn, double t, double g)
{
    constexpr int p = P8<IR, K>::p, q = P8<IR, K>::q;
    if (sn != 0.0) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const double xp = x[i][p], xq = x[i][q];
            x[i][p] = c * xp - sn * xq;
            x[i][q] = sn * xp + c * xq;
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const double wp = w[i][p], wq = w[i][q];
            w[i][p] = c * wp - sn * wq;
            w[i][q] = sn * wp + c * wq;
        }
        // column norms after the rotation that zeroes g (Hestenes): |x_p|^2 - t g, |x_q|^2 + t g
        n2[p] = n2[p] - t * g;
        n2[q] = n2[q] + t * g;
    }
}

// Sums NV per-wave totals across the waves of the block: lane 0 of each wave writes its totals,
// one barrier, then every thread adds the wave totals in a fixed order (identical in all waves).
template <int NV>
__device__ __forceinline__ void block_totals(double (&val)[NV], double (*buf)[16], int nw)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < NV; ++e) val[e] = wave_total(val[e]);
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < NV; ++e) buf[wid][e] = val[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        double acc = 0.0;
        for (int w2 = 0; w2 < nw; ++w2) acc += buf[w2][e];
        val[e] = acc;
    }
}

// One inner round IR of the 8-column sweep: the 4 dot products g = x_p . x_q from the thread's
// rows, block totals (one barrier), rotation parameters from the tracked norms, two-term updates
// of the A rows and W rows held in registers.
template <int IR, int R, int RW>
__device__ __forceinline__ void inner_round8(double (&x)[R][8], double (&w)[RW][8], double (&n2)[8],
                                             double (*part)[16][16], int &nrot, double tol2, int nw)
{
    double g[4] = {pair_dot<IR, 0, R>(x), pair_dot<IR, 1, R>(x), pair_dot<IR, 2, R>(x), pair_dot<IR, 3, R>(x)};
    block_totals<4>(g, part[IR & 1], nw);
    const double a[4] = {n2[P8<IR, 0>::p], n2[P8<IR, 1>::p], n2[P8<IR, 2>::p], n2[P8<IR, 3>::p]};
    const double b[4] = {n2[P8<IR, 0>::q], n2[P8<IR, 1>::q], n2[P8<IR, 2>::q], n2[P8<IR, 3>::q]};
    double c[4], sn[4], tt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = 1.0;
        sn[k] = 0.0;
        tt[k] = 0.0;
        if (g[k] != 0.0 && g[k] * g[k] > tol2 * a[k] * b[k]) {
            const double zeta = (b[k] - a[k]) / (2.0 * g[k]);
            tt[k] = (zeta >= 0.0 ? 1.0 : -1.0) / (__builtin_fabs(zeta) + __builtin_sqrt(1.0 + zeta * zeta));
            c[k] = 1.0 / __builtin_sqrt(1.0 + tt[k] * tt[k]);
            sn[k] = c[k] * tt[k];
            ++nrot;
        }
    }
    pair_rotate<IR, 0, R, RW>(x, w, n2, c[0], sn[0], tt[0], g[0]);
    pair_rotate<IR, 1, R, RW>(x, w, n2, c[1], sn[1], tt[1], g[1]);
    pair_rotate<IR, 2, R, RW>(x, w, n2, c[2], sn[2], tt[2], g[2]);
    pair_rotate<IR, 3, R, RW>(x, w, n2, c[3], sn[3], tt[3], g[3]);
}

template <int R, int RW, int... IR>
__device__ __forceinline__ void inner_sweep8(double (&x)[R][8], double (&w)[RW][8], double (&n2)[8],
                                             double (*part)[16][16], int &nrot, double tol2, int nw,
                                             std::integer_sequence<int, IR...>)
{
    (inner_round8<IR, R, RW>(x, w, n2, part, nrot, tol2, nw), ...);
}

// Blocked one-sided Jacobi (Hestenes) with register-resident block pairs.
//
// Columns are grouped in blocks of 4; the blocks meet pairwise in round-robin order, one block pair
// per workgroup per round, with a device-wide barrier between rounds.  A workgroup loads the 8
// columns of its pair, rows of A and rows of W alike, into registers (thread t holds rows t, t + T,
// ...), computes the 8 column norms, then runs one cyclic sweep over the 8 columns: in each of 7
// inner rounds, 4 disjoint pairs get g = x_p . x_q from a DPP + LDS reduction and a pair with
// g^2 > tol^2 |x_p|^2 |x_q|^2 is rotated by the plane rotation that zeroes g, applied as two-term
// updates (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q) to its A and W rows; the norms follow the
// rotation analytically and are recomputed from the columns at the next load.  Fresh dot products
// and two-term updates keep small columns accurate relative to their own size.  All waves compute
// the same sums in the same order, so every thread takes the same decisions.  A sweep without
// rotations ends the iteration.
template <int R, int RW, int T>
__global__ __launch_bounds__(T) void bjacobi_kernel(SvdDevView v)
{
    __shared__ double part[2][16][16];
    __shared__ int cols[8];
    const int nblk = v.colsp / 4;
    const int npairs = nblk / 2;
    const int ld = v.rows;
    const int ldw = v.colsp;
    constexpr int nw = T >> 6;
    const double tol2 = v.tol * v.tol;
    uint32_t gen = 0;
    uint32_t *bar = v.ctrl;
    uint32_t *err = v.ctrl + 1;
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        for (int t = 0; t < nblk - 1; ++t) {
            for (int pi = blockIdx.x; pi < npairs; pi += gridDim.x) {
                int P, Qb;
                pair_of(t, pi, nblk, P, Qb);
                if (threadIdx.x < 8) cols[threadIdx.x] = threadIdx.x < 4 ? P * 4 + threadIdx.x : Qb * 4 + threadIdx.x - 4;
                __syncthreads();
                double x[R][8], w[RW][8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const double *ca = v.A + static_cast<size_t>(cols[j]) * ld;
                    const double *cw = v.W + static_cast<size_t>(cols[j]) * ldw;
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const int r = threadIdx.x + i * T;
                        x[i][j] = r < ld ? ca[r] : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < RW; ++i) {
                        const int r = threadIdx.x + i * T;
                        w[i][j] = r < ldw ? cw[r] : 0.0;
                    }
                }
                double n2[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < R; ++i) acc = __builtin_fma(x[i][j], x[i][j], acc);
                    n2[j] = acc;
                }
                block_totals<8>(n2, part[1], nw);
                int nrot = 0;
                inner_sweep8<R, RW>(x, w, n2, part, nrot, tol2, nw, std::make_integer_sequence<int, 7>{});
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    double *ca = v.A + static_cast<size_t>(cols[j]) * ld;
                    double *cw = v.W + static_cast<size_t>(cols[j]) * ldw;
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const int r = threadIdx.x + i * T;
                        if (r < ld) ca[r] = x[i][j];
                    }
#pragma unroll
                    for (int i = 0; i < RW; ++i) {
                        const int r = threadIdx.x + i * T;
                        if (r < ldw) cw[r] = w[i][j];
                    }
                }
                if (threadIdx.x == 0 && nrot) atomicAdd(&v.rot[sweep], static_cast<uint32_t>(nrot));
                __syncthreads();
            }
            grid_barrier(bar, err, gridDim.x, gen);
        }
        const uint32_t rotated = __hip_atomic_load(&v.rot[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t failed = __hip_atomic_load(err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (rotated == 0u || failed) {
            ++sweep;
            break;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.info[0] = sweep;
        v.info[1] = static_cast<int32_t>(__hip_atomic_load(err, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) |
                    (sweep >= kMaxSweeps && v.rot[kMaxSweeps - 1] != 0u ? 2 : 0);
    }
}

// Launch shape by the size of the work matrix: T threads, R rows of A and RW rows of W each.
struct JacobiShape {
    const void *fn;
    int threads;
};
#define WOS_BJ(R, RW, T) JacobiShape{reinterpret_cast<const void *>(&bjacobi_kernel<R, RW, T>), T}
static JacobiShape bjacobi_shape(int rows, int colsp)
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
    return {nullptr, 0};
}
#undef WOS_BJ

__global__ void norms_kernel(SvdDevView v)
{
    __shared__ double scratch[16];
    for (int c = blockIdx.x; c < v.cols; c += gridDim.x) {
        const double *a = v.A + static_cast<size_t>(c) * v.rows;
        double acc = 0.0;
        for (int r = threadIdx.x; r < v.rows; r += blockDim.x) acc = __builtin_fma(a[r], a[r], acc);
        acc = block_sum(acc, scratch);
        if (threadIdx.x == 0) v.work[c] = __builtin_sqrt(acc);
        __syncthreads();
    }
}

__global__ void scatter_kernel(SvdDevView v)
{
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

// Single block: filter factors phi and the regularisation actually used.
__global__ void recon_select_kernel(SvdDevView v, RegDev reg, int32_t *rank_out, double *alpha_out)
{
    __shared__ double scratch[16];
    __shared__ double sh_alpha;
    __shared__ int sh_rank;
    const int k = v.k;
    const double s0 = k > 0 ? v.s[0] : 0.0;
    const double rank_tol = static_cast<double>(v.m > v.n ? v.m : v.n) * 0x1.0p-52 * s0;
    if (threadIdx.x == 0) {
        int kpos = 0;
        for (int l = 0; l < k; ++l) kpos += v.s[l] > rank_tol ? 1 : 0;
        int r = 0;
        double alpha = 0.0;
        if (reg.kind == 0) {
            r = reg.rank < 0 ? 0 : (reg.rank > kpos ? kpos : reg.rank);
        } else if (reg.kind == 1) {
            const double target = reg.tau * reg.delta;
            double res2 = v.work[v.cols];
            r = kpos;
            for (int l = 0; l < kpos; ++l) {
                res2 -= v.cvec[l] * v.cvec[l];
                const double res = __builtin_sqrt(res2 > 0.0 ? res2 : 0.0);
                if (res <= target) {
                    r = l + 1;
                    break;
                }
            }
        }
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

}  // namespace

hipError_t svd_launch(const SvdDevView &v, const uint32_t *counts, double inv_n, int coop_grid,
                      hipStream_t stream)
{
    const size_t total = static_cast<size_t>(v.rows) * v.colsp;
    int g = static_cast<int>((total + 255) / 256);
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    assemble_kernel<<<g, 256, 0, stream>>>(v, counts, inv_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        SvdDevView vv = v;
        void *args[] = {&vv};
        const JacobiShape sh = bjacobi_shape(v.rows, v.colsp);
        if (!sh.fn) return hipErrorInvalidValue;
        e = hipLaunchCooperativeKernel(sh.fn, dim3(coop_grid), dim3(sh.threads), args, 0, stream);
        if (e != hipSuccess) return e;
    }
    const int gc = v.cols < 1 ? 1 : (v.cols > 2048 ? 2048 : v.cols);
    norms_kernel<<<gc, 256, 0, stream>>>(v);
    scatter_kernel<<<gc, 256, 0, stream>>>(v);
    return hipGetLastError();
}

int svd_coop_grid(int rows, int colsp, int n_cu)
{
    int per_cu = 0;
    const JacobiShape sh = bjacobi_shape(rows, colsp);
    if (!sh.fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sh.fn, sh.threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int maxres = per_cu * n_cu;
    int npairs = colsp / 8;
    if (npairs < 1) npairs = 1;
    return npairs < maxres ? npairs : maxres;
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

}  // namespace wos
