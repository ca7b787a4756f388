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

__device__ __forceinline__ void pair_of(int t, int i, int colsp, int &p, int &q)
{
    const int m1 = colsp - 1;
    int a, b;
    if (i == 0) {
        a = 0;
    } else {
        a = ((i - 1 + t) % m1) + 1;
    }
    b = ((colsp - 2 - i + t) % m1) + 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__global__ __launch_bounds__(256) void jacobi_kernel(SvdDevView v)
{
    __shared__ double scratch[3 * 16];
    __shared__ double cs[2];
    __shared__ int flag;
    const int npairs = v.colsp / 2;
    const int ld = v.rows;
    uint32_t gen = 0;
    uint32_t *bar = v.ctrl;
    uint32_t *err = v.ctrl + 1;
    int sweep = 0;
    for (; sweep < kMaxSweeps; ++sweep) {
        for (int t = 0; t < v.colsp - 1; ++t) {
            for (int pi = blockIdx.x; pi < npairs; pi += gridDim.x) {
                int p, q;
                pair_of(t, pi, v.colsp, p, q);
                double *ap = v.A + static_cast<size_t>(p) * ld;
                double *aq = v.A + static_cast<size_t>(q) * ld;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = threadIdx.x; r < v.rows; r += blockDim.x) {
                    const double x = ap[r], y = aq[r];
                    al = __builtin_fma(x, x, al);
                    be = __builtin_fma(y, y, be);
                    ga = __builtin_fma(x, y, ga);
                }
                block_sum3(al, be, ga, scratch);
                if (threadIdx.x == 0) {
                    int rot = 0;
                    if (ga != 0.0 && __builtin_fabs(ga) > v.tol * __builtin_sqrt(al) * __builtin_sqrt(be)) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) /
                                          (__builtin_fabs(zeta) + __builtin_sqrt(1.0 + zeta * zeta));
                        const double c = 1.0 / __builtin_sqrt(1.0 + tt * tt);
                        cs[0] = c;
                        cs[1] = c * tt;
                        rot = 1;
                        atomicAdd(&v.rot[sweep], 1u);
                    }
                    flag = rot;
                }
                __syncthreads();
                if (flag) {
                    const double c = cs[0], s = cs[1];
                    for (int r = threadIdx.x; r < v.rows; r += blockDim.x) {
                        const double x = ap[r], y = aq[r];
                        ap[r] = c * x - s * y;
                        aq[r] = s * x + c * y;
                    }
                    double *wp = v.W + static_cast<size_t>(p) * v.colsp;
                    double *wq = v.W + static_cast<size_t>(q) * v.colsp;
                    for (int r = threadIdx.x; r < v.colsp; r += blockDim.x) {
                        const double x = wp[r], y = wq[r];
                        wp[r] = c * x - s * y;
                        wq[r] = s * x + c * y;
                    }
                }
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
    if (v.colsp >= 2) {
        SvdDevView vv = v;
        void *args[] = {&vv};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&jacobi_kernel), dim3(coop_grid),
                                       dim3(256), args, 0, stream);
        if (e != hipSuccess) return e;
    }
    const int gc = v.cols < 1 ? 1 : (v.cols > 2048 ? 2048 : v.cols);
    norms_kernel<<<gc, 256, 0, stream>>>(v);
    scatter_kernel<<<gc, 256, 0, stream>>>(v);
    return hipGetLastError();
}

int svd_coop_grid(int colsp, int n_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&jacobi_kernel), 256, 0) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    int maxres = per_cu * n_cu;
    int npairs = colsp / 2;
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
