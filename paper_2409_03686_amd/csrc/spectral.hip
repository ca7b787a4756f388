// spectral.hip -- host side of the spectral end (wos_svd*, wos_reconstruct) and HIP-graph plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/wos.h"
#include "wos_internal.h"
#include "wos_runtime.h"

using namespace wos;

struct wos_svd_t {
    wos_ctx *ctx = nullptr;
    SvdDevView v{};
    void *mem = nullptr;
    size_t bytes = 0;
    int coop_grid = 1;
    bool nu_nonzero = true;  // every nu_i != 0: the sweep's predicted data divide by nu
    SvdEvents ev{};          // recorded by wos_svd (eager calls) for wos_svd_timing
    bool timed = false;      // a wos_svd has recorded them
};

namespace {

__global__ void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

template <typename T> T *carve(uint8_t *&cur, size_t count)
{
    T *p = reinterpret_cast<T *>(cur);
    cur += (count * sizeof(T) + 255) & ~size_t(255);
    return p;
}

size_t carve_size(size_t count, size_t elt) { return (count * elt + 255) & ~size_t(255); }

}  // namespace

hipError_t wos::fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    size_t g = (n + 255) / 256;
    g = std::min<size_t>(g, 8192);
    fill_u32_kernel<<<static_cast<int>(g), 256, 0, stream>>>(p, n, v);
    return hipGetLastError();
}

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            if (ctx) (ctx)->poisoned = true;                                                      \
            return set_error(WOS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
        }                                                                                         \
    } while (0)

wos_status wos::svd_layout(int32_t n_obs, int32_t n_elem, const uint8_t *gamma1_mask_host, const double *sigma_host,
                           const double *nu_host, SvdHost &hs, int trunc_k)
{
    if (n_obs < 1 || n_elem < 1) return set_error(WOS_EINVAL, "n_obs and n_elem must be >= 1");
    if (!gamma1_mask_host || !sigma_host) return set_error(WOS_EINVAL, "gamma1 mask and sigma are required");
    hs = SvdHost{};
    hs.emap.resize(n_elem);
    for (int j = 0; j < n_elem; ++j) {
        if (gamma1_mask_host[j] > 1) return set_error(WOS_EINVAL, "gamma1 mask entries must be 0 or 1");
        if (!(sigma_host[j] > 0) || !std::isfinite(sigma_host[j])) return set_error(WOS_EINVAL, "sigma must be > 0");
        if (gamma1_mask_host[j]) {
            hs.emap[j] = static_cast<int32_t>(hs.g1.size());
            hs.g1.push_back(j);
        } else {
            hs.emap[j] = -static_cast<int32_t>(hs.g0.size()) - 1;
            hs.g0.push_back(j);
        }
    }
    if (hs.g1.empty()) return set_error(WOS_EINVAL, "Gamma_1 is empty");
    hs.nu.assign(n_obs, 1.0 / std::sqrt(static_cast<double>(n_obs)));
    if (nu_host)
        for (int i = 0; i < n_obs; ++i) {
            if (!std::isfinite(nu_host[i])) return set_error(WOS_EINVAL, "nu must be finite");
            hs.nu[i] = nu_host[i];
        }
    hs.isig.resize(hs.g1.size());
    for (size_t l = 0; l < hs.g1.size(); ++l) hs.isig[l] = 1.0 / std::sqrt(sigma_host[hs.g1[l]]);
    SvdDevView &v = hs.v;
    v = SvdDevView{};
    v.m = n_obs;
    v.n = static_cast<int>(hs.g1.size());
    v.k = std::min(v.m, v.n);
    v.trans = v.m < v.n ? 1 : 0;
    v.rows = v.trans ? v.n : v.m;
    v.cols = v.trans ? v.m : v.n;
    v.colsp = (v.cols + 15) & ~15;  // blocks of 8 columns, an even number of blocks
    v.n_elem = n_elem;
    v.n0 = static_cast<int>(hs.g0.size());
    v.tol = static_cast<double>(v.rows) * 0x1.0p-52;
    v.np = gram_order(v.cols);
    if (trunc_k > 0) {
        // truncated path: kt = 64 or 128 columns, Gram order kt; k = at most kt triplets
        v.tk = v.cols <= 64 ? 64 : kTruncRank;
        v.np = v.tk;
        v.k = std::min(v.k, v.tk);
        v.rank_cut = 1e-5;
    }
    const size_t npn = static_cast<size_t>(v.np);
    const size_t tkn = static_cast<size_t>(v.tk);
    const size_t big = v.tk && v.cols > v.tk ? tkn : 0;  // sketch buffers only when projecting
    const bool grid = !v.tk && v.np > kGramMaxCols;      // device-wide Gram path
    hs.bytes = 0;
    // device arrays, in carve order
    const size_t sz[] = {
        carve_size(size_t(v.rows) * v.colsp, 8), carve_size(v.tk ? 0 : size_t(v.colsp) * v.colsp, 8), carve_size(v.k, 8),
        carve_size(size_t(v.m) * v.k, 8), carve_size(size_t(v.n) * v.k, 8), carve_size(v.m, 8),
        carve_size(v.n, 8), carve_size(hs.g1.size(), 4), carve_size(std::max<size_t>(hs.g0.size(), 1), 4),
        carve_size(n_elem, 4), carve_size(v.cols + 2, 8), carve_size(v.m, 8), carve_size(v.k, 8),
        carve_size(v.k, 8), carve_size(2 * kMaxSweeps, 4), carve_size(kCtrlWords, 4), carve_size(kInfoWords, 4),
        carve_size(npn * npn, 8), carve_size(npn * npn, 8), carve_size(npn, 8), carve_size(grid ? npn : 0, 8),
        carve_size(grid ? kGridCtlWords : 0, 4), carve_size(grid ? 3 * npn + 1024 : 0, 4), carve_size(2, 8),
        carve_size(size_t(v.cols) * big, 8), carve_size(size_t(v.rows) * tkn, 8), carve_size(size_t(v.rows) * big, 8),
        carve_size(big * v.cols, 8), carve_size(big * big, 8), carve_size(big * big, 8), carve_size(tkn, 8),
        carve_size(std::max<size_t>(tkn, 1), 4)};
    for (size_t s : sz) hs.bytes += s;
    return WOS_OK;
}

void wos::svd_bind(SvdHost &hs, void *mem)
{
    SvdDevView &v = hs.v;
    uint8_t *cur = static_cast<uint8_t *>(mem);
    v.A = carve<double>(cur, size_t(v.rows) * v.colsp);
    v.W = carve<double>(cur, v.tk ? 0 : size_t(v.colsp) * v.colsp);  // Hestenes path only
    v.s = carve<double>(cur, v.k);
    v.U = carve<double>(cur, size_t(v.m) * v.k);
    v.V = carve<double>(cur, size_t(v.n) * v.k);
    v.nu = carve<double>(cur, v.m);
    v.isig1 = carve<double>(cur, v.n);
    v.g1idx = carve<int32_t>(cur, hs.g1.size());
    v.g0idx = carve<int32_t>(cur, std::max<size_t>(hs.g0.size(), 1));
    v.emap = carve<int32_t>(cur, v.n_elem);
    v.work = carve<double>(cur, v.cols + 2);
    v.q = carve<double>(cur, v.m);
    v.cvec = carve<double>(cur, v.k);
    v.phic = carve<double>(cur, v.k);
    v.rot = carve<uint32_t>(cur, 2 * kMaxSweeps);
    v.ctrl = carve<uint32_t>(cur, kCtrlWords);
    v.info = carve<int32_t>(cur, kInfoWords);
    const size_t npn = static_cast<size_t>(v.np);
    v.G = carve<double>(cur, npn * npn);
    v.L = carve<double>(cur, npn * npn);
    v.zs = carve<double>(cur, npn);
    const bool grid = !v.tk && v.np > kGramMaxCols;
    v.gnrm = grid ? carve<double>(cur, npn) : nullptr;
    v.gctl = grid ? carve<uint32_t>(cur, kGridCtlWords) : nullptr;
    v.gpiv = grid ? carve<int32_t>(cur, 3 * npn + 1024) : nullptr;  // row states, then the candidates
    v.crit = carve<unsigned long long>(cur, 2);
    const size_t tkn = static_cast<size_t>(v.tk);
    const size_t big = v.tk && v.cols > v.tk ? tkn : 0;
    v.Om = carve<double>(cur, size_t(v.cols) * big);
    v.Y = carve<double>(cur, size_t(v.rows) * tkn);  // also A V for the triplet residuals
    v.Q = carve<double>(cur, size_t(v.rows) * big);
    v.Cm = carve<double>(cur, big * v.cols);
    v.Gt = carve<double>(cur, big * big);
    v.Lt = carve<double>(cur, big * big);
    v.zt = carve<double>(cur, tkn);  // also the triplet residuals
    v.perm = carve<int32_t>(cur, std::max<size_t>(tkn, 1));
}

// Bytes of pinned staging svd_upload needs.
size_t wos::svd_staging_bytes(const SvdHost &hs)
{
    return 8 * (hs.nu.size() + hs.isig.size()) + 4 * (hs.g1.size() + hs.g0.size() + hs.emap.size()) + 64;
}

hipError_t wos::svd_upload(const SvdHost &hs, void *staging, hipStream_t stream)
{
    uint8_t *st = static_cast<uint8_t *>(staging);
    auto put = [&](void *dst, const void *src, size_t bytes) {
        if (bytes == 0) return hipSuccess;
        std::memcpy(st, src, bytes);
        hipError_t e = hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, stream);
        st += (bytes + 7) & ~size_t(7);
        return e;
    };
    hipError_t e = put(hs.v.nu, hs.nu.data(), 8 * hs.nu.size());
    if (e == hipSuccess) e = put(hs.v.isig1, hs.isig.data(), 8 * hs.isig.size());
    if (e == hipSuccess) e = put(hs.v.g1idx, hs.g1.data(), 4 * hs.g1.size());
    if (e == hipSuccess) e = put(hs.v.g0idx, hs.g0.data(), 4 * hs.g0.size());
    if (e == hipSuccess) e = put(hs.v.emap, hs.emap.data(), 4 * hs.emap.size());
    return e;
}

extern "C" wos_status wos_svd_create(wos_ctx *ctx, int32_t n_obs, int32_t n_elem, const uint8_t *gamma1_mask_host,
                                     const double *sigma_host, const double *nu_host, wos_svd_t **out)
{
    if (!ctx || !out) return set_error(WOS_EINVAL, "ctx or out NULL");
    *out = nullptr;
    SvdHost hs;
    wos_status st = svd_layout(n_obs, n_elem, gamma1_mask_host, sigma_host, nu_host, hs);
    if (st != WOS_OK) return st;
    wos_svd_t *h = new wos_svd_t();
    h->ctx = ctx;
    h->bytes = hs.bytes;
    st = ctx_malloc(ctx, &h->mem, h->bytes);
    if (st != WOS_OK) {
        delete h;
        return st;
    }
    svd_bind(hs, h->mem);
    std::vector<uint8_t> staging(svd_staging_bytes(hs));
    hipError_t e = hipSuccess;
    const SvdDevView &v = hs.v;
    e = hipMemcpy(v.nu, hs.nu.data(), 8 * hs.nu.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(v.isig1, hs.isig.data(), 8 * hs.isig.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(v.g1idx, hs.g1.data(), 4 * hs.g1.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !hs.g0.empty()) e = hipMemcpy(v.g0idx, hs.g0.data(), 4 * hs.g0.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(v.emap, hs.emap.data(), 4 * hs.emap.size(), hipMemcpyHostToDevice);
    int32_t zero_info[kInfoWords] = {};
    if (e == hipSuccess) e = hipMemcpy(v.info, zero_info, sizeof zero_info, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx_free(ctx, h->mem, h->bytes);
        delete h;
        return set_error(WOS_EDEVICE, "SVD workspace upload failed: %s", hipGetErrorString(e));
    }
    h->v = hs.v;
    h->coop_grid = svd_coop_grid(h->v.rows, h->v.colsp, ctx->n_cu);
    for (hipEvent_t *pe : {&h->ev.jac0, &h->ev.jac1, &h->ev.all0, &h->ev.all1}) {
        if (hipEventCreate(pe) != hipSuccess) {
            *pe = nullptr;
            (void)wos_svd_destroy(ctx, h);
            return set_error(WOS_EDEVICE, "hipEventCreate failed");
        }
    }
    for (double x : hs.nu) h->nu_nonzero = h->nu_nonzero && x != 0.0;
    *out = h;
    return WOS_OK;
}

extern "C" wos_status wos_svd_destroy(wos_ctx *ctx, wos_svd_t *h)
{
    if (!ctx || !h) return set_error(WOS_EINVAL, "ctx or handle NULL");
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : {h->ev.jac0, h->ev.jac1, h->ev.all0, h->ev.all1})
        if (e) (void)hipEventDestroy(e);
    ctx_free(ctx, h->mem, h->bytes);
    delete h;
    return WOS_OK;
}

extern "C" wos_status wos_svd(wos_ctx *ctx, wos_svd_t *h, const uint32_t *counts_dev, uint64_t n_walks, void *stream)
{
    if (!ctx || !h || !counts_dev) return set_error(WOS_EINVAL, "ctx, handle or counts NULL");
    if (n_walks == 0) return set_error(WOS_EINVAL, "n_walks must be >= 1");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // cooperative grids sized for the CUs the stream may use (all, or its CU mask)
    const int coop_grid = svd_coop_grid(h->v.rows, h->v.colsp, stream_cus(ctx, static_cast<hipStream_t>(stream)));
    // timing events only outside stream capture (a captured graph gets no event nodes from here)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(ctx, hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cap));
    const bool timed = cap == hipStreamCaptureStatusNone && h->ev.all1;
    HIP_TRY(ctx, svd_launch(h->v, counts_dev, 1.0 / static_cast<double>(n_walks), coop_grid,
                            stream_cus(ctx, static_cast<hipStream_t>(stream)), static_cast<hipStream_t>(stream),
                            timed ? &h->ev : nullptr));
    h->timed = timed;
    return WOS_OK;
}

extern "C" wos_status wos_svd_factors(const wos_svd_t *h, const double **U, const double **s, const double **V,
                                      int32_t *m, int32_t *n, int32_t *k)
{
    if (!h) return set_error(WOS_EINVAL, "handle NULL");
    if (U) *U = h->v.U;
    if (s) *s = h->v.s;
    if (V) *V = h->v.V;
    if (m) *m = h->v.m;
    if (n) *n = h->v.n;
    if (k) *k = h->v.k;
    return WOS_OK;
}

extern "C" wos_status wos_svd_info(const wos_svd_t *h, int32_t *sweeps, int32_t *error_flag, int32_t *method,
                                   void *stream)
{
    if (!h) return set_error(WOS_EINVAL, "handle NULL");
    int32_t info[kInfoWords] = {};
    hipError_t e = hipMemcpyAsync(info, h->v.info, sizeof info, hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(WOS_EDEVICE, "reading SVD info failed: %s", hipGetErrorString(e));
    if (sweeps) *sweeps = info[0];
    if (error_flag) *error_flag = info[1];
    if (method) *method = info[4] ? WOS_SVD_GRAM : WOS_SVD_HESTENES;
    return WOS_OK;
}

extern "C" wos_status wos_svd_gram_check(const wos_svd_t *h, int32_t *gram_sweeps, int32_t *gram_error_flag,
                                         double *check, double *residual, void *stream)
{
    if (!h) return set_error(WOS_EINVAL, "handle NULL");
    int32_t info[kInfoWords] = {};
    unsigned long long crit[2] = {0ull, 0ull};
    hipError_t e = hipMemcpyAsync(info, h->v.info, sizeof info, hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream));
    if (e == hipSuccess)
        e = hipMemcpyAsync(crit, h->v.crit, sizeof crit, hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(WOS_EDEVICE, "reading SVD diagnostics failed: %s", hipGetErrorString(e));
    if (gram_sweeps) *gram_sweeps = info[2];
    if (gram_error_flag) *gram_error_flag = info[3];
    double c[2];
    std::memcpy(c, crit, sizeof c);
    if (check) *check = c[0];
    if (residual) *residual = c[1];
    return WOS_OK;
}

extern "C" wos_status wos_svd_timing(const wos_svd_t *h, float *jacobi_ms, float *total_ms, uint64_t *rotations)
{
    if (!h) return set_error(WOS_EINVAL, "handle NULL");
    if (!h->timed) return set_error(WOS_EINVAL, "no timed wos_svd on this handle yet");
    if (hipEventSynchronize(h->ev.all1) != hipSuccess) return set_error(WOS_EDEVICE, "event synchronisation failed");
    float jm = 0.0f, tm = 0.0f;
    const bool jac = h->ev.jac_recorded && hipEventElapsedTime(&jm, h->ev.jac0, h->ev.jac1) == hipSuccess;
    if (hipEventElapsedTime(&tm, h->ev.all0, h->ev.all1) != hipSuccess)
        return set_error(WOS_EDEVICE, "reading SVD events failed");
    uint64_t nrot = 0;
    if (h->v.gctl) {
        uint32_t r[kMaxSweeps];
        if (hipMemcpy(r, h->v.gctl + kGridFlags, sizeof r, hipMemcpyDeviceToHost) != hipSuccess)
            return set_error(WOS_EDEVICE, "reading rotation counts failed");
        for (uint32_t x : r) nrot += x;
    }
    if (jacobi_ms) *jacobi_ms = jac ? jm : 0.0f;
    if (total_ms) *total_ms = tm;
    if (rotations) *rotations = nrot;
    return WOS_OK;
}

wos_status wos::check_reg(const wos_reg_params *reg)
{
    if (!reg) return set_error(WOS_EINVAL, "regularisation params NULL");
    if (reg->kind < 0 || reg->kind > 2) return set_error(WOS_EINVAL, "unknown regularisation kind %d", reg->kind);
    if (reg->kind == WOS_TSVD_RANK && reg->rank < 0) return set_error(WOS_EINVAL, "rank must be >= 0");
    if (reg->kind != WOS_TSVD_RANK && !(reg->alpha > 0) &&
        (!(reg->noise_delta >= 0) || !(reg->tau > 0) || !std::isfinite(reg->noise_delta)))
        return set_error(WOS_EINVAL, "discrepancy rule needs noise_delta >= 0 and tau > 0");
    if (reg->kind == WOS_TIKHONOV && !(reg->alpha >= 0)) return set_error(WOS_EINVAL, "alpha must be >= 0");
    return WOS_OK;
}

extern "C" wos_status wos_reconstruct(wos_ctx *ctx, const wos_svd_t *h, const uint32_t *counts_dev, uint64_t n_walks,
                                      const double *uD_dev, const double *u0_dev, const wos_reg_params *reg,
                                      double *u1_dev, double *pred_dev, int32_t *rank_used_dev,
                                      double *alpha_used_dev, void *stream)
{
    if (!ctx || !h || !counts_dev || !uD_dev || !u1_dev) return set_error(WOS_EINVAL, "NULL argument");
    if (n_walks == 0) return set_error(WOS_EINVAL, "n_walks must be >= 1");
    if (h->v.n0 > 0 && !u0_dev) return set_error(WOS_EINVAL, "u0_dev is required when Gamma_0 is not empty");
    wos_status st = check_reg(reg);
    if (st != WOS_OK) return st;
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    RegDev r{reg->kind, reg->rank, reg->alpha, reg->noise_delta, reg->tau};
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, recon_launch(h->v, counts_dev, 1.0 / static_cast<double>(n_walks), uD_dev, h->v.n0 ? u0_dev : nullptr,
                              r, u1_dev, pred_dev, rank_used_dev, alpha_used_dev, static_cast<hipStream_t>(stream)));
    return WOS_OK;
}

extern "C" wos_status wos_reconstruct_sweep(wos_ctx *ctx, const wos_svd_t *h, const uint32_t *counts_dev,
                                            uint64_t n_walks, const double *uD_dev, const double *u0_dev,
                                            int32_t r_max, double *u1_dev, double *pred_dev, double *resid_dev,
                                            void *stream)
{
    if (!ctx || !h || !counts_dev || !uD_dev || !u1_dev) return set_error(WOS_EINVAL, "NULL argument");
    if (n_walks == 0) return set_error(WOS_EINVAL, "n_walks must be >= 1");
    if (h->v.n0 > 0 && !u0_dev) return set_error(WOS_EINVAL, "u0_dev is required when Gamma_0 is not empty");
    if (r_max < 1 || r_max > h->v.k)
        return set_error(WOS_EINVAL, "r_max = %d outside [1, %d] (the singular triplets held)", r_max, h->v.k);
    if (pred_dev && !h->nu_nonzero) return set_error(WOS_EINVAL, "predicted data need every nu_i != 0");
    if (sweep_part_words(h->v, r_max) > static_cast<size_t>(h->v.rows) * h->v.colsp)
        return set_error(WOS_EINVAL, "residual partials exceed the work matrix");  // cannot happen for r_max <= k
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, sweep_launch(h->v, counts_dev, 1.0 / static_cast<double>(n_walks), uD_dev,
                              h->v.n0 ? u0_dev : nullptr, r_max, u1_dev, pred_dev, resid_dev,
                              static_cast<hipStream_t>(stream)));
    return WOS_OK;
}

extern "C" wos_status wos_eigenfunctions(wos_ctx *ctx, const wos_svd_t *h, int32_t n_fun, double *lambda_dev,
                                         double *ef_dev, void *stream)
{
    if (!ctx || !h) return set_error(WOS_EINVAL, "ctx or handle NULL");
    if (n_fun < 0 || n_fun > h->v.k)
        return set_error(WOS_EINVAL, "n_fun = %d outside [0, %d] (the singular triplets held)", n_fun, h->v.k);
    if (n_fun > 0 && !lambda_dev && !ef_dev) return set_error(WOS_EINVAL, "no output given");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, eigfun_launch(h->v, n_fun, lambda_dev, ef_dev, static_cast<hipStream_t>(stream)));
    return WOS_OK;
}

extern "C" wos_status wos_density(wos_ctx *ctx, const uint32_t *counts_dev, int32_t n_obs, int32_t n_elem,
                                  uint64_t n_walks, const double *sigma_dev, double *rho_dev, double *mean_dev,
                                  void *stream)
{
    if (!ctx || !counts_dev || !sigma_dev) return set_error(WOS_EINVAL, "NULL argument");
    if (!rho_dev && !mean_dev) return set_error(WOS_EINVAL, "no output given");
    if (n_obs < 1 || n_elem < 1) return set_error(WOS_EINVAL, "n_obs and n_elem must be >= 1");
    if (n_walks == 0) return set_error(WOS_EINVAL, "n_walks must be >= 1");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, density_launch(counts_dev, n_obs, n_elem, n_walks, sigma_dev, rho_dev, mean_dev,
                                static_cast<hipStream_t>(stream)));
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Plans: the whole path of one instance captured as a HIP graph (kernels only: the descriptors
// are uploaded once when the plan is made).
// ---------------------------------------------------------------------------------------------
struct wos_plan {
    wos_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *desc = nullptr;
    size_t desc_bytes = 0;
};

extern "C" wos_status wos_plan_create(wos_ctx *ctx, const wos_measure_job *job, wos_svd_t *svd, const double *uD_dev,
                                      const double *u0_dev, const wos_reg_params *reg, double *u1_dev,
                                      double *pred_dev, int32_t *rank_used_dev, double *alpha_used_dev,
                                      wos_plan **out)
{
    if (!ctx || !job || !out) return set_error(WOS_EINVAL, "NULL argument");
    *out = nullptr;
    std::vector<std::vector<int>> groups;
    wos_status st = group_jobs(job, 1, groups);
    if (st != WOS_OK) return st;
    if (groups.empty()) return set_error(WOS_EINVAL, "plan has no walks to run");
    if (svd) {
        if (!uD_dev || !u1_dev) return set_error(WOS_EINVAL, "reconstruction outputs missing");
        st = check_reg(reg);
        if (st != WOS_OK) return st;
        if (svd->v.m != job->n_obs) return set_error(WOS_EINVAL, "SVD handle is for %d points, job has %d", svd->v.m, job->n_obs);
        if (svd->v.n0 > 0 && !u0_dev) return set_error(WOS_EINVAL, "u0_dev is required when Gamma_0 is not empty");
    }
    std::vector<uint8_t> buf;
    GroupLaunch gl;
    st = prepare_group(ctx, job, groups[0], nullptr, buf, gl);
    if (st != WOS_OK) return st;
    std::lock_guard<std::recursive_mutex> lk(ctx->launch_mu);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    wos_plan *p = new wos_plan();
    p->ctx = ctx;
    p->desc_bytes = ((buf.size() + 15) & ~size_t(15)) + 4 * walk_cursor_words(gl.mode, gl.items) + 64;
    st = ctx_malloc(ctx, &p->desc, p->desc_bytes);
    if (st != WOS_OK) {
        delete p;
        return st;
    }
    uint8_t *dev = static_cast<uint8_t *>(p->desc);
    DevInst *I = reinterpret_cast<DevInst *>(buf.data());
    for (int q = 0; q < gl.n_inst; ++q)
        I[q].segs = reinterpret_cast<const PolySeg *>(reinterpret_cast<uintptr_t>(dev) + reinterpret_cast<uintptr_t>(I[q].segs));
    auto cleanup = [&](const char *what, hipError_t e) {
        ctx_free(ctx, p->desc, p->desc_bytes);
        delete p;
        return set_error(WOS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipMemcpy(dev, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup("descriptor upload", e);
    uint32_t *cursor = reinterpret_cast<uint32_t *>(dev + ((buf.size() + 15) & ~size_t(15)));
    int M = 0;
    (void)validate_geometry(&job->geom, &M);
    const uint64_t n_walks = job->walk.walk_end - job->walk.walk_begin;
    hipStream_t cs;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup("stream", e);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = fill_u32(job->counts_dev, static_cast<size_t>(job->n_obs) * M, 0u, cs);
    if (e == hipSuccess && job->stats_dev) e = fill_u32(reinterpret_cast<uint32_t *>(job->stats_dev), 2 * WOS_STATS_WORDS, 0u, cs);
    if (e == hipSuccess)
        e = launch_walks(gl.precision, gl.dim, gl.kind_sel, gl.mode, reinterpret_cast<const DevInst *>(dev), gl.n_inst,
                         gl.items, cursor, gl.hist_words, gl.seg_bytes, gl.block, gl.grid, cs);
    if (e == hipSuccess && svd) {
        e = svd_launch(svd->v, job->counts_dev, 1.0 / static_cast<double>(n_walks), svd->coop_grid, ctx->n_cu, cs);
        if (e == hipSuccess) {
            RegDev r{reg->kind, reg->rank, reg->alpha, reg->noise_delta, reg->tau};
            e = recon_launch(svd->v, job->counts_dev, 1.0 / static_cast<double>(n_walks), uD_dev,
                             svd->v.n0 ? u0_dev : nullptr, r, u1_dev, pred_dev, rank_used_dev, alpha_used_dev, cs);
        }
    }
    hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (p->graph) (void)hipGraphDestroy(p->graph);
        return cleanup("graph capture", e);
    }
    *out = p;
    return WOS_OK;
}

extern "C" wos_status wos_plan_create_batch(wos_ctx *ctx, const wos_measure_job *jobs, int32_t n_jobs, wos_plan **out)
{
    if (!ctx || !out || n_jobs < 1 || !jobs) return set_error(WOS_EINVAL, "NULL argument or empty batch");
    *out = nullptr;
    std::vector<std::vector<int>> groups;
    wos_status st = group_jobs(jobs, n_jobs, groups);
    if (st != WOS_OK) return st;
    if (groups.empty()) return set_error(WOS_EINVAL, "plan has no walks to run");
    // every group's descriptor (instances, records, then its work cursors) in one allocation
    std::vector<std::vector<uint8_t>> bufs(groups.size());
    std::vector<GroupLaunch> gls(groups.size());
    std::vector<size_t> offs(groups.size());
    size_t total = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        st = prepare_group(ctx, jobs, groups[g], nullptr, bufs[g], gls[g]);
        if (st != WOS_OK) return st;
        offs[g] = total;
        total += (((bufs[g].size() + 15) & ~size_t(15)) + 4 * walk_cursor_words(gls[g].mode, gls[g].items) + 64 + 255) &
                 ~size_t(255);
    }
    std::lock_guard<std::recursive_mutex> lk(ctx->launch_mu);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    wos_plan *p = new wos_plan();
    p->ctx = ctx;
    p->desc_bytes = total;
    st = ctx_malloc(ctx, &p->desc, p->desc_bytes);
    if (st != WOS_OK) {
        delete p;
        return st;
    }
    auto cleanup = [&](const char *what, hipError_t e) {
        ctx_free(ctx, p->desc, p->desc_bytes);
        delete p;
        return set_error(WOS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };
    std::vector<uint32_t *> cursors(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        uint8_t *dev = static_cast<uint8_t *>(p->desc) + offs[g];
        DevInst *I = reinterpret_cast<DevInst *>(bufs[g].data());
        for (int q = 0; q < gls[g].n_inst; ++q)
            I[q].segs = reinterpret_cast<const PolySeg *>(reinterpret_cast<uintptr_t>(dev) + reinterpret_cast<uintptr_t>(I[q].segs));
        hipError_t e = hipMemcpy(dev, bufs[g].data(), bufs[g].size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup("descriptor upload", e);
        cursors[g] = reinterpret_cast<uint32_t *>(dev + ((bufs[g].size() + 15) & ~size_t(15)));
    }
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup("stream", e);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (size_t g = 0; g < groups.size() && e == hipSuccess; ++g)
        for (int q : groups[g]) {
            const wos_measure_job &J = jobs[q];
            int M = 0;
            (void)validate_geometry(&J.geom, &M);
            if (e == hipSuccess) e = fill_u32(J.counts_dev, static_cast<size_t>(J.n_obs) * M, 0u, cs);
            if (e == hipSuccess && J.stats_dev)
                e = fill_u32(reinterpret_cast<uint32_t *>(J.stats_dev), 2 * WOS_STATS_WORDS, 0u, cs);
        }
    for (size_t g = 0; g < groups.size() && e == hipSuccess; ++g) {
        const GroupLaunch &gl = gls[g];
        e = launch_walks(gl.precision, gl.dim, gl.kind_sel, gl.mode,
                         reinterpret_cast<const DevInst *>(static_cast<uint8_t *>(p->desc) + offs[g]), gl.n_inst, gl.items,
                         cursors[g], gl.hist_words, gl.seg_bytes, gl.block, gl.grid, cs);
    }
    hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (p->graph) (void)hipGraphDestroy(p->graph);
        return cleanup("graph capture", e);
    }
    *out = p;
    return WOS_OK;
}

extern "C" wos_status wos_plan_launch(wos_plan *p, void *stream)
{
    if (!p) return set_error(WOS_EINVAL, "plan NULL");
    hipError_t e = hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(WOS_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(e));
    return WOS_OK;
}

extern "C" wos_status wos_plan_destroy(wos_plan *p)
{
    if (!p) return set_error(WOS_EINVAL, "plan NULL");
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    ctx_free(p->ctx, p->desc, p->desc_bytes);
    delete p;
    return WOS_OK;
}
