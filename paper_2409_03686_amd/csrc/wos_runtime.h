// wos_runtime.h -- host-side internals of libwos (context, staging ring, group launches).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/wos.h"
#include "wos_internal.h"

struct RingSlot {
    void *host = nullptr;  // pinned staging of the descriptors
    void *dev = nullptr;   // device copy + work cursor
    size_t cap = 0;
    hipEvent_t done{};     // recorded after the launch that last used the slot
    bool used = false;
};

struct LiveServer;

struct wos_ctx {
    int device = 0;
    size_t hbm_budget = 0;
    std::atomic<size_t> hbm_used{0};
    hipDeviceProp_t props{};
    int n_cu = 1;
    bool poisoned = false;
    std::array<RingSlot, 16> ring;
    size_t ring_next = 0;
    std::mutex mu;                  // tuning table
    std::recursive_mutex launch_mu; // staging ring and launches
    std::map<int, wos_tuning> tuning;
    LiveServer *live = nullptr;     // live serving thread (wos_serve_start), or none
    uint8_t *noalloc_scratch = nullptr;  // this device's copy of the allocation-free scratch array
};

namespace wos {

struct GroupLaunch {
    int n_inst = 0;
    uint64_t items = 0;
    int block = 256, grid = 1;
    int per_cu = 1;  // resident blocks per CU (grid = per_cu x CUs of the launch stream, at most items)
    int hist_words = 4, seg_bytes = 0;
    int precision = 0, dim = 2;
    int kind_sel = -1;  // shared domain kind (+ kRadiusVariant for the mapped bound), -1 if mixed
    int mode = 0;       // 0 block items, 1 wave items, 2 points (walk_lds_bytes)
};

wos_status set_error(wos_status st, const char *fmt, ...);
int stream_cus(const wos_ctx *ctx, hipStream_t s);  // CUs the stream may use (its CU mask), else all
void live_server_stop(wos_ctx *ctx);  // stops and frees the context's live server, if any
wos_status ctx_malloc(wos_ctx *ctx, void **p, size_t bytes);
void ctx_free(wos_ctx *ctx, void *p, size_t bytes);
wos_status validate_geometry(const wos_geometry *g, int *n_elem);
size_t vertex_doubles(const wos_geometry *g);  // numbers in g->verts for its kind
wos_status validate_walk(const wos_geometry *g, const wos_walk_params *w);
// S = (K / lambda_max)^{1/2} (symmetric root); optionally its eigenvectors (row-major, column k the
// k-th) and eigenvalues
wos_status conductivity_root(const double *K, int d, double S[9], double *lam_max, double *lam_min,
                             double *evec = nullptr, double *eval = nullptr);
wos_status fill_inst(const wos_geometry *g, const wos_walk_params *w, int n_elem, DevInst &I,
                     std::vector<PolySeg> &segs);
wos_tuning get_tuning(wos_ctx *ctx, int dim, int kind, int precision);
wos_status group_jobs(const wos_measure_job *jobs, int n, std::vector<std::vector<int>> &groups);
wos_status prepare_group(wos_ctx *ctx, const wos_measure_job *jobs, const std::vector<int> &idx,
                         const wos_tuning *force, std::vector<uint8_t> &buf, GroupLaunch &gl);
wos_status stage_and_launch(wos_ctx *ctx, std::vector<uint8_t> &buf, const GroupLaunch &gl, hipStream_t stream);
struct SvdHost {
    SvdDevView v{};
    size_t bytes = 0;
    std::vector<double> nu, isig;
    std::vector<int32_t> g1, g0, emap;
};
// trunc_k > 0: layout for the truncated path (tsvd_launch) keeping at most trunc_k triplets
wos_status svd_layout(int32_t n_obs, int32_t n_elem, const uint8_t *gamma1_mask_host, const double *sigma_host,
                      const double *nu_host, SvdHost &hs, int trunc_k = 0);
void svd_bind(SvdHost &hs, void *mem);
size_t svd_staging_bytes(const SvdHost &hs);
hipError_t svd_upload(const SvdHost &hs, void *staging, hipStream_t stream);
wos_status check_reg(const wos_reg_params *reg);
wos_status build_batch(wos_ctx *ctx, const wos_measure_job *jobs, int32_t n_jobs, hipStream_t stream,
                       const wos_tuning *force);

}  // namespace wos
