// serve.hip -- continuous batching of build + SVD + reconstruct requests (wos_serve).
//
// One host thread replays the arrival times (open loop).  A request is admitted when one of
// max_inflight slots is free and its device footprint fits in the HBM budget; its buffers are
// sub-allocated (first fit) from one arena allocated once, its inputs are staged through the
// slot's pinned buffer, and its whole path is enqueued on the slot's stream.  Admitted requests
// run concurrently: their persistent walk kernels share the compute units, and the SVD /
// reconstruction of one request overlaps the walks of others.  Completion is detected by polling
// an event per request; results are copied out of pinned memory and the slot and memory are
// released for the next queued request.  Every result is a pure function of its request (the
// random numbers are keyed by seed, instance, point and walk), so it is the same alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "../../include/wos.h"
#include "wos_internal.h"
#include "wos_runtime.h"

using namespace wos;

namespace {

struct Arena {  // first-fit sub-allocator over one device allocation
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t n)
    {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t &off)
    {
        n = (n + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) & ~size_t(255);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct ReqLayout {
    int M = 0, n1 = 0, n0 = 0, k = 0, dim = 2;
    size_t off_x, off_counts, off_stats, off_uD, off_u0, off_u1, off_pred, off_scal, off_svd, total;
    SvdHost svd;
};

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

wos_status layout_request(const wos_request &r, ReqLayout &L)
{
    int M = 0;
    wos_status st = validate_geometry(&r.geom, &M);
    if (st != WOS_OK) return st;
    st = validate_walk(&r.geom, &r.walk);
    if (st != WOS_OK) return st;
    if (r.n_obs < 1 || !r.x_obs_host || !r.uD_host) return set_error(WOS_EINVAL, "request needs points and data");
    if (r.walk.walk_end <= r.walk.walk_begin) return set_error(WOS_EINVAL, "request needs at least one walk");
    std::vector<double> sigma(M);
    st = wos_element_measures(&r.geom, sigma.data());
    if (st != WOS_OK) return st;
    st = svd_layout(r.n_obs, M, r.gamma1_mask_host, sigma.data(), nullptr, L.svd);
    if (st != WOS_OK) return st;
    st = check_reg(&r.reg);
    if (st != WOS_OK) return st;
    L.M = M;
    L.dim = r.geom.dim;
    L.n1 = L.svd.v.n;
    L.n0 = L.svd.v.n0;
    L.k = L.svd.v.k;
    if (L.n0 > 0 && !r.u0_host) return set_error(WOS_EINVAL, "request needs u0 (Gamma_0 is not empty)");
    size_t o = 0;
    L.off_x = o; o += up256(8ull * r.n_obs * L.dim);
    L.off_counts = o; o += up256(4ull * r.n_obs * M);
    L.off_stats = o; o += up256(8ull * WOS_STATS_WORDS);
    L.off_uD = o; o += up256(8ull * r.n_obs);
    L.off_u0 = o; o += up256(8ull * std::max(L.n0, 1));
    L.off_u1 = o; o += up256(8ull * L.n1);
    L.off_pred = o; o += up256(8ull * r.n_obs);
    L.off_scal = o; o += up256(16);
    L.off_svd = o; o += up256(L.svd.bytes);
    L.total = o;
    return WOS_OK;
}

// pinned staging: inputs then outputs
size_t staging_bytes(const wos_request &r, const ReqLayout &L)
{
    return up256(8ull * r.n_obs * L.dim) + up256(8ull * r.n_obs) + up256(8ull * std::max(L.n0, 1)) +
           up256(svd_staging_bytes(L.svd)) +
           // outputs: u1, pred, s, scalars, stats
           up256(8ull * L.n1) + up256(8ull * r.n_obs) + up256(8ull * L.k) + up256(16) + up256(8ull * WOS_STATS_WORDS);
}

struct Slot {
    hipStream_t stream{};
    hipEvent_t done{};
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    int req = -1;  // request index in flight
    size_t mem_off = 0, mem_len = 0;
    size_t out_u1 = 0, out_pred = 0, out_s = 0, out_scal = 0, out_stats = 0;
};

}  // namespace

extern "C" wos_status wos_serve(wos_ctx *ctx, const wos_request *reqs, int32_t n, wos_result *results,
                                const wos_serve_opts *opts)
{
    using clock = std::chrono::steady_clock;
    if (!ctx || (n > 0 && (!reqs || !results))) return set_error(WOS_EINVAL, "NULL argument");
    if (n < 0) return set_error(WOS_EINVAL, "n < 0");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    const int max_inflight = opts && opts->max_inflight > 0 ? std::min(opts->max_inflight, 64) : 4;
    size_t budget = opts && opts->hbm_budget_bytes ? opts->hbm_budget_bytes : (size_t(4) << 30);
    const double timeout = opts ? opts->timeout_s : 0.0;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(WOS_EDEVICE, "hipSetDevice failed");

    // validate and lay out every request up front
    std::vector<ReqLayout> lay(n);
    size_t max_stage = 0;
    for (int i = 0; i < n; ++i) {
        results[i].status = WOS_OK;
        results[i].t_arrive = reqs[i].arrival_s;
        results[i].t_admit = results[i].t_done = -1.0;
        results[i].walks = results[i].steps = 0;
        results[i].rank_used = 0;
        results[i].alpha_used = 0.0;
        wos_status st = layout_request(reqs[i], lay[i]);
        if (st != WOS_OK) {
            results[i].status = st;
            continue;
        }
        if (lay[i].total > budget) {
            results[i].status = set_error(WOS_ENOMEM, "request %d needs %zu bytes, budget %zu", i, lay[i].total, budget);
            continue;
        }
        if (!results[i].u1_host) {
            results[i].status = set_error(WOS_EINVAL, "request %d has no u1 output buffer", i);
            continue;
        }
        max_stage = std::max(max_stage, staging_bytes(reqs[i], lay[i]));
    }
    void *arena_mem = nullptr;
    wos_status st = ctx_malloc(ctx, &arena_mem, budget);
    if (st != WOS_OK) return st;
    Arena arena;
    arena.init(budget);
    std::vector<Slot> slots(max_inflight);
    for (auto &s : slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&s.pinned, std::max<size_t>(max_stage, 4096), hipHostMallocDefault) != hipSuccess) {
            ctx_free(ctx, arena_mem, budget);
            return set_error(WOS_EDEVICE, "serving slot set-up failed");
        }
        s.pinned_cap = std::max<size_t>(max_stage, 4096);
    }
    // requests in arrival order
    std::vector<int> order;
    for (int i = 0; i < n; ++i)
        if (results[i].status == WOS_OK) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

    const auto t0 = clock::now();
    auto now = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
    std::deque<int> queue;
    size_t next_arrival = 0;
    int inflight = 0;
    size_t done_count = 0;
    wos_status fatal = WOS_OK;

    auto launch = [&](Slot &s, int i) -> wos_status {
        const wos_request &r = reqs[i];
        ReqLayout &L = lay[i];
        uint8_t *base = static_cast<uint8_t *>(arena_mem) + s.mem_off;
        uint8_t *pin = static_cast<uint8_t *>(s.pinned);
        size_t po = 0;
        auto stage_in = [&](size_t dev_off, const void *src, size_t bytes) -> hipError_t {
            if (!bytes) return hipSuccess;
            std::memcpy(pin + po, src, bytes);
            hipError_t e = hipMemcpyAsync(base + dev_off, pin + po, bytes, hipMemcpyHostToDevice, s.stream);
            po += up256(bytes);
            return e;
        };
        hipError_t e = stage_in(L.off_x, r.x_obs_host, 8ull * r.n_obs * L.dim);
        if (e == hipSuccess) e = stage_in(L.off_uD, r.uD_host, 8ull * r.n_obs);
        if (e == hipSuccess && L.n0) e = stage_in(L.off_u0, r.u0_host, 8ull * L.n0);
        svd_bind(L.svd, base + L.off_svd);
        if (e == hipSuccess) e = svd_upload(L.svd, pin + po, s.stream);
        po += up256(svd_staging_bytes(L.svd));
        uint32_t *counts = reinterpret_cast<uint32_t *>(base + L.off_counts);
        uint64_t *stats = reinterpret_cast<uint64_t *>(base + L.off_stats);
        if (e == hipSuccess) e = fill_u32(counts, static_cast<size_t>(r.n_obs) * L.M, 0u, s.stream);
        if (e == hipSuccess) e = fill_u32(reinterpret_cast<uint32_t *>(stats), 2 * WOS_STATS_WORDS, 0u, s.stream);
        if (e != hipSuccess) return set_error(WOS_EDEVICE, "staging failed: %s", hipGetErrorString(e));
        wos_measure_job J;
        J.geom = r.geom;
        J.walk = r.walk;
        J.x_obs_dev = reinterpret_cast<const double *>(base + L.off_x);
        J.n_obs = r.n_obs;
        J.counts_dev = counts;
        J.stats_dev = stats;
        J.trace_dev = nullptr;
        {
            std::lock_guard<std::recursive_mutex> lk(ctx->launch_mu);
            wos_status st2 = build_batch(ctx, &J, 1, s.stream, nullptr);
            if (st2 != WOS_OK) return st2;
        }
        const uint64_t nw = r.walk.walk_end - r.walk.walk_begin;
        const int grid = svd_coop_grid(L.svd.v.rows, L.svd.v.colsp, ctx->n_cu);
        e = svd_launch(L.svd.v, counts, 1.0 / static_cast<double>(nw), grid, s.stream);
        double *u1 = reinterpret_cast<double *>(base + L.off_u1);
        double *pred = reinterpret_cast<double *>(base + L.off_pred);
        int32_t *rank = reinterpret_cast<int32_t *>(base + L.off_scal);
        double *alpha = reinterpret_cast<double *>(base + L.off_scal + 8);
        RegDev rg{r.reg.kind, r.reg.rank, r.reg.alpha, r.reg.noise_delta, r.reg.tau};
        if (e == hipSuccess)
            e = recon_launch(L.svd.v, counts, 1.0 / static_cast<double>(nw), reinterpret_cast<const double *>(base + L.off_uD),
                             L.n0 ? reinterpret_cast<const double *>(base + L.off_u0) : nullptr, rg, u1, pred, rank, alpha,
                             s.stream);
        // outputs back to pinned memory
        s.out_u1 = po; po += up256(8ull * L.n1);
        s.out_pred = po; po += up256(8ull * r.n_obs);
        s.out_s = po; po += up256(8ull * L.k);
        s.out_scal = po; po += up256(16);
        s.out_stats = po; po += up256(8ull * WOS_STATS_WORDS);
        if (e == hipSuccess) e = hipMemcpyAsync(pin + s.out_u1, u1, 8ull * L.n1, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pin + s.out_pred, pred, 8ull * r.n_obs, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pin + s.out_s, L.svd.v.s, 8ull * L.k, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pin + s.out_scal, base + L.off_scal, 16, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pin + s.out_stats, stats, 8ull * WOS_STATS_WORDS, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) return set_error(WOS_EDEVICE, "enqueue failed: %s", hipGetErrorString(e));
        return WOS_OK;
    };

    while (done_count < order.size() && fatal == WOS_OK) {
        const double t = now();
        while (next_arrival < order.size() && reqs[order[next_arrival]].arrival_s <= t) queue.push_back(order[next_arrival++]);
        // time out queued requests
        if (timeout > 0) {
            for (auto it = queue.begin(); it != queue.end();) {
                if (t - reqs[*it].arrival_s > timeout) {
                    results[*it].status = WOS_ETIMEOUT;
                    results[*it].t_done = t;
                    ++done_count;
                    it = queue.erase(it);
                } else {
                    ++it;
                }
            }
        }
        // admit in arrival order while a slot and memory are free
        while (!queue.empty() && inflight < max_inflight) {
            const int i = queue.front();
            size_t off = 0;
            if (!arena.alloc(lay[i].total, off)) break;  // wait for memory
            Slot *slot = nullptr;
            for (auto &s : slots)
                if (s.req < 0) {
                    slot = &s;
                    break;
                }
            slot->req = i;
            slot->mem_off = off;
            slot->mem_len = lay[i].total;
            queue.pop_front();
            results[i].t_admit = now();
            wos_status st2 = launch(*slot, i);
            if (st2 != WOS_OK) {
                fatal = st2;
                break;
            }
            ++inflight;
        }
        // completions
        bool any = false;
        for (auto &s : slots) {
            if (s.req < 0) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            const int i = s.req;
            wos_result &R = results[i];
            if (q != hipSuccess) {
                R.status = WOS_EDEVICE;
                fatal = set_error(WOS_EDEVICE, "request %d failed on the device: %s", i, hipGetErrorString(q));
            } else {
                const uint8_t *pin = static_cast<const uint8_t *>(s.pinned);
                std::memcpy(R.u1_host, pin + s.out_u1, 8ull * lay[i].n1);
                if (R.pred_host) std::memcpy(R.pred_host, pin + s.out_pred, 8ull * reqs[i].n_obs);
                if (R.s_host) std::memcpy(R.s_host, pin + s.out_s, 8ull * lay[i].k);
                std::memcpy(&R.rank_used, pin + s.out_scal, 4);
                std::memcpy(&R.alpha_used, pin + s.out_scal + 8, 8);
                uint64_t stw[WOS_STATS_WORDS];
                std::memcpy(stw, pin + s.out_stats, sizeof stw);
                R.walks = stw[WOS_STAT_WALKS];
                R.steps = stw[WOS_STAT_STEPS];
                R.t_done = now();
                if (timeout > 0 && R.t_done - R.t_arrive > timeout) R.status = WOS_ETIMEOUT;
            }
            arena.release(s.mem_off, s.mem_len);
            s.req = -1;
            --inflight;
            ++done_count;
            any = true;
        }
        if (!any) {
            const double next_t = next_arrival < order.size() ? reqs[order[next_arrival]].arrival_s : 1e300;
            if (inflight == 0 && queue.empty() && next_t > now())
                std::this_thread::sleep_for(std::chrono::duration<double>(std::min(next_t - now(), 0.001)));
            else
                std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    for (auto &s : slots) {
        (void)hipStreamSynchronize(s.stream);
        (void)hipStreamDestroy(s.stream);
        (void)hipEventDestroy(s.done);
        (void)hipHostFree(s.pinned);
    }
    ctx_free(ctx, arena_mem, budget);
    if (fatal != WOS_OK) {
        ctx->poisoned = fatal == WOS_EDEVICE;
        return fatal;
    }
    return WOS_OK;
}
