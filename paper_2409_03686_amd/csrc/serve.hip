// serve.hip -- continuous batching of build + SVD + reconstruct requests (wos_serve).
//
// The blocking driver (wos_serve) replays the arrival times (open loop) on the calling thread; the
// live form (wos_serve_start / submit / poll / stop) runs the same engine on a thread owned by the
// context.  A request is admitted when one of
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
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
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
    int M = 0, n1 = 0, n0 = 0, k = 0, kfull = 0, dim = 2;
    size_t off_x, off_counts, off_stats, off_uD, off_u0, off_u1, off_pred, off_scal, off_svd, total;
    SvdHost svd;
};

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

wos_status layout_request(const wos_request &r, ReqLayout &L, int svd_mode)
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
    st = svd_layout(r.n_obs, M, r.gamma1_mask_host, sigma.data(), nullptr, L.svd, svd_mode != 0 ? kTruncRank : 0);
    if (st != WOS_OK) return st;
    L.svd.v.certified = svd_mode == 2 ? 1 : 0;
    st = check_reg(&r.reg);
    if (st != WOS_OK) return st;
    L.M = M;
    L.dim = r.geom.dim;
    L.n1 = L.svd.v.n;
    L.n0 = L.svd.v.n0;
    L.k = L.svd.v.k;
    L.kfull = std::min(L.svd.v.m, L.svd.v.n);
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
    struct Job *job = nullptr;  // request in flight
    size_t mem_off = 0, mem_len = 0;
    size_t out_u1 = 0, out_pred = 0, out_s = 0, out_scal = 0, out_stats = 0;
};

// One request inside the engine.  The blocking driver points req/res at the caller's memory; the
// live form owns copies of the inputs and of the outputs until they are polled.
struct Job {
    wos_request req{};
    wos_result *res = nullptr;
    ReqLayout L;
    std::vector<double> x, uD, u0, u1, pred, sv, verts;
    std::vector<uint8_t> mask;
    wos_result own{};
    bool full = false;  // served by the full SVD after the truncated one could not resolve its rank
    bool done = false;
};

// Admission, launch and completion of requests on max_inflight slots (a stream, an event and a
// pinned staging buffer each) with their device memory sub-allocated from one arena.
class Engine {
  public:
    Engine(wos_ctx *ctx, const wos_serve_opts *opts) : ctx_(ctx)
    {
        max_inflight_ = opts && opts->max_inflight > 0 ? std::min(opts->max_inflight, 64) : 4;
        budget_ = opts && opts->hbm_budget_bytes ? opts->hbm_budget_bytes : (size_t(4) << 30);
        timeout_ = opts ? opts->timeout_s : 0.0;
        svd_mode_ = opts ? opts->svd_mode : 0;
    }
    ~Engine() { shutdown(); }

    wos_status init(size_t stage_hint)
    {
        if (hipSetDevice(ctx_->device) != hipSuccess) return set_error(WOS_EDEVICE, "hipSetDevice failed");
        wos_status st = ctx_malloc(ctx_, &arena_mem_, budget_);
        if (st != WOS_OK) return st;
        arena_.init(budget_);
        slots_.resize(max_inflight_);
        // Each of the first kMaskedSlots slots gets a stream with a CU mask of its own (every CU but
        // one, a different one per slot): HIP gives such a stream a hardware queue of its own, so a
        // request's chain of small dependent kernels (the single-workgroup factor and Jacobi kernels
        // above all) does not wait behind another request's kernels in a shared queue (plain streams
        // share the process's few hardware queues).  Further slots use plain streams.
        constexpr size_t kMaskedSlots = 16;
        const int words = (ctx_->n_cu + 31) / 32;
        std::vector<uint32_t> mask(words);
        for (size_t i = 0; i < slots_.size(); ++i) {
            Slot &s = slots_[i];
            std::fill(mask.begin(), mask.end(), 0u);
            for (int c = 0; c < ctx_->n_cu; ++c)
                if (c != static_cast<int>(i % ctx_->n_cu)) mask[c / 32] |= 1u << (c % 32);
            const hipError_t se = i < kMaskedSlots && ctx_->n_cu > 1
                                      ? hipExtStreamCreateWithCUMask(&s.stream, static_cast<uint32_t>(words), mask.data())
                                      : hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
            if (se != hipSuccess || hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
                return set_error(WOS_EDEVICE, "serving slot set-up failed");
            if (!grow_pinned(s, std::max<size_t>(stage_hint, 4096))) return set_error(WOS_EDEVICE, "pinned staging allocation failed");
        }
        return WOS_OK;
    }

    // Validates and lays out a request; on failure the status is recorded in the job's result.
    wos_status prepare(Job &j)
    {
        wos_status st = (svd_mode_ >= 0 && svd_mode_ <= 2) ? layout_request(j.req, j.L, svd_mode_)
                                                           : set_error(WOS_EINVAL, "svd_mode must be 0, 1 or 2");
        if (st == WOS_OK && j.L.total > budget_)
            st = set_error(WOS_ENOMEM, "request needs %zu bytes, budget %zu", j.L.total, budget_);
        if (st == WOS_OK && !j.res->u1_host) st = set_error(WOS_EINVAL, "request has no u1 output buffer");
        j.res->status = st;
        return st;
    }

    double timeout() const { return timeout_; }
    int inflight() const { return inflight_; }
    bool has_retry() const { return !retry_.empty(); }

    // Admits queued jobs in order while a slot and memory are free.  Returns a fatal status.
    wos_status admit(std::deque<Job *> &queue, double now)
    {
        // requests sent back for the full SVD go first
        while ((!retry_.empty() || !queue.empty()) && inflight_ < max_inflight_) {
            std::deque<Job *> &from = retry_.empty() ? queue : retry_;
            Job *j = from.front();
            size_t off = 0;
            if (!arena_.alloc(j->L.total, off)) break;  // wait for memory
            Slot *slot = nullptr;
            for (auto &sl : slots_)
                if (!sl.job) {
                    slot = &sl;
                    break;
                }
            slot->job = j;
            slot->mem_off = off;
            slot->mem_len = j->L.total;
            from.pop_front();
            if (!j->full) j->res->t_admit = now;
            wos_status st = launch(*slot, *j);
            if (st != WOS_OK) return st;
            ++inflight_;
        }
        return WOS_OK;
    }

    // Harvests finished requests; returns how many finished (fatal device errors in *fatal).
    int complete(double now, wos_status *fatal)
    {
        int n = 0;
        for (auto &s : slots_) {
            if (!s.job) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            Job &j = *s.job;
            wos_result &R = *j.res;
            if (q != hipSuccess) {
                R.status = WOS_EDEVICE;
                *fatal = set_error(WOS_EDEVICE, "request failed on the device: %s", hipGetErrorString(q));
            } else if (svd_mode_ == 2 && !j.full &&
                       static_cast<const uint8_t *>(s.pinned)[s.out_scal + 4] != 0 && resubmit_full(j)) {
                // the truncated SVD's trusted triplets do not meet the regularisation rule: the
                // request runs again with the full SVD (the same walks, so the same counts)
                arena_.release(s.mem_off, s.mem_len);
                s.job = nullptr;
                --inflight_;
                continue;
            } else {
                const uint8_t *pin = static_cast<const uint8_t *>(s.pinned);
                std::memcpy(R.u1_host, pin + s.out_u1, 8ull * j.L.n1);
                if (R.pred_host) std::memcpy(R.pred_host, pin + s.out_pred, 8ull * j.req.n_obs);
                if (R.s_host) {
                    std::memcpy(R.s_host, pin + s.out_s, 8ull * j.L.k);
                    std::fill(R.s_host + j.L.k, R.s_host + j.L.kfull, 0.0);
                }
                std::memcpy(&R.rank_used, pin + s.out_scal, 4);
                std::memcpy(&R.alpha_used, pin + s.out_scal + 8, 8);
                uint64_t stw[WOS_STATS_WORDS];
                std::memcpy(stw, pin + s.out_stats, sizeof stw);
                R.walks = stw[WOS_STAT_WALKS];
                R.steps = stw[WOS_STAT_STEPS];
                R.svd_fallback = j.full ? 1 : 0;
                R.t_done = now;
                if (timeout_ > 0 && R.t_done - R.t_arrive > timeout_) R.status = WOS_ETIMEOUT;
            }
            j.done = true;
            arena_.release(s.mem_off, s.mem_len);
            s.job = nullptr;
            --inflight_;
            ++n;
        }
        return n;
    }

    void shutdown()
    {
        for (auto &s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.pinned) (void)hipHostFree(s.pinned);
            s = Slot{};
        }
        slots_.clear();
        if (arena_mem_) ctx_free(ctx_, arena_mem_, budget_);
        arena_mem_ = nullptr;
    }

  private:
    // Lays the request out again for the full SVD and queues it for admission; false (with the
    // request's status set) when it cannot be.
    bool resubmit_full(Job &j)
    {
        ReqLayout L;
        wos_status st = layout_request(j.req, L, 0);
        if (st == WOS_OK && L.total > budget_)
            st = set_error(WOS_ENOMEM, "request needs %zu bytes for the full SVD, budget %zu", L.total, budget_);
        if (st != WOS_OK) {
            j.res->status = st;
            return false;
        }
        j.L = L;
        j.full = true;
        retry_.push_back(&j);
        return true;
    }

    bool grow_pinned(Slot &s, size_t need)
    {
        if (s.pinned_cap >= need) return true;
        if (s.pinned) (void)hipHostFree(s.pinned);
        s.pinned = nullptr;
        s.pinned_cap = 0;
        if (hipHostMalloc(&s.pinned, need, hipHostMallocDefault) != hipSuccess) return false;
        s.pinned_cap = need;
        return true;
    }

    wos_status launch(Slot &s, Job &j)
    {
        const wos_request &r = j.req;
        ReqLayout &L = j.L;
        if (!grow_pinned(s, staging_bytes(r, L))) return set_error(WOS_EDEVICE, "pinned staging allocation failed");
        uint8_t *base = static_cast<uint8_t *>(arena_mem_) + s.mem_off;
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
            std::lock_guard<std::recursive_mutex> lk(ctx_->launch_mu);
            wos_status st2 = build_batch(ctx_, &J, 1, s.stream, nullptr);
            if (st2 != WOS_OK) return st2;
        }
        const uint64_t nw = r.walk.walk_end - r.walk.walk_begin;
        if (e == hipSuccess) {
            if (L.svd.v.tk) {
                e = tsvd_launch(L.svd.v, counts, 1.0 / static_cast<double>(nw), r.walk.seed ^ (uint64_t(r.walk.instance) << 32) ^ 0x9e3779b97f4a7c15ull, s.stream);
            } else {
                const int cus = stream_cus(ctx_, s.stream);
                const int grid = svd_coop_grid(L.svd.v.rows, L.svd.v.colsp, cus);
                e = svd_launch(L.svd.v, counts, 1.0 / static_cast<double>(nw), grid, cus, s.stream);
            }
        }
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
        // the certified truncated path's flag (rank beyond its trusted triplets) into the scalars'
        // spare word
        if (e == hipSuccess && L.svd.v.tk && L.svd.v.certified)
            e = hipMemcpyAsync(pin + s.out_scal + 4, L.svd.v.ctrl + kCtrlUnresolved, 4, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(pin + s.out_stats, stats, 8ull * WOS_STATS_WORDS, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) return set_error(WOS_EDEVICE, "enqueue failed: %s", hipGetErrorString(e));
        return WOS_OK;
    }

    wos_ctx *ctx_;
    int max_inflight_ = 4, inflight_ = 0;
    size_t budget_ = 0;
    double timeout_ = 0.0;
    int svd_mode_ = 0;
    void *arena_mem_ = nullptr;
    Arena arena_;
    std::vector<Slot> slots_;
    std::deque<Job *> retry_;
};

}  // namespace

extern "C" wos_status wos_serve(wos_ctx *ctx, const wos_request *reqs, int32_t n, wos_result *results,
                                const wos_serve_opts *opts)
{
    using clock = std::chrono::steady_clock;
    if (!ctx || (n > 0 && (!reqs || !results))) return set_error(WOS_EINVAL, "NULL argument");
    if (n < 0) return set_error(WOS_EINVAL, "n < 0");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    Engine eng(ctx, opts);
    // validate and lay out every request up front
    std::vector<Job> jobs(n);
    size_t max_stage = 0;
    for (int i = 0; i < n; ++i) {
        Job &j = jobs[i];
        j.req = reqs[i];
        j.res = &results[i];
        results[i].t_arrive = reqs[i].arrival_s;
        results[i].t_admit = results[i].t_done = -1.0;
        results[i].walks = results[i].steps = 0;
        results[i].rank_used = 0;
        results[i].alpha_used = 0.0;
        results[i].svd_fallback = 0;
        if (eng.prepare(j) == WOS_OK) max_stage = std::max(max_stage, staging_bytes(reqs[i], j.L));
    }
    wos_status st = eng.init(max_stage);
    if (st != WOS_OK) return st;
    // requests in arrival order
    std::vector<int> order;
    for (int i = 0; i < n; ++i)
        if (results[i].status == WOS_OK) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

    const auto t0 = clock::now();
    auto now = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
    std::deque<Job *> queue;
    size_t next_arrival = 0, done_count = 0;
    wos_status fatal = WOS_OK;
    const double timeout = eng.timeout();
    while (done_count < order.size() && fatal == WOS_OK) {
        const double t = now();
        while (next_arrival < order.size() && reqs[order[next_arrival]].arrival_s <= t) queue.push_back(&jobs[order[next_arrival++]]);
        if (timeout > 0) {  // time out queued requests
            for (auto it = queue.begin(); it != queue.end();) {
                if (t - (*it)->req.arrival_s > timeout) {
                    (*it)->res->status = WOS_ETIMEOUT;
                    (*it)->res->t_done = t;
                    ++done_count;
                    it = queue.erase(it);
                } else {
                    ++it;
                }
            }
        }
        fatal = eng.admit(queue, now());
        if (fatal != WOS_OK) break;
        const int fin = eng.complete(now(), &fatal);
        done_count += static_cast<size_t>(fin);
        if (fin == 0) {
            const double next_t = next_arrival < order.size() ? reqs[order[next_arrival]].arrival_s : 1e300;
            if (eng.inflight() == 0 && queue.empty() && !eng.has_retry() && next_t > now())
                std::this_thread::sleep_for(std::chrono::duration<double>(std::min(next_t - now(), 0.001)));
            else
                std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    eng.shutdown();
    if (fatal != WOS_OK) {
        ctx->poisoned = fatal == WOS_EDEVICE;
        return fatal;
    }
    return WOS_OK;
}

// ---------------------------------------------------------------------------------------------
// Live form: a serving thread owned by the context; requests are submitted and polled by ticket.
// ---------------------------------------------------------------------------------------------
struct LiveServer {
    wos_ctx *ctx = nullptr;
    std::unique_ptr<Engine> eng;
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> pending;                    // submitted, not yet seen by the thread
    std::map<uint64_t, std::unique_ptr<Job>> jobs;  // every ticket not yet polled
    uint64_t next_ticket = 1;
    bool stop = false;
    wos_status fatal = WOS_OK;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    void run()
    {
        std::deque<Job *> queue;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                if (queue.empty() && eng->inflight() == 0 && pending.empty() && !eng->has_retry())
                    cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] { return stop || !pending.empty(); });
                if (stop && pending.empty() && queue.empty() && eng->inflight() == 0 && !eng->has_retry()) return;
                while (!pending.empty()) {
                    queue.push_back(pending.front());
                    pending.pop_front();
                }
            }
            const double t = now();
            const double timeout = eng->timeout();
            int finished = 0;
            if (timeout > 0) {
                for (auto it = queue.begin(); it != queue.end();) {
                    if (t - (*it)->res->t_arrive > timeout) {
                        std::lock_guard<std::mutex> lk(mu);
                        (*it)->res->status = WOS_ETIMEOUT;
                        (*it)->res->t_done = t;
                        (*it)->done = true;
                        ++finished;
                        it = queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            wos_status f = WOS_OK;
            if (fatal == WOS_OK) f = eng->admit(queue, now());
            {
                std::lock_guard<std::mutex> lk(mu);
                if (f == WOS_OK) finished += eng->complete(now(), &f);
                if (f != WOS_OK && fatal == WOS_OK) {
                    fatal = f;
                    ctx->poisoned = f == WOS_EDEVICE;
                }
                if (fatal != WOS_OK) {  // fail whatever is still queued
                    for (Job *j : queue) {
                        j->res->status = fatal;
                        j->done = true;
                    }
                    finished += static_cast<int>(queue.size());
                    queue.clear();
                }
            }
            if (finished) cv_done.notify_all();
            if (finished == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
};

void wos::live_server_stop(wos_ctx *ctx)
{
    LiveServer *L = ctx->live;
    if (!L) return;
    {
        std::lock_guard<std::mutex> lk(L->mu);
        L->stop = true;
    }
    L->cv_work.notify_all();
    if (L->thr.joinable()) L->thr.join();
    L->eng->shutdown();
    delete L;
    ctx->live = nullptr;
}

extern "C" wos_status wos_serve_start(wos_ctx *ctx, const wos_serve_opts *opts)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx is NULL");
    if (ctx->poisoned) return set_error(WOS_EDEVICE, "context is unusable after a device error");
    if (ctx->live) return set_error(WOS_EBUSY, "the live server of this context is already running");
    auto *L = new LiveServer();
    L->ctx = ctx;
    L->eng = std::make_unique<Engine>(ctx, opts);
    wos_status st = L->eng->init(4096);
    if (st != WOS_OK) {
        delete L;
        return st;
    }
    L->t0 = std::chrono::steady_clock::now();
    ctx->live = L;
    L->thr = std::thread([L] {
        (void)hipSetDevice(L->ctx->device);
        L->run();
    });
    return WOS_OK;
}

extern "C" wos_status wos_serve_stop(wos_ctx *ctx)
{
    if (!ctx) return set_error(WOS_EINVAL, "ctx is NULL");
    if (!ctx->live) return set_error(WOS_EINVAL, "no live server is running");
    live_server_stop(ctx);
    return WOS_OK;
}

extern "C" wos_status wos_serve_submit(wos_ctx *ctx, const wos_request *req, uint64_t *ticket)
{
    if (!ctx || !req || !ticket) return set_error(WOS_EINVAL, "NULL argument");
    LiveServer *L = ctx->live;
    if (!L) return set_error(WOS_EINVAL, "no live server is running (wos_serve_start)");
    auto j = std::make_unique<Job>();
    j->req = *req;
    j->res = &j->own;
    // own copies of the host inputs, so the caller may reuse its buffers after this call
    int M = 0;
    wos_status st = validate_geometry(&req->geom, &M);
    if (st != WOS_OK) return st;
    if (req->n_obs < 1 || !req->x_obs_host || !req->uD_host || !req->gamma1_mask_host)
        return set_error(WOS_EINVAL, "request needs points, data and the Gamma_1 mask");
    j->x.assign(req->x_obs_host, req->x_obs_host + static_cast<size_t>(req->n_obs) * req->geom.dim);
    j->uD.assign(req->uD_host, req->uD_host + req->n_obs);
    j->mask.assign(req->gamma1_mask_host, req->gamma1_mask_host + M);
    int n0 = 0;
    for (int e = 0; e < M; ++e) n0 += j->mask[e] ? 0 : 1;
    if (n0 > 0) {
        if (!req->u0_host) return set_error(WOS_EINVAL, "request needs u0 (Gamma_0 is not empty)");
        j->u0.assign(req->u0_host, req->u0_host + n0);
    }
    j->req.x_obs_host = j->x.data();
    j->req.uD_host = j->uD.data();
    j->req.u0_host = n0 ? j->u0.data() : nullptr;
    j->req.gamma1_mask_host = j->mask.data();
    if (req->geom.verts && req->geom.n_verts > 0) {  // polygon vertices, holes, or mesh triangles
        const size_t nv = wos::vertex_doubles(&req->geom);
        j->verts.assign(req->geom.verts, req->geom.verts + nv);
        j->req.geom.verts = j->verts.data();
    }
    const int n1 = M - n0, k = std::min(req->n_obs, n1);
    j->u1.assign(std::max(n1, 1), 0.0);
    j->pred.assign(req->n_obs, 0.0);
    j->sv.assign(std::max(k, 1), 0.0);
    j->own.u1_host = j->u1.data();
    j->own.pred_host = j->pred.data();
    j->own.s_host = j->sv.data();
    j->own.t_admit = j->own.t_done = -1.0;
    st = L->eng->prepare(*j);
    if (st != WOS_OK) return st;
    std::lock_guard<std::mutex> lk(L->mu);
    if (L->fatal != WOS_OK) return set_error(L->fatal, "the live server stopped after a device error");
    j->own.t_arrive = L->now();
    *ticket = L->next_ticket++;
    L->pending.push_back(j.get());
    L->jobs.emplace(*ticket, std::move(j));
    L->cv_work.notify_one();
    return WOS_OK;
}

extern "C" wos_status wos_serve_poll(wos_ctx *ctx, uint64_t ticket, wos_result *out, int32_t wait_ms)
{
    if (!ctx || !out) return set_error(WOS_EINVAL, "NULL argument");
    LiveServer *L = ctx->live;
    if (!L) return set_error(WOS_EINVAL, "no live server is running");
    std::unique_lock<std::mutex> lk(L->mu);
    auto it = L->jobs.find(ticket);
    if (it == L->jobs.end()) return set_error(WOS_EINVAL, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    Job *j = it->second.get();
    if (!j->done && wait_ms != 0) {
        auto pred = [&] { return j->done; };
        if (wait_ms < 0) L->cv_done.wait(lk, pred);
        else L->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
    }
    if (!j->done) return WOS_EBUSY;
    const wos_result &R = j->own;
    if (out->u1_host) std::memcpy(out->u1_host, j->u1.data(), 8ull * j->L.n1);
    if (out->pred_host) std::memcpy(out->pred_host, j->pred.data(), 8ull * j->req.n_obs);
    if (out->s_host) std::memcpy(out->s_host, j->sv.data(), 8ull * j->sv.size());
    out->rank_used = R.rank_used;
    out->alpha_used = R.alpha_used;
    out->status = R.status;
    out->t_arrive = R.t_arrive;
    out->t_admit = R.t_admit;
    out->t_done = R.t_done;
    out->walks = R.walks;
    out->steps = R.steps;
    out->svd_fallback = R.svd_fallback;
    L->jobs.erase(it);
    return WOS_OK;
}
