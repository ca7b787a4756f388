// walk_kernel.hip -- persistent walk-on-ellipsoids kernel for gfx950 (Algorithm MC-REM).
//
// Work decomposition: a work item is (instance, point i, chunk c of walk ids).  Blocks pull items
// from one global atomic cursor until the queue is empty, so uneven instances and geometric-tailed
// walk lengths share one launch.  Inside an item every wavefront keeps 64 walks in flight, one per
// lane; a lane whose walk stops is refilled with the next walk id of the item through a wave ballot
// and one LDS atomic for the whole wave (the paper's compaction of the active index vector).
//
// Randomness is counter-based (Philox4x32-10 keyed by instance seed; counter (block, walk, point,
// instance)), so which lane runs which walk never changes a result.  One Philox block feeds
// SPB consecutive steps of a walk (4 in 2D FP32, 2 in 3D FP32 and 2D FP64, 1 in 3D FP64); new
// walks start only at wave iterations that are multiples of SPB, which keeps every live lane of a
// wave on the same phase, so the generator runs wave-uniformly once per SPB steps.
//
// Stop points are appended to a per-wave LDS queue and binned 64 at a time (full-wave FP64
// projection), then counted in an LDS histogram row of the item's point; at the end of the item
// the non-zero bins are flushed to the count matrix in HBM with atomics.
#include <type_traits>

#include "wos_device.hpp"
#include "wos_internal.h"

namespace wos {

namespace {

constexpr int kWave = 64;

template <typename R, int DIM> struct Spb;
template <> struct Spb<float, 2> { static constexpr int v = 4; };
template <> struct Spb<float, 3> { static constexpr int v = 2; };
template <> struct Spb<double, 2> { static constexpr int v = 2; };
template <> struct Spb<double, 3> { static constexpr int v = 1; };

struct BlockShared {
    uint32_t item_lo, item_hi;
    uint32_t pad0, pad1;
    unsigned long long st[8]; // per-item statistics
};

// Number of set bits of a wave mask below the calling lane (v_mbcnt_lo/hi).
__device__ __forceinline__ uint32_t prefix_count(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Direction of step s (phase = s mod SPB) from the words of the walk's current Philox block.
template <typename R, int DIM> struct Dir;

template <> struct Dir<float, 2> {
    template <int PH> static __device__ __forceinline__ void get(const uint32_t w[4], float *U)
    {
        const float u = u24(w[PH]);
        // v_sin/v_cos take revolutions: sin(2 pi u), cos(2 pi u) without range reduction; their
        // norm error (below 2^-20) is covered by the radius shrink of the FP32 step
        U[0] = __builtin_amdgcn_cosf(u);
        U[1] = __builtin_amdgcn_sinf(u);
    }
};
template <> struct Dir<float, 3> {
    template <int PH> static __device__ __forceinline__ void get(const uint32_t w[4], float *U)
    {
        const float u1 = u24(w[2 * PH]);
        const float u2 = u24(w[2 * PH + 1]);
        const float z = 1.0f - 2.0f * u1;
        const float rho = __builtin_amdgcn_sqrtf(__builtin_fmaxf((1.0f - z) * (1.0f + z), 0.0f));
        U[0] = rho * __builtin_amdgcn_cosf(u2);
        U[1] = rho * __builtin_amdgcn_sinf(u2);
        U[2] = z;
    }
};
template <> struct Dir<double, 2> {
    template <int PH> static __device__ __forceinline__ void get(const uint32_t w[4], double *U)
    {
#pragma clang fp contract(off)
        const double u = u53(w[2 * PH], w[2 * PH + 1]);
        const double th = kTwoPi * u;
        double s, c;
        sincos(th, &s, &c);
        U[0] = c;
        U[1] = s;
    }
};
template <> struct Dir<double, 3> {
    template <int PH> static __device__ __forceinline__ void get(const uint32_t w[4], double *U)
    {
#pragma clang fp contract(off)
        const double z = 1.0 - 2.0 * u53(w[0], w[1]);
        const double ph = kTwoPi * u53(w[2], w[3]);
        const double rho = __builtin_sqrt((1.0 - z) * (1.0 + z));
        double s, c;
        sincos(ph, &s, &c);
        U[0] = rho * c;
        U[1] = rho * s;
        U[2] = z;
    }
};

// x <- x + r S U  (FP64 keeps the order of the definition; FP32 uses fused multiply-adds)
template <int DIM> __device__ __forceinline__ void step64(const DevInst &I, double *x, double r, const double *U)
{
#pragma clang fp contract(off)
    double y[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc += I.S[a * 3 + c] * U[c];
        y[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) x[a] = x[a] + r * y[a];
}
template <int DIM> __device__ __forceinline__ void step32(const DevInst &I, float *x, float r, const float *U)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc = __builtin_fmaf(I.Sf[a * 3 + c], U[c], acc);
        x[a] = __builtin_fmaf(r, acc, x[a]);
    }
}

// Per-wave stop queue in LDS (structure of arrays): stop position, walk offset, and the step
// count with the cap-hit flag in bit 31.
template <typename R, int DIM> struct StopQueue {
    R *pos;          // [DIM][kWave]
    uint32_t *koff;  // [kWave]
    uint32_t *steps; // [kWave]
};

constexpr uint32_t kCapBit = 0x80000000u;

// Per-lane statistics, accumulated 64 stops at a time when a queue is flushed.
struct LaneStats {
    uint32_t walks = 0, cap = 0, esc = 0, fp64 = 0, max_s = 0;
    unsigned long long steps = 0;
};

template <typename R, int DIM, int KIND>
__device__ __forceinline__ void flush_queue(const DevInst &I, const StopQueue<R, DIM> &q, uint32_t n,
                                            uint32_t point, uint32_t *hist, const PolySeg *segs,
                                            LaneStats &ls)
{
    const uint32_t lane = __lane_id();
    if (lane < n) {
        R xs[DIM];
        double x[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            xs[a] = q.pos[a * kWave + lane];
            x[a] = static_cast<double>(xs[a]) + origin<R, KIND>(I, a);
        }
        // FP32 positions on circles: the cell in FP32 where that is certain, else in FP64
        int j = -1;
        if constexpr (sizeof(R) == 4 && DIM == 2 && (KIND == kDisk || KIND == kAnnulus))
            j = element32_certified<KIND>(I, xs[0], xs[1]);
        if (j < 0) j = element64<KIND, DIM>(I, x, segs);
        atomicAdd(&hist[j], 1u);
        const uint32_t sw = q.steps[lane];
        const uint32_t st = sw & ~kCapBit;
        ls.walks += 1;
        ls.steps += st;
        ls.max_s = max(ls.max_s, st);
        ls.cap += sw >> 31;
        // escape (stop outside D): certain "no" when the FP32 distance exceeds its error bound
        bool maybe_out = true;
        if constexpr (sizeof(R) == 4 && KIND != kPolygon) maybe_out = !(dist32<KIND, DIM>(I, xs, segs) > I.delta);
        if (maybe_out && dist64<KIND, DIM>(I, x, segs) < 0.0) ls.esc += 1;
        if (I.trace) {
            const size_t t = (static_cast<size_t>(point) * I.n_walks + q.koff[lane]) * 2;
            I.trace[t] = j;
            I.trace[t + 1] = static_cast<int32_t>(st);
        }
    }
}

// Loop-invariant operands of the folded 2D FP32 step, held in VGPRs (a fused multiply-add has room
// for one scalar operand only, so scalar ones would cost a move per use).
struct Fold32 {
    float off0, off1, rs0, rs1, rn0, rn1;
};

// One sphere step of a live walk (phase PH of its Philox block).  A walk that stops gets d = -1
// when the decision was not the plain comparison d <= eps (FP64 band test, step cap), so that the
// caller's test d <= eps (FP64) / d <= eps_lo (FP32) alone tells which walks stopped.  At the cap,
// bit 31 of s is set.  CAP = false when no walk of the wave can reach the cap within this Philox
// block; then s is not advanced here (the caller adds the block's steps at its end and PH + 1 for
// a walk that stops inside it).
template <typename R, int DIM, int KIND, int PH, bool CAP>
__device__ __forceinline__ void walk_step(const DevInst &I, const PolySeg *segs, const uint32_t w[4], const Fold32 &F,
                                          R *x, R &d, uint32_t &s, uint32_t &n_fp64)
{
    if constexpr (sizeof(R) == 8) {
        R U[DIM];
        Dir<R, DIM>::template get<PH>(w, U);
        const double r = radius64<KIND, DIM>(I, x, d);
        step64<DIM>(I, x, r, U);
        d = dist64<KIND, DIM>(I, x, segs);
        s += 1;
        if (d > I.eps && s >= I.max_steps) {
            d = -1.0;
            s |= kCapBit;
        }
    } else {
        // conservative radius: below the true distance by more than the FP32 distance error
        // (2 delta) and the direction's norm error (relative 2^-16)
        const float rr = radius32<KIND, DIM>(I, x, d);
        if constexpr (DIM == 2) {
            const float t = static_cast<float>(w[PH] >> 8);
            const float c0 = __builtin_amdgcn_cosf(__builtin_fmaf(t, 0x1.0p-24f, F.off0));
            const float c1 = __builtin_amdgcn_cosf(__builtin_fmaf(t, 0x1.0p-24f, F.off1));
            x[0] = __builtin_fmaf(__builtin_fmaf(rr, F.rs0, F.rn0), c0, x[0]);
            x[1] = __builtin_fmaf(__builtin_fmaf(rr, F.rs1, F.rn1), c1, x[1]);
        } else {
            R U[DIM];
            Dir<R, DIM>::template get<PH>(w, U);
            const float r = __builtin_fmaf(rr, 1.0f - 0x1.0p-16f, I.neg2delta);
            step32<DIM>(I, x, r, U);
        }
        d = dist32<KIND, DIM>(I, x, segs);
        if constexpr (CAP) s += 1;
        if (d > I.eps_lo && d <= I.eps_hi) {
            // ambiguous band: decide in FP64 at the stored position
            double xd[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) xd[a] = static_cast<double>(x[a]) + origin<R, KIND>(I, a);
            if (!(dist64<KIND, DIM>(I, xd, segs) > I.eps)) d = -1.0f;
            ++n_fp64;
        }
        if constexpr (CAP) {
            if (d > I.eps_lo && s >= I.max_steps) {
                d = -1.0f;
                s |= kCapBit;
            }
        }
    }
}

template <typename R, int DIM, int KIND>
__device__ __forceinline__ void run_item(const DevInst &I, uint32_t point, uint32_t k0, uint32_t cnt, uint32_t *hist,
                         PolySeg *lds_segs, uint8_t *qbase, BlockShared &sh)
{
    constexpr int SPB = Spb<R, DIM>::v;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int M = I.n_elem;
    for (int j = tid; j < M; j += nthr) hist[j] = 0u;
    const PolySeg *segs = I.segs;
    if constexpr (KIND == kPolygon || KIND == kPerforated || KIND == kPerfBox) {  // edges / holes read every step
        for (int e = tid; e < I.n_verts; e += nthr) lds_segs[e] = I.segs[e];
        segs = lds_segs;
    }
    if (tid < 8) sh.st[tid] = 0ull;
    __syncthreads();

    double x0d[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) x0d[a] = I.x_obs[static_cast<size_t>(point) * DIM + a];
    const double d0d = dist64<KIND, DIM>(I, x0d, segs);

    if (!(d0d > I.eps)) {
        // The start point lies in the eps-shell (or outside D): every walk stops with zero steps
        // in the cell of the start point's projection.
        const int j0 = element64<KIND, DIM>(I, x0d, segs);
        if (tid == 0) {
            hist[j0] += cnt;
            sh.st[0] = cnt;
            if (d0d < 0.0) sh.st[4] = cnt;
        }
        if (I.trace) {
            for (uint32_t w = tid; w < cnt; w += nthr) {
                const size_t t = (static_cast<size_t>(point) * I.n_walks + k0 + w) * 2;
                I.trace[t] = j0;
                I.trace[t + 1] = 0;
            }
        }
    } else {
        const uint32_t lane = __lane_id();
        const int wv = tid / kWave;
        StopQueue<R, DIM> q;
        {
            uint8_t *b = qbase + static_cast<size_t>(wv) * kWave * (DIM * sizeof(R) + 8);
            q.pos = reinterpret_cast<R *>(b);
            q.koff = reinterpret_cast<uint32_t *>(b + kWave * DIM * sizeof(R));
            q.steps = q.koff + kWave;
        }
        R x0[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) x0[a] = static_cast<R>(x0d[a] - origin<R, KIND>(I, a));
        Fold32 F{};
        if constexpr (sizeof(R) == 4 && DIM == 2) {
            F = Fold32{I.fold_off[0], I.fold_off[1], I.fold_rs[0], I.fold_rs[1], I.fold_rn[0], I.fold_rn[1]};
            asm volatile("" : "+v"(F.off0), "+v"(F.off1), "+v"(F.rs0), "+v"(F.rs1), "+v"(F.rn0), "+v"(F.rn1));
        }
        R d0;
        if constexpr (sizeof(R) == 8) d0 = d0d; else d0 = dist32<KIND, DIM>(I, x0, segs);

        // A lane holds a walk while d is finite: d = +inf marks a free lane (a lane flag kept in
        // memory form would cost a compare and a select per phase).
        constexpr R kFree = static_cast<R>(__builtin_inf());
        uint32_t koff = 0, s = 0;
        R x[DIM];
        R d = kFree;
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[a] = x0[a];
        // The item's walks are dealt to the waves round-robin (walk offset wv + nw i for the wave's
        // i-th walk); within a wave, free lanes take the wave's next walks in lane order.
        const uint32_t nw = static_cast<uint32_t>(nthr / kWave);
        const uint32_t wave_cnt = cnt > static_cast<uint32_t>(wv) ? (cnt - wv + nw - 1) / nw : 0u;
        uint32_t wave_next = 0;  // wave-uniform
        uint32_t qn = 0;  // wave-uniform queue length
        uint32_t n_fp64 = 0;
        unsigned long long wave_iters = 0;
        LaneStats ls;

        // One outer iteration per Philox block: refill, draw the block, then SPB unrolled steps.
        for (;;) {
            const uint64_t need = __ballot(d == kFree);
            if (need != 0ull && wave_next < wave_cnt) {
                const uint32_t mine = wave_next + prefix_count(need);
                wave_next += static_cast<uint32_t>(__popcll(need));
                if (d == kFree && mine < wave_cnt) {
                    koff = k0 + static_cast<uint32_t>(wv) + nw * mine;
                    s = 0;
                    d = d0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) x[a] = x0[a];
                }
            }
            if (!__any(d != kFree)) break;
            uint32_t w[4];
            {
                uint32_t c0 = s / SPB, c1 = I.walk_begin + koff, c2 = point, c3 = I.inst;
                philox4x32_10(c0, c1, c2, c3, I.key0, I.key1);
                w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
            }
            wave_iters += SPB;
            // A walk that stops frees its lane in its phase (d = +inf, so the single compare below is
            // the stop mask of every phase) and joins the stop queue at the end of the block, all
            // stops of the block in one append.
            constexpr uint32_t kNoStop = 0xFFu;
            uint32_t fph = kNoStop;  // phase of the stop within the block
            auto phase = [&](auto ph_tag, auto cap_tag) {
                constexpr int PH = decltype(ph_tag)::value;
                constexpr bool CAP = decltype(cap_tag)::value;
                if (d != kFree) walk_step<R, DIM, KIND, PH, CAP>(I, segs, w, F, x, d, s, n_fp64);
                const bool fin = !(d > (sizeof(R) == 8 ? static_cast<R>(I.eps) : static_cast<R>(I.eps_lo)));
                fph = fin ? static_cast<uint32_t>(PH) : fph;
                d = fin ? kFree : d;
            };
            auto append = [&](auto cap_tag) {
                constexpr bool CAP = decltype(cap_tag)::value;
                const bool stopped = fph != kNoStop;
                const uint64_t fmask = __ballot(stopped);
                if (fmask != 0ull) {
                    const uint32_t nf = __popcll(fmask);
                    if (qn + nf > static_cast<uint32_t>(kWave)) {
                        flush_queue<R, DIM, KIND>(I, q, qn, point, hist, segs, ls);
                        qn = 0;
                    }
                    if (stopped) {
                        const uint32_t slot = qn + prefix_count(fmask);
#pragma unroll
                        for (int a = 0; a < DIM; ++a) q.pos[a * kWave + slot] = x[a];
                        q.koff[slot] = koff;
                        q.steps[slot] = (sizeof(R) == 8 || CAP) ? s : s + fph + 1;
                    }
                    qn += nf;
                }
            };
            auto block = [&](auto cap_tag) {
                phase(std::integral_constant<int, 0>{}, cap_tag);
                if constexpr (SPB > 1) phase(std::integral_constant<int, 1>{}, cap_tag);
                if constexpr (SPB > 2) {
                    phase(std::integral_constant<int, 2>{}, cap_tag);
                    phase(std::integral_constant<int, 3>{}, cap_tag);
                }
                append(cap_tag);
            };
            // FP32: the step cap is tested only in blocks where some walk can reach it (the second copy
            // of the block costs the FP64 variants more in registers than it saves)
            if constexpr (sizeof(R) == 4) {
                if (__any(d != kFree && s + SPB >= I.max_steps)) {
                    block(std::true_type{});
                } else {
                    block(std::false_type{});
                    s += SPB;  // steps of the block (the stops of the block were appended with s + PH + 1)
                }
            } else {
                block(std::true_type{});
            }
        }
        if (qn) flush_queue<R, DIM, KIND>(I, q, qn, point, hist, segs, ls);

        if (ls.walks) atomicAdd(&sh.st[0], static_cast<unsigned long long>(ls.walks));
        if (ls.steps) atomicAdd(&sh.st[1], ls.steps);
        if (ls.max_s) atomicMax(&sh.st[2], static_cast<unsigned long long>(ls.max_s));
        if (ls.cap) atomicAdd(&sh.st[3], static_cast<unsigned long long>(ls.cap));
        if (ls.esc) atomicAdd(&sh.st[4], static_cast<unsigned long long>(ls.esc));
        if (n_fp64) atomicAdd(&sh.st[5], static_cast<unsigned long long>(n_fp64));
        if (lane == 0) atomicAdd(&sh.st[6], wave_iters * kWave);
    }
    __syncthreads();
    uint32_t *row = I.counts + static_cast<size_t>(point) * M;
    for (int j = tid; j < M; j += nthr) {
        const uint32_t v = hist[j];
        if (v) atomicAdd(&row[j], v);
    }
    if (I.stats && tid < 7) {
        const unsigned long long v = sh.st[tid];
        if (tid == 2) {
            if (v) atomicMax(&I.stats[2], v);
        } else if (v) {
            atomicAdd(&I.stats[tid], v);
        }
    }
    __syncthreads();
}

// KSEL: the domain kind of every instance of the launch (its own register allocation), or -1 for
// launches that mix kinds (dispatch per item).
template <typename R, int DIM, int KSEL>
__global__ __launch_bounds__(1024) void walk_kernel(const DevInst *__restrict__ insts, int n_inst,
                                                    uint64_t total_items, uint32_t *cursor,
                                                    int hist_words, int seg_bytes)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ BlockShared sh;
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem);
    PolySeg *lds_segs = reinterpret_cast<PolySeg *>(smem + static_cast<size_t>(hist_words) * 4);
    uint8_t *qbase = smem + static_cast<size_t>(hist_words) * 4 + seg_bytes;

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t it = atomicAdd(cursor, 1u);
            sh.item_lo = it;
        }
        __syncthreads();
        const uint64_t item = __builtin_amdgcn_readfirstlane(sh.item_lo);
        __syncthreads();
        if (item >= total_items) return;
        // instance of this item (descriptors sorted by item_begin)
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (insts[mid].item_begin <= item) lo = mid; else hi = mid - 1;
        }
        const int idx = __builtin_amdgcn_readfirstlane(lo);
        const DevInst &I = insts[idx];
        const uint64_t local = item - I.item_begin;
        const uint64_t n_big_items = static_cast<uint64_t>(I.n_obs) * I.n_big;
        uint32_t point, k0, cnt;
        if (local < n_big_items) {
            point = static_cast<uint32_t>(local / I.n_big);
            k0 = static_cast<uint32_t>(local % I.n_big) * I.big_chunk;
            cnt = I.big_chunk;
        } else {
            const uint64_t l2 = local - n_big_items;
            point = static_cast<uint32_t>(l2 / I.n_chunks);
            k0 = I.n_big * I.big_chunk + static_cast<uint32_t>(l2 % I.n_chunks) * I.chunk;
            cnt = min(I.chunk, I.n_walks - k0);
        }
        if constexpr (KSEL >= 0) {
            run_item<R, DIM, KSEL>(I, point, k0, cnt, hist, lds_segs, qbase, sh);
        } else if constexpr (DIM == 2) {
            switch (I.kind) {
            case kDisk: run_item<R, 2, kDisk>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kAnnulus: run_item<R, 2, kAnnulus>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kEllipse: run_item<R, 2, kEllipse>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kPolygon: run_item<R, 2, kPolygon>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kPerforated: run_item<R, 2, kPerforated>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kPerfBox: run_item<R, 2, kPerfBox>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            default: run_item<R, 2, kBox>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            }
        } else {
            switch (I.kind) {
            case kBall: run_item<R, 3, kBall>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kPerforated: run_item<R, 3, kPerforated>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            case kPerfBox: run_item<R, 3, kPerfBox>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            default: run_item<R, 3, kBox>(I, point, k0, cnt, hist, lds_segs, qbase, sh); break;
            }
        }
    }
}

__global__ void reset_cursor_kernel(uint32_t *cursor) { *cursor = 0u; }

}  // namespace

size_t walk_queue_bytes(int precision, int dim, int block)
{
    const size_t rs = precision == 0 ? 8 : 4;
    return static_cast<size_t>(block / kWave) * kWave * (dim * rs + 8);
}

template <typename R, int DIM, int KSEL> static const void *kptr()
{
    return reinterpret_cast<const void *>(&walk_kernel<R, DIM, KSEL>);
}

template <typename R> static const void *kernel_of(int dim, int ksel)
{
    if (dim == 2) {
        switch (ksel) {
        case kDisk: return kptr<R, 2, kDisk>();
        case kAnnulus: return kptr<R, 2, kAnnulus>();
        case kEllipse: return kptr<R, 2, kEllipse>();
        case kPolygon: return kptr<R, 2, kPolygon>();
        case kPerforated: return kptr<R, 2, kPerforated>();
        case kPerfBox: return kptr<R, 2, kPerfBox>();
        case kBox: return kptr<R, 2, kBox>();
        default: return kptr<R, 2, -1>();
        }
    }
    switch (ksel) {
    case kBall: return kptr<R, 3, kBall>();
    case kPerforated: return kptr<R, 3, kPerforated>();
    case kPerfBox: return kptr<R, 3, kPerfBox>();
    case kBox: return kptr<R, 3, kBox>();
    default: return kptr<R, 3, -1>();
    }
}

const void *walk_kernel_ptr(int precision, int dim, int kind_sel)
{
    return precision == 0 ? kernel_of<double>(dim, kind_sel) : kernel_of<float>(dim, kind_sel);
}

hipError_t launch_walks(int precision, int dim, int kind_sel, const DevInst *insts, int n_inst, uint64_t total_items,
                        uint32_t *cursor, int hist_words, int seg_bytes, int block, int grid,
                        hipStream_t stream)
{
    reset_cursor_kernel<<<1, 1, 0, stream>>>(cursor);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = static_cast<size_t>(hist_words) * 4 + seg_bytes + walk_queue_bytes(precision, dim, block);
    const void *fn = walk_kernel_ptr(precision, dim, kind_sel);
    void *args[] = {&insts, &n_inst, &total_items, &cursor, &hist_words, &seg_bytes};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
}

}  // namespace wos
