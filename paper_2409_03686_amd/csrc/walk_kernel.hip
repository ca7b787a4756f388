// walk_kernel.hip -- persistent walk-on-ellipsoids kernel for gfx950 (Algorithm MC-REM).
//
// Work decomposition: a work item is (instance, point i, chunk c of walk ids).  Blocks pull items
// from one global atomic cursor until the queue is empty, so uneven instances and geometric-tailed
// walk lengths share one launch.  Inside an item every wavefront keeps 64 walks in flight, one per
// lane; a lane whose walk stops is refilled with the wave's next walk id through a wave ballot and
// a prefix count over it (the paper's compaction of the active index vector); the item's walks are
// dealt to its waves round-robin, so no atomic is needed.  Two other owners of the work exist:
// waves owning items (run_chain, overlapping consecutive items) and blocks owning points (walks
// reserved chunk by chunk from a per-point cursor); the launch mode picks one.
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
#include <algorithm>
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
        // error (below 2^-20 each) is covered by the radius shrink of the FP32 step
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
        double s, c;
        sincos2pi(u53(w[2 * PH], w[2 * PH + 1]), &s, &c);
        U[0] = c;
        U[1] = s;
    }
};
template <> struct Dir<double, 3> {
    template <int PH> static __device__ __forceinline__ void get(const uint32_t w[4], double *U)
    {
#pragma clang fp contract(off)
        const double z = 1.0 - 2.0 * u53(w[0], w[1]);
        const double rho = __builtin_sqrt((1.0 - z) * (1.0 + z));
        double s, c;
        sincos2pi(u53(w[2], w[3]), &s, &c);
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
    uint32_t *slot;  // [kWave], wave-item mode only: the item slot (0 or 1) of the entry
};

constexpr uint32_t kCapBit = 0x80000000u;

// Per-lane statistics, accumulated 64 stops at a time when a queue is flushed.
struct LaneStats {
    uint32_t walks = 0, cap = 0, esc = 0, fp64 = 0, max_s = 0;
    unsigned long long steps = 0;
};

// W (wave-item mode): an entry belongs to item slot q.slot[lane], whose point is point1 for slot 1,
// and its cell goes to that slot's histogram row (hist + slot hist_words).
template <typename R, int DIM, int KIND, bool W = false>
__device__ __forceinline__ void flush_queue(const DevInst &I, const StopQueue<R, DIM> &q, uint32_t n,
                                            uint32_t point0, uint32_t *hist0, const PolySeg *segs,
                                            LaneStats &ls, uint32_t point1 = 0, int hist_words = 0)
{
    const uint32_t lane = __lane_id();
    if (lane < n) {
        uint32_t point = point0;
        uint32_t *hist = hist0;
        if constexpr (W) {
            if (q.slot[lane]) {
                point = point1;
                hist = hist0 + hist_words;
            }
        }
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
        // escape (stop outside D): certain "no" when the FP32 distance exceeds its error bound; a mesh's
        // walk distance is unsigned, its escapes are decided at the start point
        bool maybe_out = KIND != kTriMesh;
        if constexpr (sizeof(R) == 4 && KIND != kPolygon && KIND != kTriMesh)
            maybe_out = !(dist32<KIND, DIM>(I, xs, segs) > I.delta);
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
template <typename R, int DIM, int KIND, int PH, bool CAP, int RV>
__device__ __forceinline__ void walk_step(const DevInst &I, const PolySeg *segs, const uint32_t w[4], const Fold32 &F,
                                          R *x, R &d, uint32_t &s, uint32_t &n_fp64, int &hint, R &rnext)
{
    // Meshes with the mapped-exact radius: the radius at the new position is computed right after the
    // step (rnext, used by the next step), and since the step ellipsoid holds the ball of radius
    // sigma_min r and touches dD, sigma_min r <= dist <= r: while sigma_min r is above the exit
    // threshold the walk certainly goes on and the search of the surface itself is skipped.
    constexpr bool kMeshMapped = KIND == kTriMesh;
    const bool mapped = kMeshMapped && I.radius_mode == 1;
    if constexpr (sizeof(R) == 8) {
        R U[DIM];
        Dir<R, DIM>::template get<PH>(w, U);
        const double r = (mapped && rnext >= 0.0) ? static_cast<double>(rnext) : radius64<KIND, DIM, RV>(I, x, d, segs);
        step64<DIM>(I, x, r, U);
        if (mapped) {
            rnext = radius64<KIND, DIM, RV>(I, x, d, segs);
            const double lb = rnext * I.mesh_sig64;
            d = lb > I.eps ? lb : dist64<KIND, DIM>(I, x, segs, &hint);
        } else {
            d = dist64<KIND, DIM>(I, x, segs, &hint);
        }
        s += 1;
        if (d > I.eps && s >= I.max_steps) {
            d = -1.0;
            s |= kCapBit;
        }
    } else {
        // conservative radius: below the true distance by more than the FP32 distance error
        // (2 delta) and the direction's error (the relative shrink 1 - rshrink)
        const float rr = (mapped && rnext >= 0.0f) ? static_cast<float>(rnext) : radius32<KIND, DIM, RV>(I, x, d, segs);
        if constexpr (DIM == 2) {
            const float t = static_cast<float>(w[PH] >> 8);
            const float c0 = __builtin_amdgcn_cosf(__builtin_fmaf(t, 0x1.0p-24f, F.off0));
            const float c1 = __builtin_amdgcn_cosf(__builtin_fmaf(t, 0x1.0p-24f, F.off1));
            x[0] = __builtin_fmaf(__builtin_fmaf(rr, F.rs0, F.rn0), c0, x[0]);
            x[1] = __builtin_fmaf(__builtin_fmaf(rr, F.rs1, F.rn1), c1, x[1]);
        } else {
            R U[DIM];
            Dir<R, DIM>::template get<PH>(w, U);
            const float r = __builtin_fmaf(rr, I.rshrink, I.neg2delta);
            step32<DIM>(I, x, r, U);
        }
        bool certain = false;
        if (mapped) {
            rnext = radius32<KIND, DIM, RV>(I, x, d, segs);  // below the mapped distance (its error bound is off)
            const float lb = rnext * I.mesh_sig32;
            certain = lb > I.eps_hi;
            d = certain ? lb : dist32<KIND, DIM>(I, x, segs, &hint);
        } else {
            d = dist32<KIND, DIM>(I, x, segs, &hint);
        }
        if constexpr (CAP) s += 1;
        if (!certain && d > I.eps_lo && d <= I.eps_hi) {
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

// PTS (point mode): the block runs point `point` with no fixed walk range; its waves reserve the
// point's walks I.chunk at a time from the point's walk cursor *pcur until it passes N, so the
// lanes drain only when the point's walks run out (several blocks may share a point).
template <typename R, int DIM, int KIND, bool PTS = false, int RV = -1>
__device__ __forceinline__ void run_item(const DevInst &I, uint32_t point, uint32_t k0, uint32_t cnt, uint32_t *hist,
                         PolySeg *lds_segs, uint8_t *qbase, BlockShared &sh, uint32_t *pcur = nullptr)
{
    constexpr int SPB = Spb<R, DIM>::v;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int M = I.n_elem;
    for (int j = tid; j < M; j += nthr) hist[j] = 0u;
    const PolySeg *segs = I.segs;
    if constexpr (KIND == kPolygon || KIND == kPerforated || KIND == kPerfBox) {  // edges / holes read every step
        for (int e = tid; e < I.n_segs; e += nthr) lds_segs[e] = I.segs[e];
        segs = lds_segs;
    }
    if (tid < 8) sh.st[tid] = 0ull;
    __syncthreads();

    double x0d[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) x0d[a] = I.x_obs[static_cast<size_t>(point) * DIM + a];
    const double d0d = start_dist64<KIND, DIM>(I, x0d, segs);  // every thread of the block, converged

    if (!(d0d > I.eps)) {
        // The start point lies in the eps-shell (or outside D): every walk stops with zero steps
        // in the cell of the start point's projection.
        if constexpr (PTS) {  // claim every walk of the point not yet claimed (idempotent: no wrap)
            if (tid == 0) sh.item_hi = atomicMax(pcur, I.n_walks);
            __syncthreads();
            const uint32_t r = sh.item_hi;
            k0 = r < I.n_walks ? r : I.n_walks;
            cnt = I.n_walks - k0;
        }
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
        int hint = -1;       // meshes: the walk's last nearest triangle
        R rnext = R(-1);     // meshes, mapped-exact radius: the radius at the walk's position (-1: unknown)
        R x[DIM];
        R d = kFree;
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[a] = x0[a];
        // The item's walks are dealt to the waves round-robin (walk offset wv + nw i for the wave's
        // i-th walk); within a wave, free lanes take the wave's next walks in lane order.
        const uint32_t nw = static_cast<uint32_t>(nthr / kWave);
        const uint32_t wave_cnt = cnt > static_cast<uint32_t>(wv) ? (cnt - wv + nw - 1) / nw : 0u;
        uint32_t wave_next = 0;  // wave-uniform
        // point mode: the wave's current reservation [res_next, res_end) of the point's walks
        uint32_t res_next = 0, res_end = 0;
        bool exhausted = false;
        uint32_t qn = 0;  // wave-uniform queue length
        uint32_t n_fp64 = 0;
        unsigned long long wave_iters = 0;
        LaneStats ls;

        // One outer iteration per Philox block: refill, draw the block, then SPB unrolled steps.
        for (;;) {
            const uint64_t need = __ballot(d == kFree);
            if constexpr (PTS) {
                if (need != 0ull && res_next >= res_end && !exhausted) {
                    uint32_t r = 0;
                    if (lane == 0) r = atomicAdd(pcur, I.chunk);
                    r = __builtin_amdgcn_readfirstlane(r);
                    if (r >= I.n_walks) {
                        exhausted = true;
                    } else {
                        res_next = r;
                        res_end = I.n_walks - r > I.chunk ? r + I.chunk : I.n_walks;
                    }
                }
                if (need != 0ull && res_next < res_end) {
                    const uint32_t mine = res_next + prefix_count(need);
                    const uint32_t np = static_cast<uint32_t>(__popcll(need));
                    res_next = res_end - res_next > np ? res_next + np : res_end;
                    if (d == kFree && mine < res_end) {
                        koff = mine;
                        s = 0;
                        hint = -1;
                        rnext = R(-1);
                        d = d0;
#pragma unroll
                        for (int a = 0; a < DIM; ++a) x[a] = x0[a];
                    }
                }
            } else if (need != 0ull && wave_next < wave_cnt) {
                const uint32_t mine = wave_next + prefix_count(need);
                wave_next += static_cast<uint32_t>(__popcll(need));
                if (d == kFree && mine < wave_cnt) {
                    koff = k0 + static_cast<uint32_t>(wv) + nw * mine;
                    s = 0;
                    hint = -1;
                    rnext = R(-1);
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
                if (d != kFree) walk_step<R, DIM, KIND, PH, CAP, RV>(I, segs, w, F, x, d, s, n_fp64, hint, rnext);
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

// Item (instance, point, first walk, walk count) of global work item `item` of instance I.
__device__ __forceinline__ void decode_item(const DevInst &I, uint64_t item, uint32_t &point, uint32_t &k0,
                                            uint32_t &cnt)
{
    const uint64_t local = item - I.item_begin;
    const uint64_t n_big_items = static_cast<uint64_t>(I.n_obs) * I.n_big;
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
}

// Wave-item mode: each wave owns its items and runs them as one stream.  When the wave has dealt
// every walk of its current item it fetches the next item of the same instance into its other
// slot and keeps refilling free lanes from it, so the walks of consecutive items overlap and the
// lanes do not drain at item boundaries.  Each slot has its own histogram row in the wave's part
// of LDS (rows[0], rows[hist_words]); a row is added to HBM as soon as every walk of its item has
// been binned, which frees the slot for the item after next.  No step of this needs another wave.
// The bookkeeping needed only when an item ends lives in the wave's LDS control block (registers
// are the kernel's limit); what a refill needs stays in scalar registers.  Returns the first item
// it fetched but could not take (another instance, or past the end).
// A wave-uniform value computed on the vector unit, made a scalar-register value explicitly.
__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ double uniform(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

struct WaveCtl {
    uint64_t next_item;  // fetched, not yet taken (valid when have_next)
    uint32_t rem[2];     // walks of the slot's item not yet binned
    uint32_t have_next, pad;
};
constexpr size_t kWaveCtlBytes = 32;

template <typename R, int DIM, int KIND, int RV = -1>
__device__ __forceinline__ uint64_t run_chain(const DevInst &I, uint64_t item, uint32_t *cursor, uint64_t total_items,
                              uint32_t *rows, int hist_words, PolySeg *lds_segs, uint8_t *qb, LaneStats &ls,
                              uint32_t &n_fp64, unsigned long long &wave_iters)
{
    constexpr int SPB = Spb<R, DIM>::v;
    const uint32_t lane = __lane_id();
    const int M = I.n_elem;
    const PolySeg *segs = I.segs;
    if constexpr (KIND == kPolygon || KIND == kPerforated || KIND == kPerfBox) {  // edges / holes read every step
        for (int e = lane; e < I.n_segs; e += kWave) lds_segs[e] = I.segs[e];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        segs = lds_segs;
    }
    StopQueue<R, DIM> q;
    q.pos = reinterpret_cast<R *>(qb);
    q.koff = reinterpret_cast<uint32_t *>(qb + kWave * DIM * sizeof(R));
    q.steps = q.koff + kWave;
    q.slot = q.steps + kWave;
    WaveCtl *wc = reinterpret_cast<WaveCtl *>(q.slot + kWave);
    Fold32 F{};
    if constexpr (sizeof(R) == 4 && DIM == 2) {
        F = Fold32{I.fold_off[0], I.fold_off[1], I.fold_rs[0], I.fold_rs[1], I.fold_rn[0], I.fold_rn[1]};
        asm volatile("" : "+v"(F.off0), "+v"(F.off1), "+v"(F.rs0), "+v"(F.rs1), "+v"(F.rn0), "+v"(F.rn1));
    }
    constexpr R kFree = static_cast<R>(__builtin_inf());

    // wave-uniform state: the points of both slots (random-number counters, binning), the item
    // being dealt (slot, first walk, count, walks dealt, start point and its distance), the stop
    // queue's fill, and whether the chain has ended
    uint32_t pt0 = 0, pt1 = 0, cur = 0, k0c = 0, cntc = 0, dealt = 0, qn = 0, qn1 = 0;
    R x0c[DIM], d0c = kFree;
#pragma unroll
    for (int a = 0; a < DIM; ++a) x0c[a] = static_cast<R>(0);
    bool ended = false;
    if (lane == 0) {
        wc->next_item = item;
        wc->have_next = 1u;
        wc->rem[0] = 0u;
        wc->rem[1] = 0u;
    }
    auto rd = [](uint32_t v) { return __builtin_amdgcn_readfirstlane(v); };

    auto flush_row = [&](uint32_t sl) {
        uint32_t *row = rows + (sl ? hist_words : 0);
        uint32_t *out = I.counts + static_cast<size_t>(sl ? pt1 : pt0) * M;
        for (int j = lane; j < M; j += kWave) {
            const uint32_t v = row[j];
            if (v) {
                atomicAdd(&out[j], v);
                row[j] = 0u;
            }
        }
    };
    auto flushq = [&]() {
        flush_queue<R, DIM, KIND, true>(I, q, qn, pt0, rows, segs, ls, pt1, hist_words);
        const uint32_t n0 = qn - qn1;
        const uint32_t r0 = rd(wc->rem[0]) - n0, r1 = rd(wc->rem[1]) - qn1;
        if (lane == 0) {
            wc->rem[0] = r0;
            wc->rem[1] = r1;
        }
        if (n0 && r0 == 0u) flush_row(0);
        if (qn1 && r1 == 0u) flush_row(1);
        qn = 0;
        qn1 = 0;
    };
    // Takes items into slot `sl` until one has walks to run (true) or the chain ends (false).  Items
    // whose start point lies in the eps-shell (or outside D) are binned at once with zero steps.
    auto take = [&](uint32_t sl) -> bool {
        for (;;) {
            uint64_t it = rd(static_cast<uint32_t>(wc->next_item));
            if (!rd(wc->have_next)) {
                uint32_t t = 0;
                if (lane == 0) t = atomicAdd(cursor, 1u);
                it = rd(t);
            }
            if (it >= total_items || it < I.item_begin || it >= I.item_begin + I.n_items) {
                if (lane == 0) {
                    wc->next_item = it;
                    wc->have_next = 1u;
                }
                return false;
            }
            uint32_t point, k0, cnt;
            decode_item(I, it, point, k0, cnt);
            if (lane == 0) wc->have_next = 0u;
            double x0d[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) x0d[a] = I.x_obs[static_cast<size_t>(point) * DIM + a];
            const double d0d = start_dist64<KIND, DIM>(I, x0d, segs);  // the whole wave, converged
            if (!(d0d > I.eps)) {
                const int j0 = element64<KIND, DIM>(I, x0d, segs);
                if (lane == 0) {
                    atomicAdd(&I.counts[static_cast<size_t>(point) * M + j0], cnt);
                    ls.walks += cnt;
                    if (d0d < 0.0) ls.esc += cnt;
                }
                if (I.trace) {
                    for (uint32_t w = lane; w < cnt; w += kWave) {
                        const size_t t = (static_cast<size_t>(point) * I.n_walks + k0 + w) * 2;
                        I.trace[t] = j0;
                        I.trace[t + 1] = 0;
                    }
                }
                continue;
            }
            if (sl) pt1 = point; else pt0 = point;
            if (lane == 0) wc->rem[sl] = cnt;
            cur = sl;
            k0c = k0;
            cntc = cnt;
            dealt = 0u;
#pragma unroll
            for (int a = 0; a < DIM; ++a) x0c[a] = uniform(static_cast<R>(x0d[a] - origin<R, KIND>(I, a)));
            if constexpr (sizeof(R) == 8) d0c = uniform(d0d); else d0c = uniform(dist32<KIND, DIM>(I, x0c, segs));
            return true;
        }
    };

    uint32_t koff = 0, s = 0, sl = 0;
    int hint = -1;       // meshes: the walk's last nearest triangle
    R rnext = R(-1);     // meshes, mapped-exact radius: the radius at the walk's position (-1: unknown)
    R x[DIM];
    R d = kFree;
#pragma unroll
    for (int a = 0; a < DIM; ++a) x[a] = static_cast<R>(0);
    if (!take(0)) ended = true;
    // deals the current item's next walks to the lanes in `need` (free lanes) in lane order
    auto deal = [&](uint64_t need) {
        const uint32_t mine = dealt + prefix_count(need);
        const uint32_t np = static_cast<uint32_t>(__popcll(need));
        dealt = cntc - dealt > np ? dealt + np : cntc;
        if (d == kFree && mine < cntc) {
            koff = k0c + mine;
            sl = cur;
            s = 0;
            hint = -1;
            rnext = R(-1);
            d = d0c;
#pragma unroll
            for (int a = 0; a < DIM; ++a) x[a] = x0c[a];
        }
    };

    for (;;) {
        const uint64_t need = __ballot(d == kFree);
        if (need != 0ull && dealt >= cntc && !ended) {
            // the current item is fully dealt: move on to the other slot once its item is binned
            const uint32_t other = cur ^ 1u;
            if (rd(wc->rem[other]) != 0u && qn != 0u) flushq();
            if (rd(wc->rem[other]) == 0u && !take(other)) ended = true;
        }
        // one refill site: lanes left free when an item runs out take the next item's walks one
        // Philox block later
        if (need != 0ull && dealt < cntc) deal(need);
        if (!__any(d != kFree)) break;
        uint32_t w[4];
        {
            uint32_t c0 = s / SPB, c1 = I.walk_begin + koff, c2 = sl ? pt1 : pt0, c3 = I.inst;
            // the round keys are formed in the loop on the scalar unit rather than held in 20 SGPRs
            uint32_t k0 = I.key0, k1 = I.key1;
            asm volatile("" : "+s"(k0), "+s"(k1));
            philox4x32_10(c0, c1, c2, c3, k0, k1);
            w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
        }
        wave_iters += SPB;
        constexpr uint32_t kNoStop = 0xFFu;
        uint32_t fph = kNoStop;
        auto phase = [&](auto ph_tag, auto cap_tag) {
            constexpr int PH = decltype(ph_tag)::value;
            constexpr bool CAP = decltype(cap_tag)::value;
            if (d != kFree) walk_step<R, DIM, KIND, PH, CAP, RV>(I, segs, w, F, x, d, s, n_fp64, hint, rnext);
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
                if (qn + nf > static_cast<uint32_t>(kWave)) flushq();
                if (stopped) {
                    const uint32_t slot = qn + prefix_count(fmask);
#pragma unroll
                    for (int a = 0; a < DIM; ++a) q.pos[a * kWave + slot] = x[a];
                    q.koff[slot] = koff;
                    q.steps[slot] = (sizeof(R) == 8 || CAP) ? s : s + fph + 1;
                    q.slot[slot] = sl;
                }
                qn += nf;
                qn1 += static_cast<uint32_t>(__popcll(fmask & __ballot(sl != 0u)));
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
        if constexpr (sizeof(R) == 4) {
            if (__any(d != kFree && s + SPB >= I.max_steps)) {
                block(std::true_type{});
            } else {
                block(std::false_type{});
                s += SPB;
            }
        } else {
            block(std::true_type{});
        }
    }
    if (qn) flushq();
    // every walk is binned by now; add whatever a row still holds (nothing, when the counts above
    // are exact) so that no count can be lost
    flush_row(0);
    flush_row(1);
    return rd(wc->have_next) ? static_cast<uint64_t>(rd(static_cast<uint32_t>(wc->next_item))) : total_items;
}

// Adds a wave's statistics for instance I (sums over its lanes, one atomic per counter).
__device__ __forceinline__ void wave_stats_flush(const DevInst &I, LaneStats &ls, uint32_t &n_fp64,
                                                 unsigned long long &wave_iters)
{
    unsigned long long v[7] = {ls.walks, ls.steps, ls.max_s, ls.cap, ls.esc, n_fp64, 0ull};
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const unsigned long long t = __shfl_xor(v[c], o);
            v[c] = c == 2 ? (t > v[c] ? t : v[c]) : v[c] + t;
        }
    }
    v[6] = wave_iters * kWave;
    if (I.stats && __lane_id() == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            if (c == 2) {
                if (v[c]) atomicMax(&I.stats[2], v[c]);
            } else if (v[c]) {
                atomicAdd(&I.stats[c], v[c]);
            }
        }
    }
    ls = LaneStats{};
    n_fp64 = 0;
    wave_iters = 0;
}

__device__ __forceinline__ int instance_of(const DevInst *insts, int n_inst, uint64_t item)
{
    int lo = 0, hi = n_inst - 1;  // descriptors sorted by item_begin
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (insts[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Instance of global point / item index q for one lane (descriptors sorted by item_begin).
__device__ __forceinline__ int instance_of_lane(const DevInst *insts, int n_inst, uint64_t q)
{
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (insts[mid].item_begin <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Point mode, once every point has been handed out: the block looks for a point whose walks are
// not all reserved yet, scanning all points from a block-dependent start, blockDim points per
// round.  Returns total_points when there is none.
__device__ uint32_t steal_point(const DevInst *insts, int n_inst, uint32_t total_points, const uint32_t *pcur,
                                BlockShared &sh)
{
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    const uint32_t start = static_cast<uint32_t>((blockIdx.x * 2654435761ull) % total_points);
    if (threadIdx.x == 0) sh.pad0 = kNone;
    __syncthreads();
    for (uint32_t base = 0; base < total_points; base += blockDim.x) {
        const uint32_t k = base + threadIdx.x;
        if (k < total_points) {
            const uint32_t q = static_cast<uint32_t>((static_cast<uint64_t>(start) + k) % total_points);
            const uint32_t n = insts[instance_of_lane(insts, n_inst, q)].n_walks;
            if (__hip_atomic_load(&pcur[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n) atomicMin(&sh.pad0, k);
        }
        __syncthreads();
        const bool found = sh.pad0 != kNone;
        __syncthreads();
        if (found) break;
    }
    const uint32_t k = sh.pad0;
    return k == kNone ? total_points : static_cast<uint32_t>((static_cast<uint64_t>(start) + k) % total_points);
}

// MODE 0: block-item mode (run_item over items).  1: wave-item mode (run_chain); LDS holds, per
// wave, two histogram rows, the staged segments and the stop queue.  2: point mode (run_item over
// points with walk reservations; cursor[2 + p] is point p's walk cursor).
// KSEL: -1 for launches that mix kinds (kind and radius mode read per instance), else the kind plus
// kRadiusVariant when the launch uses the mapped-bound radius (the mapped-exact one for polygons),
// both then fixed at compile time.
template <typename R, int DIM, int KSEL, int MODE>
__global__ __launch_bounds__(1024) void walk_kernel(const DevInst *__restrict__ insts, int n_inst,
                                                    uint64_t total_items, uint32_t *cursor,
                                                    int hist_words, int seg_bytes)
{
    constexpr int KK = KSEL >= 0 ? KSEL % kRadiusVariant : -1;
    constexpr int RV = KSEL >= 0 ? KSEL / kRadiusVariant : -1;
    extern __shared__ __align__(16) uint8_t smem[];
    if constexpr (MODE == 1) {
        const int wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
        const uint32_t lane = __lane_id();
        const size_t row_bytes = static_cast<size_t>(2 * hist_words) * 4;
        uint32_t *rows = reinterpret_cast<uint32_t *>(smem + static_cast<size_t>(wv) * row_bytes);
        PolySeg *segs_w = reinterpret_cast<PolySeg *>(smem + nw * row_bytes + static_cast<size_t>(wv) * seg_bytes);
        uint8_t *qb = smem + nw * (row_bytes + seg_bytes) +
                      static_cast<size_t>(wv) * (kWave * (DIM * sizeof(R) + 12) + kWaveCtlBytes);
        for (int j = lane; j < 2 * hist_words; j += kWave) rows[j] = 0u;
        LaneStats ls;
        uint32_t n_fp64 = 0;
        unsigned long long wave_iters = 0;
        uint32_t it0 = 0;
        if (lane == 0) it0 = atomicAdd(cursor, 1u);
        uint64_t item = __builtin_amdgcn_readfirstlane(it0);
        while (item < total_items) {
            const DevInst &I = insts[instance_of(insts, n_inst, item)];
            const int kind = KSEL >= 0 ? KK : I.kind;
            const uint64_t first = item;
            if constexpr (KSEL >= 0) {
                item = run_chain<R, DIM, KK, RV>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters);
            } else if constexpr (DIM == 2) {
                switch (kind) {
                case kDisk: item = run_chain<R, 2, kDisk>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kAnnulus: item = run_chain<R, 2, kAnnulus>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kEllipse: item = run_chain<R, 2, kEllipse>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kPolygon: item = run_chain<R, 2, kPolygon>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kPerforated: item = run_chain<R, 2, kPerforated>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kPerfBox: item = run_chain<R, 2, kPerfBox>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                default: item = run_chain<R, 2, kBox>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                }
            } else {
                switch (kind) {
                case kBall: item = run_chain<R, 3, kBall>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kPerforated: item = run_chain<R, 3, kPerforated>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                case kPerfBox: item = run_chain<R, 3, kPerfBox>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                default: item = run_chain<R, 3, kBox>(I, first, cursor, total_items, rows, hist_words, segs_w, qb, ls, n_fp64, wave_iters); break;
                }
            }
            wave_stats_flush(I, ls, n_fp64, wave_iters);
        }
        return;
    }
    __shared__ BlockShared sh;
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem);
    PolySeg *lds_segs = reinterpret_cast<PolySeg *>(smem + static_cast<size_t>(hist_words) * 4);
    uint8_t *qbase = smem + static_cast<size_t>(hist_words) * 4 + seg_bytes;

    if constexpr (MODE == 2) {
        const uint32_t total_points = static_cast<uint32_t>(total_items);
        if (total_points == 0u) return;
        uint32_t *pcur = cursor + 2;
        for (;;) {
            if (threadIdx.x == 0) sh.item_lo = atomicAdd(cursor, 1u);
            __syncthreads();
            uint32_t p = __builtin_amdgcn_readfirstlane(sh.item_lo);
            __syncthreads();
            if (p >= total_points) {
                p = __builtin_amdgcn_readfirstlane(steal_point(insts, n_inst, total_points, pcur, sh));
                if (p >= total_points) return;
            }
            const int idx = instance_of(insts, n_inst, p);
            const DevInst &I = insts[idx];
            const uint32_t point = p - static_cast<uint32_t>(I.item_begin);
            if constexpr (KSEL >= 0) {
                run_item<R, DIM, KK, true, RV>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p);
            } else if constexpr (DIM == 2) {
                switch (I.kind) {
                case kDisk: run_item<R, 2, kDisk, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kAnnulus: run_item<R, 2, kAnnulus, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kEllipse: run_item<R, 2, kEllipse, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kPolygon: run_item<R, 2, kPolygon, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kPerforated: run_item<R, 2, kPerforated, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kPerfBox: run_item<R, 2, kPerfBox, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                default: run_item<R, 2, kBox, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                }
            } else {
                switch (I.kind) {
                case kBall: run_item<R, 3, kBall, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kPerforated: run_item<R, 3, kPerforated, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                case kPerfBox: run_item<R, 3, kPerfBox, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                default: run_item<R, 3, kBox, true>(I, point, 0, 0, hist, lds_segs, qbase, sh, pcur + p); break;
                }
            }
        }
    }
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
            run_item<R, DIM, KK, false, RV>(I, point, k0, cnt, hist, lds_segs, qbase, sh);
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

__global__ void reset_cursor_kernel(uint32_t *cursor, size_t n)
{
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        cursor[i] = 0u;
}

}  // namespace

size_t walk_lds_bytes(int precision, int dim, int block, int hist_words, int seg_bytes, int mode)
{
    const size_t rs = precision == 0 ? 8 : 4;
    const size_t nw = static_cast<size_t>(block / kWave);
    if (mode == 1) return nw * (static_cast<size_t>(2 * hist_words) * 4 + seg_bytes + kWave * (dim * rs + 12) + kWaveCtlBytes);
    return static_cast<size_t>(hist_words) * 4 + seg_bytes + nw * kWave * (dim * rs + 8);
}

template <typename R, int DIM, int KSEL> static const void *kptr(int mode)
{
    return mode == 1   ? reinterpret_cast<const void *>(&walk_kernel<R, DIM, KSEL, 1>)
           : mode == 2 ? reinterpret_cast<const void *>(&walk_kernel<R, DIM, KSEL, 2>)
                       : reinterpret_cast<const void *>(&walk_kernel<R, DIM, KSEL, 0>);
}

template <typename R> static const void *kernel_of(int dim, int ksel, int wave)
{
    if (dim == 2) {
        switch (ksel) {
        case kDisk: return kptr<R, 2, kDisk>(wave);
        case kAnnulus: return kptr<R, 2, kAnnulus>(wave);
        case kRadiusVariant + kDisk: return kptr<R, 2, kRadiusVariant + kDisk>(wave);
        case kRadiusVariant + kAnnulus: return kptr<R, 2, kRadiusVariant + kAnnulus>(wave);
        case kEllipse: return kptr<R, 2, kEllipse>(wave);
        case kRadiusVariant + kEllipse: return kptr<R, 2, kRadiusVariant + kEllipse>(wave);
        case kPolygon: return kptr<R, 2, kPolygon>(wave);
        case kRadiusVariant + kPolygon: return kptr<R, 2, kRadiusVariant + kPolygon>(wave);
        case kPerforated: return kptr<R, 2, kPerforated>(wave);
        case kRadiusVariant + kPerforated: return kptr<R, 2, kRadiusVariant + kPerforated>(wave);
        case kPerfBox: return kptr<R, 2, kPerfBox>(wave);
        case kRadiusVariant + kPerfBox: return kptr<R, 2, kRadiusVariant + kPerfBox>(wave);
        case kBox: return kptr<R, 2, kBox>(wave);
        default: return kptr<R, 2, -1>(wave);
        }
    }
    switch (ksel) {
    case kBall: return kptr<R, 3, kBall>(wave);
    case kRadiusVariant + kBall: return kptr<R, 3, kRadiusVariant + kBall>(wave);
    case kPerforated: return kptr<R, 3, kPerforated>(wave);
    case kRadiusVariant + kPerforated: return kptr<R, 3, kRadiusVariant + kPerforated>(wave);
    case kPerfBox: return kptr<R, 3, kPerfBox>(wave);
    case kRadiusVariant + kPerfBox: return kptr<R, 3, kRadiusVariant + kPerfBox>(wave);
    case kBox: return kptr<R, 3, kBox>(wave);
    case kTriMesh: return kptr<R, 3, kTriMesh>(wave);  // meshes always launch on their own
    default: return kptr<R, 3, -1>(wave);
    }
}

const void *walk_kernel_ptr(int precision, int dim, int kind_sel, int mode)
{
    return precision == 0 ? kernel_of<double>(dim, kind_sel, mode) : kernel_of<float>(dim, kind_sel, mode);
}

size_t walk_cursor_words(int mode, uint64_t total_items)
{
    return mode == 2 ? 2 + static_cast<size_t>(total_items) : 2;
}

hipError_t launch_walks(int precision, int dim, int kind_sel, int mode, const DevInst *insts, int n_inst,
                        uint64_t total_items, uint32_t *cursor, int hist_words, int seg_bytes, int block, int grid,
                        hipStream_t stream)
{
    const size_t nc = walk_cursor_words(mode, total_items);
    reset_cursor_kernel<<<static_cast<int>(std::min<size_t>((nc + 255) / 256, 1024)), 256, 0, stream>>>(cursor, nc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = walk_lds_bytes(precision, dim, block, hist_words, seg_bytes, mode);
    const void *fn = walk_kernel_ptr(precision, dim, kind_sel, mode);
    void *args[] = {&insts, &n_inst, &total_items, &cursor, &hist_words, &seg_bytes};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
}

}  // namespace wos
