// kernels.hpp -- the hot path of the level-line splitter on gfx950.
//
// A call splits a list of types, each a polynomial P = q_{l,n} (l = 0: p_n)
// of degree D = 2^(N-1), N = l + n, in the closed upper half plane (Section
// 6.1).  All types share one launch per stage; a device table of type_desc
// maps global item indices (seeds, segments, starts) to their type.  Types
// are laid out by decreasing order N so that the persistent queues end on
// the cheap items.
//
//   k_seeds     seed lift      seed j of type t at Phi-angle pi j / S, lifted
//                              from the circle |p_1| = lambda_0 through p_2
//                              .. p_N (Section 4.2, lifting p_k -> p_{k+1})
//   k_walk      level line     a lane walks the F fine points of one segment,
//                              value phase 2 pi s / M (Prop. computeLevelLine);
//                              every (M/4)-th point is a start (Thm
//                              practicalFTA: values lambda_0 {1, i, -1, -i})
//   k_descend   Newton descent one lane per start, capped (Algorithm S_par)
//   k_prekeys .. k_scatter     nset collection (Section 6.1)
//   k_classify                 exact period (eq. def:hyp) / type (eq. def:mis)
//
// Work distribution: k_walk and k_descend are persistent; each wave takes
// chunks of items from a global counter and hands them to its lanes as they
// free up, so lanes whose Newton iterations end early do not wait for the
// slowest lane of their wave (the divergence the paper names as its
// objection to GPUs).
#pragma once
#include "common.hpp"
#include "dd.hpp"

namespace msplit {

// status of a descent
// ST_DD: converged in double-double (the low parts are in roots_lo);
// ST_STALL: the FP64 descent met its step test without the quadratic
// convergence of a simple root (redone in double-double)
enum : uint8_t { ST_NONE = 0, ST_CONVERGED = 1, ST_DIVERGED = 2, ST_TIMEOUT = 3, ST_DD = 4, ST_STALL = 5 };
__device__ __forceinline__ bool st_converged(uint8_t s) { return s == ST_CONVERGED || s == ST_DD; }

// global counters
// G_HARD_CLS / G_HARD_CERT: lengths of the lists of hard cases of the
// classification and of the certificate (handled by kernels of their own)
// G_DD_NEXT: work queue of the double-double descents
// G_FAILED_SEGS: length of the list of walk segments that failed their phase check
enum { G_SEG_NEXT = 0, G_START_NEXT, G_FAILED_SEGS, G_START_NEXT2, G_DD_COUNT, G_HARD_CLS, G_HARD_CERT, G_DD_NEXT,
       G_NCOUNTERS = 8 };
// per-type counters (uint64 slots, C_NCOUNTERS per type)
enum {
    C_CONVERGED = 0, C_DIVERGED, C_TIMEOUT, C_PHASE_FAIL, C_SEED_FAIL, C_STEPS_LIFT, C_STEPS_WALK,
    C_STEPS_DESC, C_STEPS_FP32, C_UNIQUE, C_REAL, C_CERTIFIED, C_LABEL, C_OVERLAP, C_MIN_SEP_BITS,
    C_MAX_RAD_BITS, C_SURVIVORS, C_KEPT, C_DD_ROUTED, C_STEPS_DD, C_BASIN, C_MIN_BASIN_BITS, C_MARK_CAPPED,
    C_NCOUNTERS = 23
};

// types of one call (batch_args.T)
constexpr int MAX_TYPES = 256;

struct plan_t {
    int l, n, N;          // type and order N = l + n
    int el, eN;           // the polynomial P evaluated (eval_q_t): q_{l,n} and p_n are (l, N); the
                          // simplified s_{l,n} = p_{N-1} + p_{l-1} is (-(l-1), N-1)
    int M;                // fine points per turn
    int q;                // M / 4: fine points between starts
    int cap;              // Newton cap
    int64_t D;            // degree 2^(N-1)
    int64_t F;            // fine points per segment
    int64_t S;            // segments in the upper half plane (the seed angle is pi j / S)
    int64_t seg0, nseg;   // the segments [seg0, seg0 + nseg) of this item: the whole upper half
                          // (0, S), or one chunk of it when the level line is streamed
    int64_t NS;           // starts of this item: nseg F / q, + 1 with the left end (2 D + 1 in all)
    double level;         // lambda_0
    double tau;           // nset identification radius
    double tol_desc;      // relative step of a converged descent
    double x_tip;         // |c + 2| below which descents are redone in double-double (0: none)
    double tau_dd;        // identification radius between double-double roots
    int tip_starts;       // last starts of the type re-solved in double-double (left tip)
    uint32_t divmask_lo;  // bit k set when k | n, k < n (k < 32)
    int precision;
    float fp32_switch;
};

struct type_desc {
    plan_t p;
    int64_t seed_off, seg_off, start_off; // global offsets of this type's items
    int64_t out_off;                      // first output slot
    uint64_t cap;                         // output capacity
    int64_t uniq_off;                     // offset in the compact unique index space
    int64_t tip_lo_off;                   // first slot of this type in the tip-start low parts
};

struct batch_args {
    const type_desc *types;
    const int64_t *seed_offs, *seg_offs, *start_offs; // T + 1 entries each
    int64_t *uniq_offs;       // output index space: min(kept, capacity) roots per type, set on the device
    int64_t *coll_offs;       // collected (identified) roots per type, set on the device
    int64_t *kept_offs;       // roots kept by the classification per type, set on the device
    int64_t *surv_offs;       // sorted candidates per type, set on the device
    const double *cis;        // cos, then sin, of 2 pi s / M, s < 64 (k_cis)
    double dphi;              // 2 pi / M (a kernel argument: wave-uniform, no VGPR)
    double x_tip_max;         // the largest tip radius of the call's types (0: none)
    int T;
    int64_t n_seeds, n_segs, n_starts;
    uint32_t chunk_seg, chunk_start;
    // the starts of the types an FP32 pass runs on (MIXED), as one index
    // space: type t holds [fp32_offs[t], fp32_offs[t + 1]), empty for the
    // others; n_fp32 = fp32_offs[T]
    const int64_t *fp32_offs;
    int64_t n_fp32;
    uint32_t chunk_fp32;
    unsigned long long *gctr;   // global counters
    unsigned long long *ctr;    // T x C_NCOUNTERS, folded from spread
    unsigned long long *spread; // CTR_SPREAD copies of T x C_NCOUNTERS
};

// Waves add their per-type counts into one of CTR_SPREAD copies of the
// counter table (chosen by wave index) and a fold kernel combines the copies.
// With one table every wave of the grid flushes into the same few addresses
// at the same moment (when the work queue crosses from one type to the next,
// and at the end): those atomics serialise and stall every wave on its next
// memory wait.
constexpr int CTR_SPREAD = 64;

__device__ __forceinline__ unsigned long long *wave_ctr(const batch_args &b)
{
    const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    return b.spread + (size_t)(w & (CTR_SPREAD - 1)) * (size_t)b.T * C_NCOUNTERS;
}

// cis(2 pi s / M) for s = 0..63 (s taken mod M), M <= 64, exact at the
// quarter turns; one thread per entry
__global__ void k_cis(int M, double *cis)
{
    const int s = threadIdx.x;
    if (s >= 64) return;
    const int r = s % M;
    double sn, cs;
    sincospi(2.0 * (double)r / (double)M, &sn, &cs);
    if (4 * r == 0) { cs = 1.0; sn = 0.0; }
    if (4 * r == M) { cs = 0.0; sn = 1.0; }
    if (4 * r == 2 * M) { cs = -1.0; sn = 0.0; }
    if (4 * r == 3 * M) { cs = 0.0; sn = -1.0; }
    cis[s] = cs;
    cis[64 + s] = sn;
}

// index of the type owning global item g: offs is non-decreasing, T + 1
// entries, offs[0] = 0 <= g < offs[T]
__device__ __forceinline__ int find_type(const int64_t *offs, int T, int64_t g)
{
    int lo = 0, hi = T; // invariant: offs[lo] <= g < offs[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offs[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Per-type counter accumulation: lanes add to a register while they stay on
// the same type and flush (wave-reduced when the whole wave agrees on the
// type) when it changes and at the end.
struct type_count {
    int t = -1;
    unsigned long long v = 0;
};

__device__ __forceinline__ void flush_count(unsigned long long *ctr, int slot, type_count &c)
{
    // all lanes of the wave call this together
    wave_reduce_by_key<RED_ADD>(ctr, C_NCOUNTERS, slot, c.v ? c.t : -1, c.v);
    c.v = 0;
}

// Type of global item g with a per-lane cache of the current type's item
// range [lo, hi): the binary search runs only when g leaves it.
struct type_cache {
    int t = -1;
    int64_t lo = 0, hi = 0;
};

__device__ __forceinline__ int cached_type(type_cache &c, const int64_t *offs, int T, int64_t g)
{
    if (c.t < 0 || g < c.lo || g >= c.hi) {
        c.t = find_type(offs, T, g);
        c.lo = offs[c.t];
        c.hi = offs[c.t + 1];
    }
    return c.t;
}

// ------------------------------------------------------------ seed lift
// Seed j of a type lies at Phi-angle pi j / S.  On p_1 = z the level line is
// the circle |z| = lambda_0, so it starts at lambda_0 e^{i pi j / S}.  At p_k
// its value must be lambda_0 e^{i pi a_k / S} with a_k = 2^(k-1) j mod 2S (the
// value phase doubles from p_k to p_{k+1}: p_{k+1} = p_k^2 + c with |c| small
// against lambda_0^2).  Each level is solved with the Newton method on log P,
// whose step z += log(T/P) P/P' is the discrete level-line / iso-angle flow
// of Section 4.1.  For q_{l,n} a last stage moves the p_{l+n} point onto
// q_{l,n} = lambda_0 e^{i pi a_N / S} (same phase: |p_l| << lambda_0 there).
// Grid-stride loop: per-type counts stay in registers and are flushed when a
// lane's type changes and at the end (a few atomics per wave in all).
// Every writer of a start also writes the descent's first Newton iterate
// from it, first[k] = z - P(z)/P'(z): the seeds and the walk have just
// evaluated P and P' there (the lifts evaluate once more), and the value is
// bitwise the descent's own first step (same evaluation, same division), so
// the descent starts one step in.
__global__ void k_seeds(batch_args b, cd *seeds, cd *starts, cd *first)
{
    unsigned long long *const wc = wave_ctr(b);
    type_count steps, fail;
    type_cache tc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < b.n_seeds; g0 += stride) {
        const int64_t g = g0 + threadIdx.x;
        const int t = g < b.n_seeds ? cached_type(tc, b.seed_offs, b.T, g) : steps.t;
        if (__ballot(g < b.n_seeds && t != steps.t)) {
            flush_count(wc, C_STEPS_LIFT, steps);
            flush_count(wc, C_SEED_FAIL, fail);
        }
        steps.t = fail.t = t;
        if (g >= b.n_seeds) continue;
        const plan_t &plr = b.types[t].p;
        // (l, N) of the evaluated polynomial: its leading term p_N is the last lift
        const struct { int l, N; int64_t S, F, q; double level; } pl = {plr.el, plr.eN, plr.S, plr.F, plr.q, plr.level};
        bool failed = false;
        const int64_t jl = g - b.seed_offs[t]; // seed within the item
        const int64_t j = jl + plr.seg0;       // seed on the whole line
        const int64_t twoS = 2 * pl.S;
        double sn, cs;
        sincospi((double)j / (double)pl.S, &sn, &cs);
        cd z = {pl.level * cs, pl.level * sn};
        if (j == pl.S) z = {-pl.level, 0.0};
        if (j == 0) z = {pl.level, 0.0};
        int64_t a = j % twoS;
        const int top = pl.l ? pl.N + 1 : pl.N;
        cd P = {0.0, 0.0}, dP = {1.0, 0.0}; // at z, of the last level (the type's polynomial)
        for (int k = 2; k <= top && !failed; ++k) {
            int ll = 0, NN = k;
            if (k <= pl.N) a = (2 * a) % twoS;
            else { ll = pl.l; NN = pl.N; }
            sincospi((double)a / (double)pl.S, &sn, &cs);
            cd T = {pl.level * cs, pl.level * sn};
            if (a == 0) T = {pl.level, 0.0};
            // intermediate levels only have to land in the basin of the
            // next one (accepted like the walk's intermediate fine points: a
            // seed that lands on another branch fails the phase checks of its
            // segments, whose starts are then lifted again one by one); the
            // last level is solved to rounding level
            const double tolv2 = (k < top) ? 0x1p-4 : 1e-26;
            for (int it = 0;; ++it) {
                eval_q(ll, NN, z, P, dP);
                ++steps.v;
                cd w = cdiv(T, P);
                cd v = {w.re - 1.0, w.im};
                if (cabs2(v) < tolv2) break;
                if (it >= 40 || !cfinite(P)) { failed = true; break; }
                cd h = cmul(clog_near1(w), cdiv(P, dP));
                // near the tip of M the value carries ~4^N u of rounding
                // noise; stop once the update itself is at rounding level
                if (cabs2(h) <= 0x1p-96 * fmax(cabs2(z), 0x1p-16)) break;
                z = cadd(z, h);
                if (j == 0 || j == pl.S) z.im = 0.0; // the two real end points stay real
            }
        }
        fail.v += failed;
        seeds[g] = z;
        // the last seed of a chunk is the next chunk's first start
        if (jl * (pl.F / pl.q) < plr.NS) {
            const int64_t k = b.types[t].start_off + jl * (pl.F / pl.q);
            starts[k] = z;
            first[k] = failed ? z : csub(z, cdiv_fast(P, dP));
        }
    }
    flush_count(wc, C_STEPS_LIFT, steps);
    flush_count(wc, C_SEED_FAIL, fail);
}

// --------------------------------------------------------- level-line walk
// Lane state machine: each loop trip is one evaluation of P, P' followed by
// one update, so lanes never wait for each other inside a segment.  Fine point
// s targets T_s = lambda_0 e^{2 i pi s / M}; the step towards it is Newton on
// log P, z += log(T_s / P) P / P' (an Euler step of the level-line flow
// lambda' = i P / P' of Section 4.1 with its correction).  A fine point that
// becomes a start (every q-th) is accepted once |P / T_s - 1| < 2^-5, the
// others at |T_s / P - 1| < 2^-2, or when the update is at rounding level:
// an intermediate point only has to lie in the Newton basin of the next
// target, and the next target is aimed from the actual value, so no error
// accumulates.  M, q = M / 4 and F are powers of two: the phase index and
// the start test are masks, and the M values e^{2 i pi r / M} sit in LDS.
//
// Each segment is walked by two lanes: forward from its seed (fine points
// 1 .. F/2) and backward from the next seed (F - 1 .. F/2), which halves the
// longest chain of dependent evaluations and doubles the lanes at work.  Both
// end on the middle point; where they disagree by more than a tenth of a
// Newton step, one of them changed turns (a skipped turn lands about
// 2 pi |P/P'| away) and the segment fails its phase check (k_failed_list).
// Work item h: segment h >> 1, backward when h is odd.
// Per-type fields the walk reads, staged in LDS by every block (the lanes
// keep only their item, type, fine point and iterate in registers).
struct walk_type {
    uint32_t seg_lo;   // first global segment of the type
    uint32_t start_lo; // first global start of the type
    uint32_t seg0;     // first segment of the item on the whole line
    uint32_t F;        // fine points per segment (a power of two, >= 2)
    int l, N;          // the evaluated polynomial (eval_q_t)
    double level;      // lambda_0
};

// The middle fine point of a segment from both of its walks, and the squared
// Newton step there (forward walk).
struct walk_mid { cd f, b; double s2; };

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_walk(batch_args b, const cd *seeds, cd *starts, uint8_t *item_flag, walk_mid *mid, cd *first)
{
    constexpr uint32_t NONE = 0xffffffffu;
    // |T/P - 1| < 2^-5 sqrt(0.9) keeps |P/T - 1| = |v| / |1 + v| below 2^-5
    const double tol2_start = 0.9 * 0x1p-10, tol2_mid = 0x1p-4;
    __shared__ double cis_l[128];
    __shared__ walk_type wt[MAX_TYPES + 1];
    for (int i = threadIdx.x; i < 128; i += blockDim.x) cis_l[i] = b.cis[i];
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) {
        walk_type w;
        w.seg_lo = (uint32_t)b.seg_offs[i];
        if (i < b.T) {
            const type_desc &td = b.types[i];
            w.start_lo = (uint32_t)td.start_off;
            w.seg0 = (uint32_t)td.p.seg0;
            w.F = (uint32_t)td.p.F;
            w.l = td.p.el;
            w.N = td.p.eN;
            w.level = td.p.level;
        }
        wt[i] = w;
    }
    __syncthreads();
    unsigned long long *const wc = wave_ctr(b);
    const uint32_t n_items = 2u * (uint32_t)b.n_segs;
    int ct = -1;
    uint32_t cnt[4] = {0u, 0u, 0u, 0u}; // steps
    const int slots[4] = {C_STEPS_WALK, C_STEPS_WALK, C_STEPS_WALK, C_STEPS_WALK};
    uint32_t h = NONE; // current work item
    bool exhausted = false;
    int t = 0;
    // M and q are the same for every type of a call (wave-uniform), powers of two
    const int pl_M = b.types[0].p.M, pl_q = b.types[0].p.q;
    const uint32_t mmask = (uint32_t)pl_M - 1u, qmask = (uint32_t)pl_q - 1u;
    const int qshift = __builtin_ctz((uint32_t)pl_q);
    uint32_t s = 0, r0 = 0; // fine point within the segment (1..F-1); (j F) mod M
    int it = 0;
    cd z = {0.0, 0.0};
    // P/P' at the last accepted fine point (the seed first), for the second-order
    // prediction only: FP32 is enough there and saves two VGPRs
    cf gprev = {0.f, 0.f};
    wave_queue wq = wave_queue_start(b.chunk_seg);
    while (true) {
        const bool need = !exhausted && h == NONE;
        const uint64_t got = wave_take(wq, &b.gctr[G_SEG_NEXT], b.chunk_seg, n_items, need);
        if (need) {
            if (got >= n_items) {
                exhausted = true;
            } else {
                h = (uint32_t)got;
                const uint32_t g = h >> 1;
                if (g < wt[t].seg_lo || g >= wt[t + 1].seg_lo) {
                    int lo = 0, hi = b.T; // wt[lo].seg_lo <= g < wt[hi].seg_lo
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (wt[mid].seg_lo <= g) lo = mid; else hi = mid;
                    }
                    t = lo;
                }
                r0 = ((g - wt[t].seg_lo + wt[t].seg0) * wt[t].F) & mmask;
                // seed j of the type sits at seed_offs[t] + j = g + t (a type of
                // S segments has S + 1 seeds); the backward walk starts on seed
                // j + 1
                const bool back = h & 1u;
                z = seeds[g + (uint32_t)t + (back ? 1u : 0u)];
                s = back ? wt[t].F - 1u : 1u;
                it = 0;
            }
        }
        const bool change = h != NONE && t != ct;
        if (__ballot(change)) {
            wave_add4_by_key(wc, C_NCOUNTERS, ct, slots, cnt);
            cnt[0] = 0u;
            if (change) ct = t;
        }
        if (__ballot(h != NONE || !exhausted) == 0) break;
        if (h == NONE) continue;
        cd P, dP;
        eval_q_wave(wt[t].l, wt[t].N, z, P, dP);
        cnt[0] += 1u;
        const uint32_t g = h >> 1;
        const bool back = h & 1u;
        const uint32_t F = wt[t].F, Fh = F >> 1;
        // at the seed (P = T of the seed's fine point, to rounding) the first
        // update aims from that point: log(T_s / P) = +-i dphi + log(T_seed / P),
        // whose log is near 1 where the series below is accurate
        const bool at_seed = it == 0 && s == (back ? F - 1u : 1u);
        const uint32_t r = (r0 + s + (at_seed ? (back ? 1u : 0xffffffffu) : 0u)) & mmask;
        const double dphi = back ? -b.dphi : b.dphi;
        const double lev = wt[t].level;
        const cd T = {lev * cis_l[r], lev * cis_l[64 + r]};
        const cd w = cdiv_fast(T, P);
        const double a2 = cabs2({w.re - 1.0, w.im});
        const cd step = cdiv_fast(P, dP);
        const uint32_t start0 = wt[t].start_lo + (g - wt[t].seg_lo) * (F >> qshift);
        if (!cfinite(w) || !cfinite(step) || it > 24) {
            // the starts of this half not reached yet get no value (NaN:
            // their descents end as divergent); the middle start is the
            // forward walk's
            const double nan = __longlong_as_double(0x7ff8000000000000ll);
            if (!back) {
                for (uint32_t s2 = (s + qmask) & ~qmask; s2 <= Fh; s2 += (uint32_t)pl_q) {
                    const uint32_t k = start0 + (s2 >> qshift);
                    starts[k] = {nan, nan};
                    first[k] = {nan, nan};
                }
            } else {
                for (uint32_t s2 = s & ~qmask; s2 > Fh; s2 -= (uint32_t)pl_q) {
                    const uint32_t k = start0 + (s2 >> qshift);
                    starts[k] = {nan, nan};
                    first[k] = {nan, nan};
                }
            }
            item_flag[h] = 2;
            h = NONE;
            continue;
        }
        cd u0 = clog_series(w);
        if (at_seed) {
            gprev = {(float)step.re, (float)step.im};
            u0.im += dphi;
        }
        const cd hs = cmul(u0, step);
        const bool is_start = (s & qmask) == 0;
        const bool last = s == Fh;
        if (!at_seed && (a2 < (is_start || last ? tol2_start : tol2_mid) ||
                         cabs2(hs) <= 0x1p-96 * fmax(cabs2(z), 0x1p-16))) {
            if (is_start && !(back && last)) {
                const uint32_t k = start0 + (s >> qshift);
                starts[k] = z;
                first[k] = csub(z, step);
            }
            if (last) {
                // the walks of the segment meet here (phase check in k_failed_list)
                if (back) {
                    mid[g].b = z;
                } else {
                    mid[g].f = z;
                    mid[g].s2 = cabs2(step);
                }
                item_flag[h] = 0;
                h = NONE;
                continue;
            }
            // aim at the next fine point: log(T_{s+-1}/P) = +-i dphi + log(T_s/P)
            s += back ? 0xffffffffu : 1u;
            it = 0;
            u0.im += dphi;
            // second order along the level-line flow (uniform phase steps):
            // the change of P/P' since the last accepted point
            const cd dg = {step.re - (double)gprev.re, step.im - (double)gprev.im};
            z = cadd(z, cmul(u0, cadd(step, {0.5 * dg.re, 0.5 * dg.im})));
            gprev = {(float)step.re, (float)step.im};
        } else {
            ++it;
            z = cadd(z, hs);
        }
    }
    wave_add4_by_key(wc, C_NCOUNTERS, ct, slots, cnt);
}

// ---------------------------------------------------------- Newton descent
// One lane per start, Newton map N_P (eq. Newton), cap max{20, I_N log d}
// (Algorithm S_par).  Discarded as divergent: non-finite, |z| > 8 (far from
// M, which lies in D(0,2) u {-2}), or a long-distance jump (step more than 8
// times the previous one after the third step, Section 6.4.2).  Converged
// when the step falls below tol * max(|z|, 2^-8); one more step is taken
// unless quadratic convergence predicts the next step below the rounding.
// In FP64 the first step from every start was taken where the start was
// written (its P and P' were evaluated there), so the descent begins at the
// first iterate with one step counted.
//
// MIXED precision runs k_descend32 first, over the starts of the types with
// an FP32 pass (fp32_eligible; their own index space, fp32_offs), from the
// first iterates: FP32 Newton steps while the step exceeds
// fp32_switch * max(|z|, 2^-8).  The rounding noise of
// an FP32 Newton step of p_n is about 8 u |z| (the orbit's error grows like
// its derivative), far below that threshold, so FP32 only takes the steps it
// resolves.  A start whose first FP32 step is already below the threshold --
// near the tip of M, where FP32 cannot even tell neighbouring starts apart --
// keeps its FP64 value untouched.  The FP64 pass then continues every start
// not discarded in FP32, counting the FP32 steps against the cap.  Each pass
// is precision-uniform, so no wave runs both code paths.
// Rounding in the orbit is amplified by up to about 2^N, so an FP32
// evaluation of an order-N polynomial has a relative error near 2^(N-24):
// FP32 steps are taken only up to order FP32_MAX_ORDER (error below 2^-4),
// and only for p_n: the roots of q_{l,n} next to -2 are about 8^-N apart
// (against 4^-N for p_n), closer than steps with that error can aim, so an
// FP32 step there can carry a start into the basin of a neighbouring root.
constexpr int FP32_MAX_ORDER = 20;
__host__ __device__ __forceinline__ bool fp32_eligible(int l, int N) { return l == 0 && N <= FP32_MAX_ORDER; }

__global__ void k_descend32(batch_args b, cd *roots, uint8_t *status, uint8_t *iters)
{
    unsigned long long *const wc = wave_ctr(b);
    type_count steps32, ndiv, ntime;
    int64_t g = -1;
    int t = -1;
    int pl_l = 0, pl_N = 1, pl_cap = 20;
    float pl_sw = 0.f;
    cf z = {0.f, 0.f};
    float prev = 0.f; // previous squared step length
    int it = 0;
    bool done = false;
    wave_queue wq = wave_queue_start(b.chunk_fp32);
    type_cache tc;
    int64_t to_start = 0; // start index minus FP32 index within the current type
    while (true) {
        const bool need = !done && g < 0;
        const uint64_t got = wave_take(wq, &b.gctr[G_START_NEXT], b.chunk_fp32, (uint64_t)b.n_fp32, need);
        bool change = false;
        if (need) {
            if (got >= (uint64_t)b.n_fp32) {
                done = true;
            } else {
                const int t1 = cached_type(tc, b.fp32_offs, b.T, (int64_t)got);
                if (t1 != t) {
                    t = t1;
                    const plan_t &pl = b.types[t].p;
                    pl_l = pl.el;
                    pl_N = pl.eN;
                    pl_cap = pl.cap;
                    pl_sw = pl.fp32_switch;
                    to_start = b.types[t].start_off - tc.lo;
                }
                g = (int64_t)got + to_start;
                change = steps32.t != t;
                // from the first iterate (the first step was taken in FP64
                // where the start was written)
                const cd zd = roots[g];
                z = {(float)zd.re, (float)zd.im};
                it = 1;
                prev = 0.f;
            }
        }
        if (__ballot(change)) {
            flush_count(wc, C_STEPS_FP32, steps32);
            flush_count(wc, C_DIVERGED, ndiv);
            flush_count(wc, C_TIMEOUT, ntime);
        }
        if (change) steps32.t = ndiv.t = ntime.t = t;
        if (__ballot(!done) == 0) break;
        if (done) continue;
        cf P, dP;
        eval_q_f32_wave(pl_l, pl_N, z, P, dP);
        ++steps32.v;
        const float den = dP.re * dP.re + dP.im * dP.im;
        const float rd = __builtin_amdgcn_rcpf(den);
        const float sr = (P.re * dP.re + P.im * dP.im) * rd;
        const float si = (P.im * dP.re - P.re * dP.im) * rd;
        const float a2 = sr * sr + si * si;
        const float az2 = z.re * z.re + z.im * z.im;
        uint8_t st = ST_NONE;
        bool handoff = false;
        if (!isfinite(a2) || !(den > 0.f) || !isfinite(den) || a2 <= pl_sw * pl_sw * fmaxf(az2, 0x1p-16f)) {
            handoff = true; // FP64 continues from the last applied step
        } else {
            z = {z.re - sr, z.im - si};
            ++it;
            // FP32 only discards what is far outside M (|z| > 8); a long jump
            // or the cap hands the start to FP64, which decides (next to -2
            // FP32 evaluates P to rounding noise, and its steps mean nothing)
            const float zz = z.re * z.re + z.im * z.im;
            if (!(zz <= 64.f)) st = ST_DIVERGED;
            else if ((it > 3 && a2 > 64.f * prev) || it >= pl_cap) handoff = true;
            prev = a2;
        }
        if (handoff || st != ST_NONE) {
            // without an FP32 step the FP64 first iterate stays
            if (it > 1) roots[g] = cd{(double)z.re, (double)z.im};
            status[g] = st;
            iters[g] = (uint8_t)it;
            ndiv.v += st == ST_DIVERGED;
            ntime.v += st == ST_TIMEOUT;
            g = -1;
        }
    }
    flush_count(wc, C_STEPS_FP32, steps32);
    flush_count(wc, C_DIVERGED, ndiv);
    flush_count(wc, C_TIMEOUT, ntime);
}

// src holds the first iterates (one step counted) and, after the FP32 pass
// (AFTER32), its results for the types it ran on: starts it discarded keep
// their status, the others resume with the step count in iters.
// The lane state is kept small (32-bit start indices and type bounds, one
// type tag for the four 32-bit counts, branch-free status selection) so that
// the kernel fits 64 VGPRs: 8 waves per SIMD hide the load of a new start
// and the FP64 dependency latency of the orbit loop.
//
// ROUTE (some type of the call has a double-double route): a converged
// descent is marked ST_STALL, to be redone in double-double, when its last
// step did not show the quadratic convergence of a simple root, or when the
// root is too ill-conditioned for an FP64 centre: the certificate needs the
// image of D(c, R) under the orbit to stay small, R |P'| << 1, and an FP64
// centre leaves R ~ 2^-46 |z|, so |P'| 2^-46 |z| > 1/16 asks for a
// double-double centre.  iters[g] receives 1 when the descent ended within
// x_tip_max (the largest tip radius of the call, a kernel argument) of -2,
// whatever its status, 0 else: the routing pass reads that byte and tests
// the root against its type's own radius only where it is set.
template <bool ROUTE, bool AFTER32>
__global__ void __launch_bounds__(256) k_descend(batch_args b, const cd *src, cd *roots, uint8_t *status,
                                                 uint8_t *iters)
{
    constexpr uint32_t NONE = 0xffffffffu;
    unsigned long long *const wc = wave_ctr(b);
    const uint32_t n_starts = (uint32_t)b.n_starts;
    // per-lane counts of type ct: steps, converged, diverged, timeouts
    int ct = -1;
    uint32_t cnt[4] = {0u, 0u, 0u, 0u};
    const int slots[4] = {C_STEPS_DESC, C_CONVERGED, C_DIVERGED, C_TIMEOUT};
    uint32_t g = NONE;
    bool exhausted = false;
    int t = -1;
    uint32_t t_lo = 0, t_hi = 0;
    int pl_l = 0, pl_N = 1, pl_cap = 20;
    double pl_tol2 = 0.0;
    bool pl_route = false; // the type has a double-double route
    cd z = {0.0, 0.0};
    double prev = 0.0; // previous squared step length
    int it = 0, it0 = 0;
    bool fin = false, stall = false;
    wave_queue wq = wave_queue_start(b.chunk_start);
    unsigned long long *counter = &b.gctr[AFTER32 ? G_START_NEXT2 : G_START_NEXT];
    while (true) {
        const bool need = !exhausted && g == NONE;
        const uint64_t got = __ballot(need) ? wave_take_plain(wq, counter, b.chunk_start, need) : ~0ull;
        if (need) {
            if (got >= n_starts) {
                exhausted = true;
            } else {
                const uint32_t gg = (uint32_t)got;
                if (gg < t_lo || gg >= t_hi) {
                    t = find_type(b.start_offs, b.T, gg);
                    t_lo = (uint32_t)b.start_offs[t];
                    t_hi = (uint32_t)b.start_offs[t + 1];
                    const plan_t &pl = b.types[t].p;
                    pl_l = pl.el;
                    pl_N = pl.eN;
                    pl_cap = pl.cap;
                    pl_tol2 = pl.tol_desc * pl.tol_desc;
                    if (ROUTE) pl_route = pl.x_tip > 0.0;
                }
                // the FP32 pass ran on the starts of this type
                const bool ran32 = AFTER32 && fp32_eligible(pl_l, pl_N);
                if (!(ran32 && status[gg] != ST_NONE)) { // else: discarded by the FP32 pass
                    g = gg;
                    z = src[g];
                    // the first step from a start was taken where the start
                    // was written; after FP32 steps, their count
                    it0 = it = ran32 ? iters[g] : 1;
                    prev = 0.0;
                    fin = stall = false;
                }
            }
        }
        const bool change = g != NONE && t != ct;
        if (__ballot(change)) {
            // every lane flushes (and restarts) its counts
            wave_add4_by_key(wc, C_NCOUNTERS, ct, slots, cnt);
            cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0u;
            if (change) ct = t;
        }
        if (__ballot(g != NONE || !exhausted) == 0) break;
        if (g == NONE) continue;
        cd P, dP;
        eval_q_wave(pl_l, pl_N, z, P, dP);
        const double dp2 = ROUTE ? cabs2(dP) : 0.0; // |P'|^2 for the routing test (P' dies here)
        const cd d = cdiv_fast(P, dP);
        z = csub(z, d);
        ++it;
        // squared lengths: |d| and |z| compared without square roots;
        // a NaN or infinite value fails the <= tests
        const double a2 = cabs2(d);
        const double az2 = cabs2(z);
        // (the jump test counts the steps from the start, the first one or
        // the FP32 pass included, and needs a previous step of this descent)
        // wild: non-finite, or far outside M; such an iterate is never kept,
        // not even as the extra step after a small one (a P' = 0 there)
        const bool wild = !(a2 <= 0x1p1000) || !(az2 <= 64.0);
        const bool bad = wild || (it > 3 && it > it0 + 1 && a2 > 64.0 * prev);
        // converged once a step is small.  At a simple root the next step
        // would be about K |d|^2 with K = |d| / |d_prev|^2 (quadratic
        // convergence): when that is below the FP64 rounding of z the point
        // is final, else one more step is taken (the certificate settles the
        // accuracy a posteriori, Section 4.2)
        const bool small = a2 <= pl_tol2 * fmax(az2, 0x1p-16);
        const bool done = small && a2 * a2 * a2 <= 0x1p-106 * fmax(az2, 0x1p-16) * prev * prev;
        // a simple root is met by a step far below the one before (quadratic
        // convergence); a descent that creeps onto close roots or meets the
        // test on rounding noise does not, and is redone in double-double
        // (precision routing: progress stalled at the precision floor)
        if (ROUTE && small && !fin) {
            const bool slow = it > it0 + 1 && 64.0 * a2 > prev;
            const bool ill = dp2 * fmax(az2, 0x1p-16) > 0x1p84;
            stall = pl_route && (slow || ill);
        }
        const uint8_t st = (fin || done) && !wild ? (stall ? ST_STALL : ST_CONVERGED)
                           : bad ? ST_DIVERGED : (!small && it >= pl_cap) ? ST_TIMEOUT : ST_NONE;
        fin = small;
        prev = a2;
        cnt[0] += 1u;
        if (st != ST_NONE) {
            roots[g] = z;
            status[g] = st;
            if (ROUTE) {
                const double x = b.x_tip_max;
                iters[g] = (uint8_t)((int)(fabs(z.re + 2.0) < x) & (int)(fabs(z.im) < x));
            }
            cnt[1] += st == ST_CONVERGED || st == ST_STALL;
            cnt[2] += st == ST_DIVERGED;
            cnt[3] += st == ST_TIMEOUT;
            g = NONE;
        }
    }
    wave_add4_by_key(wc, C_NCOUNTERS, ct, slots, cnt);
}

// -------------------------------------------------------- nset collection
// Sort key of a root of the type of rank t: t above bit KEY_TYPE_SHIFT, then
// q = floor((re + 2.125) 2^KEY_RES), an exact integer below 2^KEY_BITS over
// re in [-2.125, 1.875).  Keys order the roots of a type by real part up to
// the resolution 2^-KEY_RES; the identification below reasons on key
// differences, so equal keys are harmless.  The candidates reach the sort
// grouped by type (start order), and the sort keeps that grouping, so only
// the KEY_BITS of the real part are sorted.
constexpr int KEY_TYPE_SHIFT = 50;
constexpr int KEY_RES = 46;
constexpr int KEY_BITS = KEY_RES + 2;
// Bit KEY_BITS of a stored candidate key: the candidate is a double-double
// root.  The sort orders the KEY_BITS bits below it, so the flag travels with
// its key (the gather then needs no status of the start).
constexpr int KEY_DD_BIT = KEY_BITS;
constexpr uint64_t KEY_POS_MASK = (1ull << KEY_BITS) - 1ull;

__device__ __forceinline__ uint64_t root_key(int t, double re, bool dd = false)
{
    const double x = fmin(fmax(re, -2.125), 1.875 - 0x1p-46);
    const int64_t q = (int64_t)floor(x * 0x1p46) + (int64_t)(17ll << 43); // 2.125 2^46
    return ((uint64_t)t << KEY_TYPE_SHIFT) | ((uint64_t)dd << KEY_DD_BIT) | (uint64_t)q;
}
__device__ __forceinline__ int key_type(uint64_t key) { return (int)(key >> KEY_TYPE_SHIFT); }
__device__ __forceinline__ bool key_dd(uint64_t key) { return (key >> KEY_DD_BIT) & 1ull; }

// Keys i > j of one type with key_i - key_j >= key_window(tau) have
// re_i - re_j > (key_i - key_j - 1) 2^-KEY_RES >= tau, and so have all
// earlier j.
__device__ __forceinline__ uint64_t key_window(double tau) { return 1ull + (uint64_t)ceil(tau * 0x1p46); }

// Fold to the closed upper half plane and snap to the real axis when the
// imaginary part is below both tau/2 and the rounding level of a converged
// descent (2^-46 |z|): q_{l,n} has genuine non-real roots next to -2 whose
// imaginary part (about 4^-(l+n)) falls below tau/2.
__device__ __forceinline__ cd fold_snap(cd z, double tau)
{
    z.im = fabs(z.im);
    if (z.im < fmin(0.5 * tau, 0x1p-46 * fmax(fabs(z.re), 0x1p-8))) z.im = 0.0;
    return z;
}

// The same for a double-double root (hi, lo): the sign of the imaginary part
// is that of hi + lo; snapped below the double-double rounding level.
__device__ __forceinline__ void fold_snap_dd(cd &hi, cd &lo, double tau_dd)
{
    if (hi.im < 0.0 || (hi.im == 0.0 && lo.im < 0.0)) {
        hi.im = -hi.im;
        lo.im = -lo.im;
    }
    if (hi.im + lo.im < fmin(0.5 * tau_dd, 0x1p-96 * fmax(fabs(hi.re), 0x1p-8))) {
        hi.im = 0.0;
        lo.im = 0.0;
    }
}

// nset identification of two folded roots: within tau_dd in both coordinates
// when both are double-double (differences of hi parts are exact for close
// values), else within tau on the FP64 parts.
__device__ __forceinline__ bool same_root(cd a, cd alo, bool add, cd b, cd blo, bool bdd, double tau, double tau_dd)
{
    if (add && bdd) {
        const double dr = (a.re - b.re) + (alo.re - blo.re);
        const double di = (a.im - b.im) + (alo.im - blo.im);
        return fabs(dr) < tau_dd && fabs(di) < tau_dd;
    }
    return fabs(a.re - b.re) < tau && fabs(a.im - b.im) < tau;
}

// Type of item g from a copy of the offsets in LDS (T + 1 entries).
__device__ __forceinline__ int find_type_lds(const int64_t *offs, int T, int64_t g)
{
    int lo = 0, hi = T;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offs[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// LDS copies of the start offsets and of each type's identification radius
struct collect_tables {
    int64_t offs[MAX_TYPES + 1];
    double tau[MAX_TYPES], tau_dd[MAX_TYPES];
};

__device__ __forceinline__ void load_tables_lds(collect_tables &c, const batch_args &b)
{
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) {
        c.offs[i] = b.start_offs[i];
        if (i < b.T) {
            c.tau[i] = b.types[i].p.tau;
            c.tau_dd[i] = b.types[i].p.tau_dd;
        }
    }
}

// Fold to the closed upper half plane, snap |Im| < tau/2 to the real axis
// (Section 6.1, nset), and drop a start whose root repeats the root of one
// of the PREKEY_WINDOW previous converged starts of the same type: the starts
// of one level-line turn mostly reach the same root (73% repeats, Section
// 6.4.2), so this local identification removes most duplicates before the
// sort.  A block stages its starts and the window before them in LDS; every
// global load is issued before the first wait.
constexpr int PREKEY_WINDOW = 8;
constexpr int COLLECT_BLOCK = 256;

// window = 0 keeps every converged start (candidates that are already
// identified, where only the sort's identification may decide).  Tiles of
// PK_TILE starts, four per thread (launched one tile per block; a smaller
// grid loops over them): each thread has five starts' loads in flight at
// once, and the barriers of a tile serve four starts per thread.  A tile
// inside one type (almost every tile) takes its type from the previous tile
// or one search, not one search per start, and each start reads its window
// from LDS before comparing, so that no comparison waits on the one before.
//
// The survivors of tile k leave as (key, start index) pairs at tile-local
// positions k PK_TILE + rank (rank: survivors of the tile before it, in start
// order), tcount[k] their number; k_compact moves them to the scanned
// positions, so the roots are read once.  surv_offs[t] receives the
// tile-local rank of type t's first start (made a position by k_compact).
constexpr int PK_PER = 4;
constexpr int PK_TILE = COLLECT_BLOCK * PK_PER;
constexpr int PK_WAVES = COLLECT_BLOCK / 64;

__global__ void __launch_bounds__(COLLECT_BLOCK) k_prekeys(batch_args b, const cd *roots, const cd *roots_lo,
                                                           const uint8_t *status, uint64_t *tkeys, uint32_t *tvals,
                                                           uint32_t *tcount, int window)
{
    __shared__ collect_tables tabs;
    __shared__ cd zs[PK_TILE + PREKEY_WINDOW];
    __shared__ int ts[PK_TILE + PREKEY_WINDOW]; // type, | 1 << 16 when double-double; -1: not converged
    __shared__ uint32_t wcnt[PK_PER][PK_WAVES];  // survivors per (start slot, wave) of the tile
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    load_tables_lds(tabs, b);
    const int64_t ntiles = (b.n_starts + PK_TILE - 1) / PK_TILE;
    const bool has1 = threadIdx.x < PREKEY_WINDOW;
    int tc = 0; // type of the last tile (block-uniform)
    auto stage = [&](int i, int64_t g, uint8_t st, cd z, int tu) {
        int t = -1;
        if (st_converged(st)) {
            t = tu >= 0 ? tu : find_type_lds(tabs.offs, b.T, g);
            if (st == ST_DD) {
                cd lo = roots_lo[g];
                fold_snap_dd(z, lo, tabs.tau_dd[t]);
                t |= 1 << 16;
            } else {
                z = fold_snap(z, tabs.tau[t]);
            }
        }
        ts[i] = t;
        zs[i] = z;
    };
    // the low part of a double-double start, folded like its high part
    auto lo_of = [&](int64_t g, double tdd) {
        cd z = roots[g], lo = roots_lo[g];
        fold_snap_dd(z, lo, tdd);
        return lo;
    };
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // staged item k of the thread: start base + threadIdx.x + k COLLECT_BLOCK
        // (k = PK_PER: the last PREKEY_WINDOW starts, threads below PREKEY_WINDOW)
        const int64_t base = tile * PK_TILE - PREKEY_WINDOW;
        uint8_t st[PK_PER + 1];
        cd zz[PK_PER + 1];
#pragma unroll
        for (int k = 0; k <= PK_PER; ++k) {
            const int64_t g = base + threadIdx.x + (int64_t)k * COLLECT_BLOCK;
            const bool v = (k < PK_PER || has1) && g >= 0 && g < b.n_starts;
            st[k] = v ? status[g] : ST_NONE;
            zz[k] = v ? roots[g] : cd{0.0, 0.0};
        }
        __syncthreads(); // the tables (first tile), or the previous tile's reads
        // the staged range [lo_g, hi_g] inside type tc: one type for the tile
        const int64_t lo_g = base > 0 ? base : 0;
        const int64_t hi_g = min(base + PK_TILE + PREKEY_WINDOW, b.n_starts) - 1;
        if (!(tabs.offs[tc] <= lo_g && lo_g < tabs.offs[tc + 1])) tc = find_type_lds(tabs.offs, b.T, lo_g);
        tc = __builtin_amdgcn_readfirstlane(tc);
        const int tu = hi_g < tabs.offs[tc + 1] ? tc : -1;
#pragma unroll
        for (int k = 0; k <= PK_PER; ++k)
            if (k < PK_PER || has1)
                stage(threadIdx.x + k * COLLECT_BLOCK, base + threadIdx.x + (int64_t)k * COLLECT_BLOCK, st[k], zz[k],
                      tu);
        __syncthreads();
        bool surv[PK_PER];
#pragma unroll
        for (int k = 0; k < PK_PER; ++k) {
            const int i = PREKEY_WINDOW + threadIdx.x + k * COLLECT_BLOCK;
            const int64_t g = base + i;
            const int tt = g < b.n_starts ? ts[i] : -1;
            bool f = false;
            if (tt >= 0) {
                const int t = tt & 0xffff;
                const bool dd = (tt >> 16) != 0;
                const double tau = tabs.tau[t], tdd = tabs.tau_dd[t];
                const cd z = zs[i];
                bool same = false, dd_pair = false;
                // the window in two halves: each half read from LDS before its
                // comparisons
                constexpr int H = PREKEY_WINDOW / 2;
#pragma unroll
                for (int h = 0; h < PREKEY_WINDOW; h += H) {
                    int tj[H];
                    cd zj[H];
#pragma unroll
                    for (int d = 0; d < H; ++d) {
                        tj[d] = ts[i - 1 - h - d];
                        zj[d] = zs[i - 1 - h - d];
                    }
                    // bitwise, not short-circuit: no branch per comparison
#pragma unroll
                    for (int d = 0; d < H; ++d) {
                        const bool ok = (h + d < window) & (tj[d] >= 0) & ((tj[d] & 0xffff) == t);
                        const bool both = dd & ((tj[d] >> 16) != 0);
                        const bool near = (int)(fabs(z.re - zj[d].re) < tau) & (int)(fabs(z.im - zj[d].im) < tau);
                        dd_pair |= ok & both;
                        same |= ok & !both & near;
                    }
                }
                // two double-double roots compare with their low parts (rare:
                // read again from the descents' results)
                if (!same && dd_pair) {
                    const cd zl = lo_of(g, tdd);
                    for (int d = 1; d <= window && !same; ++d) {
                        const int tjd = ts[i - d];
                        if (tjd < 0 || (tjd & 0xffff) != t || (tjd >> 16) == 0) continue;
                        same = same_root(z, zl, true, zs[i - d], lo_of(g - d, tdd), true, tau, tdd);
                    }
                }
                f = !same;
            }
            surv[k] = f;
        }
        // ranks in start order (slot k of every thread, then slot k + 1):
        // survivors per (slot, wave) by ballot, then prefix sums
        uint64_t bal[PK_PER];
#pragma unroll
        for (int k = 0; k < PK_PER; ++k) {
            bal[k] = __ballot(surv[k]);
            if (lane == 0) wcnt[k][wv] = (uint32_t)__popcll(bal[k]);
        }
        __syncthreads();
        const int64_t tile0 = tile * PK_TILE;
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < PK_PER; ++k) {
            uint32_t before = 0, all = 0;
#pragma unroll
            for (int w = 0; w < PK_WAVES; ++w) {
                const uint32_t c = wcnt[k][w];
                before += w < wv ? c : 0u;
                all += c;
            }
            const uint32_t rank = run + before +
                                  __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[k] >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bal[k], 0u));
            run += all;
            const int i = PREKEY_WINDOW + threadIdx.x + k * COLLECT_BLOCK;
            const int64_t g = base + i;
            if (g >= b.n_starts) continue;
            if (surv[k]) {
                const int tt = ts[i];
                tkeys[tile0 + rank] = root_key(tt & 0xffff, zs[i].re, (tt >> 16) != 0);
                tvals[tile0 + rank] = (uint32_t)g;
            }
            const int t = tu >= 0 ? tu : find_type_lds(tabs.offs, b.T, g);
            if (g == tabs.offs[t]) b.surv_offs[t] = (int64_t)rank;
        }
        if (threadIdx.x == 0) tcount[tile] = run;
        __syncthreads(); // the reads above before the next tile's staging
    }
}

// Survivors of each prekeys tile to their positions tpos[k] (the scan of
// tcount): (key, start index) pairs grouped by type in start order.  Block 0
// turns surv_offs[t] (a tile-local rank) into the first position of type t,
// and sets surv_offs[T] = the number of survivors.
__global__ void __launch_bounds__(COLLECT_BLOCK) k_compact(batch_args b, const uint64_t *tkeys, const uint32_t *tvals,
                                                           const uint32_t *tcount, const uint32_t *tpos,
                                                           uint64_t *keys, uint32_t *vals)
{
    const int64_t ntiles = (b.n_starts + PK_TILE - 1) / PK_TILE;
    if (blockIdx.x == 0) {
        const int64_t total = ntiles ? (int64_t)tpos[ntiles - 1] + tcount[ntiles - 1] : 0;
        for (int t = threadIdx.x; t <= b.T; t += blockDim.x) {
            const int64_t g = b.start_offs[t];
            b.surv_offs[t] = t < b.T && g < b.n_starts ? b.surv_offs[t] + (int64_t)tpos[g / PK_TILE] : total;
        }
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t c = tcount[tile];
        const int64_t dst = tpos[tile], src = tile * PK_TILE;
        for (uint32_t e = threadIdx.x; e < c; e += blockDim.x) {
            keys[dst + e] = tkeys[src + e];
            vals[dst + e] = tvals[src + e];
        }
    }
}

// The sorted candidates, folded and snapped, in sort order: one gather, so
// that the identification and the output pass read them in sequence.
// Grid-stride over the m = surv_offs[T] candidates.
// The low part (zs_lo) is written for double-double candidates only, and
// read only where zs_dd is set.
__global__ void k_gather(batch_args b, const cd *roots, const cd *roots_lo, const uint64_t *keys,
                         const uint32_t *vals, cd *zs, cd *zs_lo, uint8_t *zs_dd)
{
    const int64_t m = b.surv_offs[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const uint32_t v = vals[i];
        const uint64_t key = keys[i];
        const int t = key_type(key);
        if (v >= b.n_starts || t >= b.T) { // not a sorted candidate: never matches
            const double nan = __longlong_as_double(0x7ff8000000000000ll);
            zs[i] = {nan, nan};
            zs_dd[i] = 0;
            continue;
        }
        const plan_t &pl = b.types[t].p;
        cd z = roots[v];
        const bool dd = key_dd(key);
        if (dd) {
            cd lo = roots_lo[v];
            fold_snap_dd(z, lo, pl.tau_dd);
            zs_lo[i] = lo;
        } else {
            z = fold_snap(z, pl.tau);
        }
        zs[i] = z;
        zs_dd[i] = dd;
    }
}

// A sorted point is a duplicate when an earlier point of the same type is the
// same root (same_root: the nset identification, the first point of a
// cluster kept).  The backward scan stops at the key window (real parts tau
// apart) or after MARK_LOOKBACK points.  The window is crowded only where
// FP64 keys collapse: next to -2, where the roots of p_n lie about 4^-n apart
// and each is reached from several starts, some hundred candidates of order
// 31 share a window.  A scan ended by the bound, not by the window, is
// counted (C_MARK_CAPPED): a duplicate may survive it.
constexpr int MARK_LOOKBACK = 4096;

__global__ void k_mark(batch_args b, const uint64_t *keys, const cd *zs, const cd *zs_lo, const uint8_t *zs_dd,
                       uint32_t *flag)
{
    unsigned long long *const wc = wave_ctr(b);
    const int64_t m = b.surv_offs[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    type_count capped;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < m; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        bool cap_hit = false;
        int t = -1;
        if (i < m) {
            const uint64_t ki = keys[i];
            t = key_type(ki);
            uint32_t f = 1;
            if (t < b.T) {
                const double tau = b.types[t].p.tau, tdd = b.types[t].p.tau_dd;
                const uint64_t win = key_window(tau);
                const cd zero = {0.0, 0.0};
                const bool di = zs_dd[i];
                const cd zi = zs[i], li = di ? zs_lo[i] : zero;
                int c = 0;
                for (int64_t j = i - 1; j >= 0 && c < MARK_LOOKBACK; --j, ++c) {
                    const uint64_t kj = keys[j];
                    if (key_type(kj) != t || (ki & KEY_POS_MASK) - (kj & KEY_POS_MASK) >= win) break;
                    const bool dj = zs_dd[j];
                    if (same_root(zi, li, di, zs[j], di && dj ? zs_lo[j] : zero, dj, tau, tdd)) { f = 0; break; }
                }
                cap_hit = f && c == MARK_LOOKBACK;
            }
            flag[i] = f;
        }
        if (__ballot(cap_hit && t != capped.t)) flush_count(wc, C_MARK_CAPPED, capped);
        if (cap_hit) {
            capped.t = t;
            capped.v += 1;
        }
    }
    flush_count(wc, C_MARK_CAPPED, capped);
}

// Per type: first index in the collected index space (coll_offs, from the
// scanned marks at the type's first sorted index); the number of collected
// roots (C_UNIQUE) and of sorted candidates (C_SURVIVORS) go to the first
// counter copy (the fold adds the copies).  One block.
__global__ void k_type_bounds(batch_args b, const uint32_t *flag, const uint32_t *pos)
{
    const int64_t m = b.surv_offs[b.T];
    auto pos_at = [&](int64_t i) -> int64_t { return i < m ? pos[i] : (m ? pos[m - 1] + flag[m - 1] : 0); };
    for (int t = threadIdx.x; t <= b.T; t += blockDim.x) b.coll_offs[t] = pos_at(b.surv_offs[t]);
    __syncthreads();
    for (int t = threadIdx.x; t < b.T; t += blockDim.x) {
        b.spread[(int64_t)t * C_NCOUNTERS + C_UNIQUE] = (uint64_t)(b.coll_offs[t + 1] - b.coll_offs[t]);
        b.spread[(int64_t)t * C_NCOUNTERS + C_SURVIVORS] = (uint64_t)(b.surv_offs[t + 1] - b.surv_offs[t]);
    }
}

// The identified roots into the collected index space (type-major, by real
// part within a type).
__global__ void k_scatter(batch_args b, const uint32_t *flag, const uint32_t *pos, const cd *zs, const cd *zs_lo,
                          const uint8_t *zs_dd, cd *uz, cd *uz_lo, uint8_t *uz_dd)
{
    const int64_t m = b.surv_offs[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        if (!flag[i]) continue;
        const uint32_t u = pos[i];
        if (u >= b.n_starts) continue;
        const bool dd = zs_dd[i];
        uz[u] = zs[i];
        uz_lo[u] = dd ? zs_lo[i] : cd{0.0, 0.0};
        uz_dd[u] = dd;
    }
}

// ---------------------------------------------------------- classification
// p_n: exact period = least k | n with p_k(root) = 0 (eq. def:hyp), tested by
// the Newton distance |p_k / p_k'| < tau.  tau is the identification radius,
// far below the least distance between roots of p_n (118.4 / 4^n, Section
// 6.3.2): a root of period n can sit that close to a root of period n/2 (the
// centre of a satellite next to its parent), so the scale of p_k alone would
// not do.  One orbit pass serves all divisors.
__device__ __forceinline__ int classify_p(int n, uint32_t divmask, double tau, cd c)
{
    // the orbit on u = 2 p_k from p_1 = c, p_1' = 1; |p_k|^2 = |u|^2 / 4,
    // up to the largest strict divisor of n (no test after it)
    orbit2_state<double> s = {2.0 * c.re, 2.0 * c.im, 1.0, 0.0};
    const double c4r = 4.0 * c.re, c2i = 2.0 * c.im;
    const int kmax = divmask ? 31 - __builtin_clz(divmask) : 0;
    for (int k = 1; k <= kmax; ++k) {
        if (k > 1) orbit2_step(s, c4r, c2i);
        if ((divmask >> k) & 1u) {
            const double a2 = 0.25 * (s.ur * s.ur + s.ui * s.ui);
            const double d2 = s.dr * s.dr + s.di * s.di;
            if (a2 < tau * tau * d2) return k;
        }
    }
    return n;
}

// q_{l,n}, l >= 2: keep c when it is a root of type Mis(l,n) (eq. def:mis).
// By Thm fact_mis the roots of q_{l,n} are the centres Hyp(k), k | n, with
// multiplicity eta_l(k) >= 2, and the simple roots Mis(j,k), 2 <= j <= l,
// k | n.  The lower types are recognised by a vanishing Newton distance
// (< tau):
//   Hyp(k):        p_k,          k | n;
//   Mis(j,n), j<l: q_{l-1,n} = z_{l-1+n} - z_{l-1};
//   Mis(j,k), k<n: q_{l,k}   = z_{l+k} - z_l,  k | n, k < n.
// A descent can also stop next to a multiple root, where FP64 evaluates q at
// noise level: at distance d from Hyp(k) the exact Newton step of q is
// d / eta and the Newton distance of p_k (a simple root there) is d, so their
// ratio is at most eta <= 64, while at a genuine simple root of q the step is
// at the rounding of c and p_k is a root separation away.  Near a centre
// (p_k Newton distance < 1e-6) both are taken from a double-double orbit and
// the point is kept only when 64 |step| < |p_k / p_k'|.
__device__ __forceinline__ bool newton_dist_below(double ar, double ai, double br, double bi, double tau)
{
    return ar * ar + ai * ai < tau * tau * (br * br + bi * bi);
}

__device__ __noinline__ bool stalled_at_multiple_root(int l, int n, int k, cd c)
{
    const cdd cc = {{c.re, 0.0}, {c.im, 0.0}};
    cdd z = {{0.0, 0.0}, {0.0, 0.0}}, zl = z, zk = z;
    double dr = 0.0, di = 0.0, dlr = 0.0, dli = 0.0, dkr = 0.0, dki = 0.0;
    for (int i = 1; i <= l + n; ++i) {
        // dz <- 2 z dz + 1 (FP64 scale), z <- z^2 + c (double-double)
        const double tr = z.re.hi * dr - z.im.hi * di, ti = z.re.hi * di + z.im.hi * dr;
        dr = 2.0 * tr + 1.0;
        di = 2.0 * ti;
        z = cdd_sqr_add(z, cc);
        if (i == k) { zk = z; dkr = dr; dki = di; }
        if (i == l) { zl = z; dlr = dr; dli = di; }
    }
    const cdd q = cdd_sub(z, zl);
    const double s2 = cdd_abs2_hi(q) / ((dr - dlr) * (dr - dlr) + (di - dli) * (di - dli));
    const double h2 = cdd_abs2_hi(zk) / (dkr * dkr + dki * dki);
    return !(64.0 * 64.0 * s2 < h2);
}

__device__ __forceinline__ bool classify_q(int l, int n, uint32_t divmask, double tau, cd c, double &hmin2_out,
                                           int &kmin_out)
{
    orbit_state<double> s = {0.0, 0.0, 0.0, 0.0};
    double zlm_r = 0.0, zlm_i = 0.0, dlm_r = 0.0, dlm_i = 0.0; // z_{l-1}, dz_{l-1}
    double zl_r = 0.0, zl_i = 0.0, dl_r = 0.0, dl_i = 0.0;     // z_l, dz_l
    bool keep = true;
    double hmin2 = INFINITY; // least squared Newton distance of p_k, k | n
    int kmin = 0;
    const int N = l + n;
    for (int i = 1; i <= N; ++i) {
        orbit_step(s, c.re, c.im);
        if (i <= n && (i == n || ((divmask >> i) & 1u))) {
            const double h2 = (s.zr * s.zr + s.zi * s.zi) / (s.dr * s.dr + s.di * s.di);
            if (h2 < hmin2) { hmin2 = h2; kmin = i; }
            if (newton_dist_below(s.zr, s.zi, s.dr, s.di, tau)) keep = false; // Hyp(i), i | n
        }
        if (i == l - 1) { zlm_r = s.zr; zlm_i = s.zi; dlm_r = s.dr; dlm_i = s.di; }
        if (i == l) { zl_r = s.zr; zl_i = s.zi; dl_r = s.dr; dl_i = s.di; }
        const int k = i - l;
        if (k >= 1 && k < n && ((divmask >> k) & 1u) &&
            newton_dist_below(s.zr - zl_r, s.zi - zl_i, s.dr - dl_r, s.di - dl_i, tau))
            keep = false; // Mis(j,k), k < n
        if (i == l - 1 + n && newton_dist_below(s.zr - zlm_r, s.zi - zlm_i, s.dr - dlm_r, s.di - dlm_i, tau))
            keep = false; // Mis(j,n), j < l
    }
    hmin2_out = hmin2;
    kmin_out = kmin;
    return keep;
}

// The same classifications for a double-double root: the orbit z_k in
// double-double, its derivative in FP64 (a Newton distance |A / B| only needs
// B to FP64 accuracy), identification radius tau_dd.
__device__ __forceinline__ bool dd_dist_below(cdd a, double br, double bi, double tau)
{
    return cdd_abs2_hi(a) < tau * tau * (br * br + bi * bi);
}

__device__ __noinline__ int classify_p_dd(int n, uint32_t divmask, double tau, cdd c)
{
    cdd z = {{0.0, 0.0}, {0.0, 0.0}};
    double dr = 0.0, di = 0.0;
    // up to the largest strict divisor of n (no test after it)
    const int kmax = divmask ? 31 - __builtin_clz(divmask) : 0;
    for (int k = 1; k <= kmax; ++k) {
        const double tr = z.re.hi * dr - z.im.hi * di, ti = z.re.hi * di + z.im.hi * dr;
        dr = 2.0 * tr + 1.0;
        di = 2.0 * ti;
        z = cdd_sqr_add(z, c);
        if (((divmask >> k) & 1u) && dd_dist_below(z, dr, di, tau)) return k;
    }
    return n;
}

// Inside the rounding-noise ball of a multiple root q evaluates to noise
// (even to exactly 0), so the step ratio can miss a point stalled there; the
// caller settles every candidate near a centre with the certificate.
__device__ __noinline__ bool classify_q_dd(int l, int n, uint32_t divmask, double tau, cdd c, double &hmin2_out,
                                           int &kmin_out)
{
    const cdd zero = {{0.0, 0.0}, {0.0, 0.0}};
    cdd z = zero, zlm = zero, zl = zero;
    double dr = 0.0, di = 0.0, dlm_r = 0.0, dlm_i = 0.0, dl_r = 0.0, dl_i = 0.0;
    bool keep = true;
    double hmin2 = INFINITY;
    int kmin = n;
    const int N = l + n;
    for (int i = 1; i <= N; ++i) {
        const double tr = z.re.hi * dr - z.im.hi * di, ti = z.re.hi * di + z.im.hi * dr;
        dr = 2.0 * tr + 1.0;
        di = 2.0 * ti;
        z = cdd_sqr_add(z, c);
        if (i <= n && (i == n || ((divmask >> i) & 1u))) {
            const double h2 = cdd_abs2_hi(z) / (dr * dr + di * di);
            if (h2 < hmin2) { hmin2 = h2; kmin = i; }
            if (dd_dist_below(z, dr, di, tau)) keep = false; // Hyp(i)
        }
        if (i == l - 1) { zlm = z; dlm_r = dr; dlm_i = di; }
        if (i == l) { zl = z; dl_r = dr; dl_i = di; }
        const int k = i - l;
        if (k >= 1 && k < n && ((divmask >> k) & 1u) && dd_dist_below(cdd_sub(z, zl), dr - dl_r, di - dl_i, tau))
            keep = false; // Mis(j,k), k < n
        if (i == l - 1 + n && dd_dist_below(cdd_sub(z, zlm), dr - dlm_r, di - dlm_i, tau))
            keep = false; // Mis(j,n), j < l
    }
    // next to a multiple root (Hyp(k)): step of q within 64 times the p_k distance
    const cdd q = cdd_sub(z, zl);
    const double s2 = cdd_abs2_hi(q) / ((dr - dl_r) * (dr - dl_r) + (di - dl_i) * (di - dl_i));
    if (keep && hmin2 < 1e-12 && !(64.0 * 64.0 * s2 < hmin2)) keep = false;
    hmin2_out = hmin2;
    kmin_out = kmin;
    return keep;
}

// Per type: first index in the kept index space; kept count in C_KEPT; the
// output index space of the certificate, uniq_offs, with min(kept, capacity)
// roots per type.  One block.
__global__ void k_kept_bounds(batch_args b, const uint32_t *keep, const uint32_t *kpos)
{
    const int64_t n = b.coll_offs[b.T];
    auto kpos_at = [&](int64_t u) -> int64_t { return u < n ? kpos[u] : (n ? kpos[n - 1] + keep[n - 1] : 0); };
    for (int t = threadIdx.x; t <= b.T; t += blockDim.x) {
        b.kept_offs[t] = kpos_at(b.coll_offs[t]);
        if (t < b.T)
            b.spread[(int64_t)t * C_NCOUNTERS + C_KEPT] =
                (uint64_t)(kpos_at(b.coll_offs[t + 1]) - kpos_at(b.coll_offs[t]));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0;
        b.uniq_offs[0] = 0;
        for (int t = 0; t < b.T; ++t) {
            const int64_t k = b.kept_offs[t + 1] - b.kept_offs[t];
            a += (uint64_t)k < b.types[t].cap ? k : (int64_t)b.types[t].cap;
            b.uniq_offs[t + 1] = a;
        }
    }
}

// Kept roots to the caller's output slices (at most the capacity of each),
// with period, preperiod and the real flag; real roots counted per type.
// Grid-stride over the collected index space.
__global__ void __launch_bounds__(256) k_emit(batch_args b, const cd *uz, const cd *uz_lo, const uint8_t *uz_dd,
                                              const uint32_t *keep, const uint32_t *kpos, const int32_t *cls,
                                              double *ore, double *oim, double *ore_lo, double *oim_lo,
                                              int32_t *period, int32_t *preperiod, uint8_t *flags)
{
    __shared__ int64_t offs[MAX_TYPES + 1];
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) offs[i] = b.coll_offs[i];
    __syncthreads();
    unsigned long long *const wc = wave_ctr(b);
    const int64_t n = offs[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    type_count nreal;
    for (int64_t u0 = (int64_t)blockIdx.x * blockDim.x; u0 < n; u0 += stride) {
        const int64_t u = u0 + threadIdx.x;
        const bool act = u < n && keep[u];
        const int t = act ? find_type_lds(offs, b.T, u) : nreal.t;
        if (__ballot(act && t != nreal.t)) flush_count(wc, C_REAL, nreal);
        nreal.t = t;
        if (!act) continue;
        const type_desc &td = b.types[t];
        const int64_t rank = (int64_t)kpos[u] - b.kept_offs[t];
        const cd z = uz[u];
        if ((uint64_t)rank < td.cap) {
            const int64_t i = td.out_off + rank;
            const bool dd = uz_dd[u];
            const cd lo = dd ? uz_lo[u] : cd{0.0, 0.0};
            ore[i] = z.re;
            oim[i] = z.im;
            if (ore_lo) ore_lo[i] = lo.re;
            if (oim_lo) oim_lo[i] = lo.im;
            if (period) period[i] = cls[u];
            if (preperiod) preperiod[i] = td.p.l;
            if (flags) flags[i] = (z.im == 0.0 ? 1 : 0) | (dd ? 8 : 0); // MSPLIT_R_REAL, MSPLIT_R_DD
        }
        nreal.v += z.im == 0.0;
    }
    flush_count(wc, C_REAL, nreal);
}

// MSPLIT_F_CONJUGATES: the output as all the roots of P, a non-real root of
// the upper half plane followed by nothing but its conjugate (real
// coefficients: conj(c) is a root, certified by the mirrored disk).  Over the
// output index space (uniq_offs: type t's roots at out_off + rank): w[u] = 1
// for a real root, 2 otherwise (scanned next), and the fields to a staging
// copy, which the scatter then writes back expanded, in (Re, Im) order.
struct conj_stage {
    double *re, *im, *re_lo, *im_lo, *radius, *basin;
    int32_t *period, *preperiod;
    uint8_t *flags;
};

__device__ __forceinline__ int64_t out_index(const batch_args &b, const int64_t *uo, int64_t u, int &t)
{
    t = find_type_lds(uo, b.T, u);
    return b.types[t].out_off + (u - uo[t]);
}

__global__ void k_conj_stage(batch_args b, const double *ore, const double *oim, const double *ore_lo,
                             const double *oim_lo, const int32_t *period, const int32_t *preperiod,
                             const uint8_t *flags, const double *radius, const double *basin, conj_stage s,
                             uint32_t *w)
{
    __shared__ int64_t uo[MAX_TYPES + 1];
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) uo[i] = b.uniq_offs[i];
    __syncthreads();
    const int64_t n = uo[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        int t;
        const int64_t i = out_index(b, uo, u, t);
        const double im = oim[i], lo = oim_lo ? oim_lo[i] : 0.0;
        s.re[u] = ore[i];
        s.im[u] = im;
        if (ore_lo) s.re_lo[u] = ore_lo[i];
        if (oim_lo) s.im_lo[u] = lo;
        if (period) s.period[u] = period[i];
        if (preperiod) s.preperiod[u] = preperiod[i];
        if (flags) s.flags[u] = flags[i];
        if (radius) s.radius[u] = radius[i];
        if (basin) s.basin[u] = basin[i];
        w[u] = (im == 0.0 && lo == 0.0) ? 1u : 2u;
    }
}

__global__ void k_conj_scatter(batch_args b, conj_stage s, const uint32_t *pos, double *ore, double *oim,
                               double *ore_lo, double *oim_lo, int32_t *period, int32_t *preperiod, uint8_t *flags,
                               double *radius, double *basin)
{
    __shared__ int64_t uo[MAX_TYPES + 1];
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) uo[i] = b.uniq_offs[i];
    __syncthreads();
    const int64_t n = uo[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        const int t = find_type_lds(uo, b.T, u);
        const type_desc &td = b.types[t];
        // position within the type: scanned weights from the type's first root
        const int64_t r = (int64_t)pos[u] - (int64_t)pos[uo[t]];
        const double im = s.im[u], lo = oim_lo ? s.im_lo[u] : 0.0;
        const int w = (im == 0.0 && lo == 0.0) ? 1 : 2;
        for (int k = 0; k < w; ++k) {
            if ((uint64_t)(r + k) >= td.cap) break;
            const int64_t i = td.out_off + r + k;
            const double sg = (w == 2 && k == 0) ? -1.0 : 1.0; // the conjugate first
            ore[i] = s.re[u];
            oim[i] = sg * im;
            if (ore_lo) ore_lo[i] = s.re_lo[u];
            if (oim_lo) oim_lo[i] = sg * lo;
            if (period) period[i] = s.period[u];
            if (preperiod) preperiod[i] = s.preperiod[u];
            if (flags) flags[i] = s.flags[u];
            if (radius) radius[i] = s.radius[u];
            if (basin) basin[i] = s.basin[u];
        }
    }
}

} // namespace msplit
