// tip.hpp -- the double-double route for the roots next to c = -2.
//
// Near the tip of M the roots crowd together: for p_n their least distance
// is about 118.4 / 4^n (Section 6.3.2), and among the Misiurewicz parameters
// two real ones at the left end of M come closer still, below the FP80
// spacing at order 26 (Section 6.3.2, the Mis separation histogram).  FP64
// cannot tell such roots apart.  Descents whose FP64 result lands within
// x_tip of -2 are therefore redone from their starting point in
// double-double (Section 6.4: the high-precision fraction of the job), and
// their roots are identified, classified and certified in double-double.
#pragma once
#include "kernels.hpp"
#include "dd.hpp"

namespace msplit {

// Newton step of q_{l,n} (l = 0: p_n) at z in double-double: the orbit z_k
// in double-double, its derivative in FP64 (only the scale of the step needs
// it: the step then has a relative error of about 2^-53, so a step of 2^-53
// leaves an error of 2^-106).  Returns the step P / P' in double-double and
// |P'|^2 in FP64.
struct dd_step { cdd s; double d2; };

__device__ __forceinline__ dd dd_div_by(dd a, double b)
{
    DD_EXACT
    const double q1 = a.hi / b;
    const dd p = two_prod(q1, b);
    const double q2 = ((a.hi - p.hi) - p.lo + a.lo) / b;
    return quick_two_sum(q1, q2);
}

__device__ dd_step dd_newton_step(int l, int N, cdd c)
{
    // l < 0: P = z_N + z_{-l} (the simplified polynomial, as eval_q_t)
    const int la = l < 0 ? -l : l;
    cdd z = {{0.0, 0.0}, {0.0, 0.0}}, zl = z;
    double dr = 0.0, di = 0.0, dlr = 0.0, dli = 0.0;
    for (int i = 1; i <= N; ++i) {
        const double tr = z.re.hi * dr - z.im.hi * di, ti = z.re.hi * di + z.im.hi * dr;
        dr = 2.0 * tr + 1.0;
        di = 2.0 * ti;
        z = cdd_sqr_add(z, c);
        if (i == la) { zl = z; dlr = dr; dli = di; }
    }
    if (l < 0) {
        zl = cdd_neg(zl);
        dlr = -dlr;
        dli = -dli;
    }
    const cdd P = cdd_sub(z, zl);
    const double pr = dr - dlr, pi = di - dli;
    const double d2 = pr * pr + pi * pi;
    // P conj(P') / |P'|^2
    const dd nr = dd_add(dd_mul_d(P.re, pr), dd_mul_d(P.im, pi));
    const dd ni = dd_sub(dd_mul_d(P.im, pr), dd_mul_d(P.re, pi));
    return {{dd_div_by(nr, d2), dd_div_by(ni, d2)}, d2};
}

// P(z) and P'(z) of the polynomial (l, N) of eval_q_t: P in double-double,
// P' in FP64.
__device__ void dd_eval(int l, int N, cdd c, cdd &P, cd &dP)
{
    const int la = l < 0 ? -l : l;
    cdd z = {{0.0, 0.0}, {0.0, 0.0}}, zl = z;
    double dr = 0.0, di = 0.0, dlr = 0.0, dli = 0.0;
    for (int i = 1; i <= N; ++i) {
        const double tr = z.re.hi * dr - z.im.hi * di, ti = z.re.hi * di + z.im.hi * dr;
        dr = 2.0 * tr + 1.0;
        di = 2.0 * ti;
        z = cdd_sqr_add(z, c);
        if (i == la) { zl = z; dlr = dr; dli = di; }
    }
    if (l < 0) {
        zl = cdd_neg(zl);
        dlr = -dlr;
        dli = -dli;
    }
    P = l ? cdd_sub(z, zl) : z;
    dP = {dr - dlr, di - dli};
}

// Start kg of the whole upper half of the level line (P = lambda_0 i^kg),
// lifted on its own in double-double like a seed (Section 4.2): from the
// circle |p_1| = lambda_0 at the start's own angle pi a / (S F) (a = its
// fine-point index) through every level p_2 .. p_N, the angle doubling at
// each level, Newton with target in log form; at the last level the target
// is the start's exact value lambda_0 i^kg and the point is polished to
// double-double accuracy by Newton on P - T.  Returns false when a level
// does not converge.
__device__ bool dd_lift_start(const plan_t &pl, int64_t kg, cdd &z)
{
    const bool real_end = kg == 0 || kg == 2 * pl.D;
    const int64_t Sp = pl.S * pl.F, twoSp = 2 * Sp; // fine points of the upper half
    const double lam = pl.level;
    int64_t a = (kg * pl.q) % twoSp;
    auto circle = [&](int64_t x) -> cd {
        double sn, cs;
        sincospi((double)x / (double)Sp, &sn, &cs);
        if (x == 0) return {lam, 0.0};
        if (x == Sp) return {-lam, 0.0};
        return {lam * cs, lam * sn};
    };
    const cd z0 = circle(a);
    z = {{z0.re, 0.0}, {z0.im, 0.0}};
    const int top = pl.el ? pl.eN + 1 : pl.eN;
    bool ok = true;
    for (int lev = 2; lev <= top && ok; ++lev) {
        int ll = 0, NN = lev;
        if (lev <= pl.eN) a = (2 * a) % twoSp;
        else { ll = pl.el; NN = pl.eN; }
        const cd T = circle(a);
        const bool last = lev == top;
        ok = false;
        for (int it = 0; it < 48; ++it) {
            cdd P;
            cd dP;
            dd_eval(ll, NN, z, P, dP);
            const cd Ph = {P.re.hi, P.im.hi};
            if (!cfinite(Ph) || !cfinite(dP)) break;
            const cd w = cdiv(T, Ph);
            const cd v = {w.re - 1.0, w.im};
            if (!last && cabs2(v) < 0x1p-10) { ok = true; break; }
            if (last && cabs2(v) < 0x1p-40) {
                // polish: Newton on P - T, the residual in double-double
                const cdd r = {dd_add_d(P.re, -T.re), dd_add_d(P.im, -T.im)};
                const double d2 = dP.re * dP.re + dP.im * dP.im;
                if (!(d2 > 0.0)) break;
                const dd nr = dd_add(dd_mul_d(r.re, dP.re), dd_mul_d(r.im, dP.im));
                const dd ni = dd_sub(dd_mul_d(r.im, dP.re), dd_mul_d(r.re, dP.im));
                const cdd st = {dd_div_by(nr, d2), dd_div_by(ni, d2)};
                z = cdd_sub(z, st);
                if (real_end) z.im = {0.0, 0.0};
                if (cdd_abs2_hi(st) <= 0x1p-200 * fmax(cdd_abs2_hi(z), 0x1p-16)) { ok = true; break; }
                continue;
            }
            const cd h = cmul(clog_near1(w), cdiv(Ph, dP));
            z.re = dd_add_d(z.re, h.re);
            z.im = dd_add_d(z.im, h.im);
            if (real_end) z.im = {0.0, 0.0};
        }
    }
    return ok;
}

// The descent's first Newton iterate from a lifted start (the same
// evaluation and division as the descent's own step).
__device__ __forceinline__ cd first_iterate(int l, int N, cd z)
{
    cd P, dP;
    eval_q(l, N, z, P, dP);
    return csub(z, cdiv_fast(P, dP));
}

// Starts at the left tip.  From order about 28 on the level line passes -2
// closer than the FP64 spacing there (its left end lies near
// -2 - 14.7 / 4^n): the fine points of the FP64 walk collapse onto the same
// values, the walk loses its way over the last segments (5 of them at order
// 30, 17 at order 31) and the starts it leaves there are not on the right
// branch of the level line.  Each of the last tip_starts starts is instead
// lifted on its own in double-double (dd_lift_start): the high part replaces
// the start, the low part goes to tip_lo (read by the double-double
// descent).  A start whose lift fails becomes NaN (its descent then ends as
// divergent) and is counted in C_SEED_FAIL.
__global__ void k_lift_tip_starts(batch_args b, cd *starts, cd *tip_lo, int64_t n_tip, cd *first)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tip) return;
    int t = 0; // type owning slot i (few types carry tip starts)
    while (t + 1 < b.T && b.types[t + 1].tip_lo_off <= i) ++t;
    const type_desc &td = b.types[t];
    const plan_t &pl = td.p;
    const int64_t j = i - td.tip_lo_off;
    if (j >= pl.tip_starts) return;
    const int64_t k = pl.NS - pl.tip_starts + j;    // start index within the item
    const int64_t kg = k + pl.seg0 * (pl.F / pl.q); // on the whole line: P = lambda_0 i^kg
    const int64_t g = td.start_off + k;
    cdd z;
    if (!dd_lift_start(pl, kg, z)) {
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        z = {{nan, 0.0}, {nan, 0.0}};
        atomicAdd(&wave_ctr(b)[(int64_t)t * C_NCOUNTERS + C_SEED_FAIL], 1ull);
    }
    starts[g] = {z.re.hi, z.im.hi};
    first[g] = first_iterate(pl.el, pl.eN, starts[g]);
    tip_lo[i] = {z.re.lo, z.im.lo};
}

// Segments whose FP64 walk failed its phase check (seg_flag != 0) to a list
// (global segment indices, count in G_FAILED_SEGS; one atomic per wave).
// A segment fails when one of its two walks failed, or when they end on the
// middle point more than a tenth of a Newton step apart (the phase check: a
// walk that changed turns lands about 2 pi |P/P'| away).  Failures are
// counted per type (C_PHASE_FAIL) and listed for k_relift_failed.
__global__ void k_failed_list(batch_args b, const uint8_t *item_flag, const walk_mid *mid, uint32_t *list)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (g < b.n_segs) {
        bad = item_flag[2 * g] != 0 || item_flag[2 * g + 1] != 0;
        if (!bad) {
            const walk_mid m = mid[g];
            bad = !(cabs2(csub(m.f, m.b)) < 1e-2 * m.s2);
        }
        if (bad) {
            const int t = find_type(b.seg_offs, b.T, g);
            atomicAdd(&wave_ctr(b)[(int64_t)t * C_NCOUNTERS + C_PHASE_FAIL], 1ull);
        }
    }
    wave_append(list, &b.gctr[G_FAILED_SEGS], bad, (uint32_t)g);
}

// The starts of a failed segment, lifted again one by one in double-double.
// A walk fails where consecutive fine points come closer than FP64 resolves
// -- next to -2 and next to the tips of M where the rays of dyadic angles
// land (angles k / 2^m: the failures of p_28 and p_29 cluster at 7/16,
// 15/32, 29/64, ...) -- or where a seed sits on another branch; the lift by
// angle does not depend on either.  Segment j's starts j F/q + 1 .. (j + 1)
// F/q (its walk's starts and the next seed) are replaced by the high parts
// of their lifts (the starts of the left tip have their own lift); a start
// whose lift fails keeps the walk's value.  One wave per failed segment.
__global__ void __launch_bounds__(64) k_relift_failed(batch_args b, const uint32_t *list, cd *starts, cd *first)
{
    const uint64_t n = b.gctr[G_FAILED_SEGS];
    for (uint64_t e = blockIdx.x; e < n; e += gridDim.x) {
        const uint32_t g = list[e];
        const int t = find_type(b.seg_offs, b.T, g);
        const type_desc &td = b.types[t];
        const plan_t &pl = td.p;
        const int64_t j = (int64_t)g - b.seg_offs[t];
        const int64_t per = pl.F / pl.q;
        for (int64_t u = threadIdx.x; u < per; u += blockDim.x) {
            const int64_t k = j * per + 1 + u;
            if (k >= pl.NS - pl.tip_starts) continue; // past the item, or a tip start
            cdd z;
            if (dd_lift_start(pl, k + pl.seg0 * per, z)) {
                const cd s = {z.re.hi, z.im.hi};
                starts[td.start_off + k] = s;
                first[td.start_off + k] = first_iterate(pl.el, pl.eN, s);
            } else {
                atomicAdd(&wave_ctr(b)[(int64_t)t * C_NCOUNTERS + C_SEED_FAIL], 1ull);
            }
        }
    }
}

// Routing: starts whose FP64 descent ended within x_tip of -2 (any status:
// a descent the FP64 rounding derailed there is retried; k_descend sets
// tip[g] within the call's largest radius, and the root is read and tested
// against its type's radius only there), and descents that stalled at the
// FP64 precision floor anywhere, go to a list (in no particular order: the
// double-double descent takes them from a queue).  At high order they are
// many and scattered, and one atomic per wave on the list's length
// serialised the pass, so each block gathers them in LDS, ROUTE_ITEMS starts
// per round (each thread's status and flag bytes in one 8-byte load each),
// and appends its buffer to the list with one atomic when it fills.
// Grid-stride over rounds of ROUTE_ITEMS starts.
constexpr int ROUTE_PER = 8;
constexpr int ROUTE_ITEMS = 256 * ROUTE_PER;
constexpr int ROUTE_BUF = 2 * ROUTE_ITEMS;

__global__ void __launch_bounds__(256) k_route_tip(batch_args b, const cd *roots, const uint8_t *status,
                                                   const uint8_t *tip, uint32_t *list)
{
    __shared__ int64_t offs[MAX_TYPES + 1];
    __shared__ double xt[MAX_TYPES];
    __shared__ uint32_t buf[ROUTE_BUF];
    __shared__ uint32_t nbuf;
    __shared__ unsigned long long base;
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) {
        offs[i] = b.start_offs[i];
        if (i < b.T) xt[i] = b.types[i].p.x_tip;
    }
    if (threadIdx.x == 0) nbuf = 0;
    __syncthreads();
    // the buffer to the list (every thread, c read by all after a barrier)
    auto flush = [&](uint32_t c) {
        if (threadIdx.x == 0) base = atomicAdd(&b.gctr[G_DD_COUNT], (unsigned long long)c);
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < c; j += blockDim.x) list[base + j] = buf[j];
        __syncthreads();
        if (threadIdx.x == 0) nbuf = 0;
        __syncthreads();
    };
    const int lane = threadIdx.x & 63;
    for (int64_t r0 = (int64_t)blockIdx.x * ROUTE_ITEMS; r0 < b.n_starts; r0 += (int64_t)gridDim.x * ROUTE_ITEMS) {
        // ROUTE_PER consecutive starts per thread, their status and tip bytes
        // in one 8-byte load each where the round is whole (r0 and the
        // workspace arrays are 8-byte aligned)
        const int64_t g0 = r0 + (int64_t)threadIdx.x * ROUTE_PER;
        uint8_t st[ROUTE_PER], tp[ROUTE_PER];
        if (g0 + ROUTE_PER <= b.n_starts) {
            const uint64_t s8 = *(const uint64_t *)(status + g0), t8 = *(const uint64_t *)(tip + g0);
#pragma unroll
            for (int k = 0; k < ROUTE_PER; ++k) {
                st[k] = (uint8_t)(s8 >> (8 * k));
                tp[k] = (uint8_t)(t8 >> (8 * k));
            }
        } else {
#pragma unroll
            for (int k = 0; k < ROUTE_PER; ++k) {
                st[k] = g0 + k < b.n_starts ? status[g0 + k] : ST_NONE;
                tp[k] = g0 + k < b.n_starts ? tip[g0 + k] : 0;
            }
        }
        const int t = g0 < b.n_starts ? find_type_lds(offs, b.T, g0) : 0;
        const int64_t t_end = offs[t + 1]; // a type boundary inside the thread's starts: search again
#pragma unroll
        for (int k = 0; k < ROUTE_PER; ++k) {
            const int64_t g = g0 + k;
            bool take = false;
            if (st[k] != ST_NONE) {
                const int tk = g < t_end ? t : find_type_lds(offs, b.T, g);
                const double x = xt[tk];
                if (st[k] == ST_STALL) {
                    take = true;
                } else if (x > 0.0 && tp[k] != 0) {
                    const cd z = roots[g];
                    take = fabs(z.re + 2.0) < x && fabs(z.im) < x;
                }
            }
            const uint64_t mask = __ballot(take);
            if (!mask) continue;
            const int leader = __ffsll((unsigned long long)mask) - 1;
            uint32_t wbase = 0;
            if (lane == leader) wbase = atomicAdd(&nbuf, (uint32_t)__popcll(mask));
            wbase = __shfl(wbase, leader, 64);
            if (take) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                buf[wbase + rank] = (uint32_t)g;
            }
        }
        __syncthreads();
        const uint32_t c = nbuf; // the same in every thread: nothing changes it before the next barrier
        __syncthreads();
        if (c > (uint32_t)(ROUTE_BUF - ROUTE_ITEMS)) flush(c);
    }
    __syncthreads();
    const uint32_t c = nbuf;
    __syncthreads();
    if (c) flush(c);
}

// Double-double Newton descent of the routed starts, from their starting
// points: same outcome rules as the FP64 descent (Algorithm S_par),
// converged when a step falls below 2^-98 max(|z|, 2^-8).  Next to two
// roots at distance s, Newton from distance d >> s contracts only by one half
// per step (the pair acts like a double root), so reaching a pair 1e-20
// apart from 1e-2 takes about 60 steps, against about 12 on average: the cap
// is DD_CAP, and the lanes take the routed starts from a per-wave work queue
// (as the FP64 descent), so that a lane whose descent ends takes the next
// start instead of idling until the slowest lane of its wave finishes.
// Work list length read on the device.
constexpr int DD_CAP = 256;

// primary: every descent of the call runs here (MSPLIT_DD), and the outcomes
// are counted as the FP64 descent counts them (converged, diverged, time-outs)
// instead of as routed starts.
__global__ void __launch_bounds__(256) k_descend_dd(batch_args b, const uint32_t *list, const cd *starts,
                                                    const cd *tip_lo, cd *roots, cd *roots_lo, uint8_t *status,
                                                    int primary)
{
    constexpr int64_t NONE = -1;
    unsigned long long *const wc = wave_ctr(b);
    const uint64_t n = b.gctr[G_DD_COUNT];
    // per-lane counts of type ct: double-double steps, then routed starts, or
    // (primary) converged, diverged and timed-out descents
    int ct = -1;
    uint32_t cnt[4] = {0u, 0u, 0u, 0u};
    const int slots[4] = {C_STEPS_DD, primary ? C_CONVERGED : C_DD_ROUTED, primary ? C_DIVERGED : C_STEPS_DD,
                          primary ? C_TIMEOUT : C_STEPS_DD};
    int64_t g = NONE;
    bool exhausted = false;
    int t = -1, el = 0, eN = 1, it = 0, cap = DD_CAP;
    bool fin = false;
    double prev = 0.0;
    cdd z = {{0.0, 0.0}, {0.0, 0.0}};
    wave_queue wq = wave_queue_start(64);
    while (true) {
        const bool need = !exhausted && g == NONE;
        const uint64_t got = __ballot(need) ? wave_take(wq, &b.gctr[G_DD_NEXT], 64, n, need) : ~0ull;
        if (need) {
            if (got >= n) {
                exhausted = true;
            } else {
                g = (int64_t)list[got];
                t = find_type(b.start_offs, b.T, g);
                const type_desc &td = b.types[t];
                el = td.p.el;
                eN = td.p.eN;
                // the routed descents near -2 need up to about 60 steps; as
                // the primary descent, the type's own cap unless it has a tip
                cap = primary && td.p.x_tip <= 0.0 ? td.p.cap : DD_CAP;
                const cd s0 = starts[g];
                z = {{s0.re, 0.0}, {s0.im, 0.0}};
                const int64_t k = g - td.start_off;
                if (k >= td.p.NS - td.p.tip_starts) { // a start lifted in double-double
                    const cd lo = tip_lo[td.tip_lo_off + (k - (td.p.NS - td.p.tip_starts))];
                    z.re.lo = lo.re;
                    z.im.lo = lo.im;
                }
                it = 0;
                fin = false;
                prev = 0.0;
            }
        }
        const bool change = g != NONE && t != ct;
        if (__ballot(change)) {
            wave_add4_by_key(wc, C_NCOUNTERS, ct, slots, cnt);
            cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0u;
            if (change) ct = t;
        }
        if (__ballot(g != NONE || !exhausted) == 0) break;
        if (g == NONE) continue;
        if (!primary) cnt[1] += it == 0;
        const dd_step r = dd_newton_step(el, eN, z);
        ++it;
        cnt[0] += 1u;
        z = cdd_sub(z, r.s);
        const double a2 = cdd_abs2_hi(r.s), az2 = cdd_abs2_hi(z);
        uint8_t st = ST_NONE;
        if (fin) {
            st = ST_DD;
        } else if (!(a2 <= 0x1p1000) || !(az2 <= 64.0) || !(r.d2 > 0.0) || (it > 3 && a2 > 64.0 * prev)) {
            st = ST_DIVERGED;
        } else if (a2 <= 0x1p-196 * fmax(az2, 0x1p-16)) {
            // final at once when the next step predicted by quadratic
            // convergence, |d|^3 / |d_prev|^2, is below the double-double
            // rounding, else after one more step
            if (a2 * a2 * a2 <= 0x1p-212 * fmax(az2, 0x1p-16) * prev * prev) st = ST_DD;
            else fin = true;
        } else if (it >= cap) {
            st = ST_TIMEOUT;
        }
        prev = a2;
        if (st != ST_NONE) {
            roots[g] = {z.re.hi, z.im.hi};
            roots_lo[g] = {z.re.lo, z.im.lo};
            status[g] = st;
            if (primary) {
                cnt[1] += st == ST_DD;
                cnt[2] += st == ST_DIVERGED;
                cnt[3] += st == ST_TIMEOUT;
            }
            g = NONE;
        }
    }
    wave_add4_by_key(wc, C_NCOUNTERS, ct, slots, cnt);
}

// MSPLIT_DD: every start to the double-double descent's list.
__global__ void k_list_all(batch_args b, uint32_t *list)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < b.n_starts) list[g] = (uint32_t)g;
    if (g == 0) b.gctr[G_DD_COUNT] = (unsigned long long)b.n_starts;
}

} // namespace msplit
