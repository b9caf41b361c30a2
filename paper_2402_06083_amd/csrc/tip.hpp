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
    cdd z = {{0.0, 0.0}, {0.0, 0.0}}, zl = z;
    double dr = 0.0, di = 0.0, dlr = 0.0, dli = 0.0;
    for (int i = 1; i <= N; ++i) {
        const double tr = z.re.hi * dr - z.im.hi * di, ti = z.re.hi * di + z.im.hi * dr;
        dr = 2.0 * tr + 1.0;
        di = 2.0 * ti;
        z = cdd_sqr_add(z, c);
        if (i == l) { zl = z; dlr = dr; dli = di; }
    }
    const cdd P = cdd_sub(z, zl);
    const double pr = dr - dlr, pi = di - dli;
    const double d2 = pr * pr + pi * pi;
    // P conj(P') / |P'|^2
    const dd nr = dd_add(dd_mul_d(P.re, pr), dd_mul_d(P.im, pi));
    const dd ni = dd_sub(dd_mul_d(P.im, pr), dd_mul_d(P.re, pi));
    return {{dd_div_by(nr, d2), dd_div_by(ni, d2)}, d2};
}

// Routing: starts whose FP64 descent ended within x_tip of -2 (any status:
// a descent the FP64 rounding derailed there is retried) go to a list; one
// atomic per wave.
__global__ void k_route_tip(batch_args b, const cd *roots, const uint8_t *status, uint32_t *list)
{
    __shared__ int64_t offs[MAX_TYPES + 1];
    __shared__ double xt[MAX_TYPES];
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) {
        offs[i] = b.start_offs[i];
        if (i < b.T) xt[i] = b.types[i].p.x_tip;
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool take = false;
    if (g < b.n_starts && status[g] != ST_NONE) {
        const int t = find_type_lds(offs, b.T, g);
        const cd z = roots[g];
        const double x = xt[t];
        take = x > 0.0 && fabs(z.re + 2.0) < x && fabs(z.im) < x;
    }
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int leader = __ffsll(mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(&b.gctr[G_DD_COUNT], (unsigned long long)__popcll(mask));
    base = read_lane_u64(base, leader);
    if (take) {
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        list[base + rank] = (uint32_t)g;
    }
}

// Double-double Newton descent of the routed starts, from their starting
// points: same outcome rules as the FP64 descent (Algorithm S_par), converged
// when the step falls below 2^-98 max(|z|, 2^-8), then one more step.  Next
// to two roots at distance s, Newton from distance d >> s contracts only by
// one half per step (the pair acts like a double root), so reaching a pair
// 1e-20 apart from 1e-2 takes about 60 steps: the cap is DD_CAP, which the
// few routed starts make cheap.  Work list length read on the device.
constexpr int DD_CAP = 256;

__global__ void __launch_bounds__(256) k_descend_dd(batch_args b, const uint32_t *list, const cd *starts, cd *roots,
                                                    cd *roots_lo, uint8_t *status)
{
    unsigned long long *const wc = wave_ctr(b);
    const uint64_t n = b.gctr[G_DD_COUNT];
    type_count steps, routed;
    type_cache tc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < (int64_t)n; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        const int64_t g = i < (int64_t)n ? (int64_t)list[i] : -1;
        const int t = g >= 0 ? cached_type(tc, b.start_offs, b.T, g) : steps.t;
        if (__ballot(g >= 0 && t != steps.t)) {
            flush_count(wc, C_STEPS_DD, steps);
            flush_count(wc, C_DD_ROUTED, routed);
        }
        steps.t = routed.t = t;
        if (g < 0) continue;
        routed.v += 1;
        const plan_t &pl = b.types[t].p;
        const cd s0 = starts[g];
        cdd z = {{s0.re, 0.0}, {s0.im, 0.0}};
        const int cap = DD_CAP;
        double prev = 0.0;
        bool fin = false;
        uint8_t st = ST_TIMEOUT;
        for (int it = 1; it <= cap + 1; ++it) {
            const dd_step r = dd_newton_step(pl.l, pl.N, z);
            ++steps.v;
            z = cdd_sub(z, r.s);
            const double a2 = cdd_abs2_hi(r.s), az2 = cdd_abs2_hi(z);
            if (fin) { st = ST_DD; break; }
            if (!(a2 <= 0x1p1000) || !(az2 <= 64.0) || !(r.d2 > 0.0) || (it > 3 && a2 > 64.0 * prev)) {
                st = ST_DIVERGED;
                break;
            }
            if (a2 <= 0x1p-196 * fmax(az2, 0x1p-16)) fin = true;
            else if (it >= cap) break;
            prev = a2;
        }
        roots[g] = {z.re.hi, z.im.hi};
        roots_lo[g] = {z.re.lo, z.im.lo};
        status[g] = st;
    }
    flush_count(wc, C_STEPS_DD, steps);
    flush_count(wc, C_DD_ROUTED, routed);
}

} // namespace msplit
