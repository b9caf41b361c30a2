// kernels.hpp -- the hot path of the level-line splitter on gfx950.
//
// One pass over a polynomial P = q_{l,n} (l = 0: p_n) of degree D = 2^(N-1),
// N = l + n, in the closed upper half plane (Section 6.1):
//
//   k_seeds   seed lift      S+1 seeds of Phi-angle pi j / S lifted from the
//                            circle |p_1| = lambda_0 through p_2 .. p_N
//                            (Section 4.2, lifting p_k -> p_{k+1})
//   k_walk    level line     each lane walks F fine points of one segment,
//                            value phase 2 pi s / M (Prop. computeLevelLine),
//                            every (M/4)-th point is a start (Thm practicalFTA)
//   k_descend Newton descent one lane per start, capped (Algorithm S_par)
//   k_keys .. k_scatter      nset collection (Section 6.1)
//   k_classify               exact period / Misiurewicz type (eq. def:hyp,
//                            eq. def:mis)
//   k_certify, k_separation  Thm proofRoots + Thm diskArithmetic, Thm certif
//
// Work distribution: k_walk and k_descend are persistent; each lane pulls
// its next item from a global counter with one wave-aggregated atomic, so
// lanes whose Newton iterations end early do not wait for the slowest lane of
// their wave (the divergence the paper names as its objection to GPUs).
#pragma once
#include "common.hpp"

namespace msplit {

// status of a descent
enum : uint8_t { ST_NONE = 0, ST_CONVERGED = 1, ST_DIVERGED = 2, ST_TIMEOUT = 3 };

// device counters (uint64 slots of the workspace)
enum {
    C_SEG_NEXT = 0, C_START_NEXT, C_CONVERGED, C_DIVERGED, C_TIMEOUT, C_PHASE_FAIL,
    C_STEPS_LIFT, C_STEPS_WALK, C_STEPS_DESC, C_STEPS_FP32, C_UNIQUE, C_REAL,
    C_CERTIFIED, C_LABEL, C_OVERLAP, C_MIN_SEP_BITS, C_MAX_RAD_BITS, C_SEED_FAIL,
    C_DISCARD, C_NCOUNTERS = 32
};

struct plan_t {
    int l, n, N;          // type and order N = l + n
    int M;                // fine points per turn
    int q;                // M / 4: fine points between starts
    int cap;              // Newton cap
    int64_t D;            // degree 2^(N-1)
    int64_t F;            // fine points per segment
    int64_t S;            // segments in the upper half plane
    int64_t NS;           // starts: 2 D + 1
    double level;         // lambda_0
    double tau;           // nset identification radius
    double tol_desc;      // relative step of a converged descent
    uint32_t divmask_lo;  // bit k set when k | n, k < n (k < 32)
    int precision;
    float fp32_switch;
    uint32_t chunk_seg;   // work-queue chunk of the walk (segments)
    uint32_t chunk_start; // work-queue chunk of the descents (starts)
};

// cis(2 pi s / M) for s = 0..M-1, M <= 64, set by the host
__constant__ double c_cis_re[64];
__constant__ double c_cis_im[64];

// ------------------------------------------------------------ seed lift
// Lane j lifts the point of Phi-angle pi j / S: on p_1 = z the level line is
// the circle |z| = lambda_0, so the seed starts at lambda_0 e^{i pi j / S}.
// At p_k its value must be lambda_0 e^{i pi a_k / S} with a_k = 2^(k-1) j mod
// 2S (the value phase doubles from p_k to p_{k+1} because p_{k+1} = p_k^2 + c
// and |c| << lambda_0^2).  Each level is solved with the Newton method on
// log P (log P(z) = log T), whose step z += log(T/P) P/P' is the discrete
// level-line / iso-angle flow of Section 4.1.
__global__ void k_seeds(plan_t pl, cd *seeds, cd *starts, unsigned long long *ctr)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long steps = 0, fail = 0;
    if (j <= pl.S) {
        const int64_t twoS = 2 * pl.S;
        double sn, cs;
        sincospi((double)j / (double)pl.S, &sn, &cs);
        cd z = {pl.level * cs, pl.level * sn};
        if (j == pl.S) z = {-pl.level, 0.0};
        if (j == 0) z = {pl.level, 0.0};
        int64_t a = j % twoS;
        const int top = pl.l ? pl.N + 1 : pl.N; // extra stage: onto q_{l,n}
        for (int k = 2; k <= top && !fail; ++k) {
            int ll = 0, NN = k;
            if (k <= pl.N) a = (2 * a) % twoS;
            else { ll = pl.l; NN = pl.N; }
            sincospi((double)a / (double)pl.S, &sn, &cs);
            cd T = {pl.level * cs, pl.level * sn};
            if (a == 0) T = {pl.level, 0.0};
            int it = 0;
            for (;; ++it) {
                cd P, dP;
                eval_q(ll, NN, z, P, dP);
                ++steps;
                cd w = cdiv(T, P);
                cd v = {w.re - 1.0, w.im};
                if (cabs2(v) < 1e-26) break;
                if (it >= 40 || !cfinite(P)) { fail = 1; break; }
                cd h = cmul(clog_near1(w), cdiv(P, dP));
                // near the tip of M the value carries ~4^N u of rounding noise;
                // stop once the update itself is at rounding level
                if (cabs2(h) <= 0x1p-96 * fmax(cabs2(z), 0x1p-16)) break;
                z = cadd(z, h);
                if (j == 0 || j == pl.S) z.im = 0.0; // the two real end points stay real
            }
        }
        seeds[j] = z;
        starts[j * (pl.F / pl.q)] = z;
    }
    wave_add(&ctr[C_STEPS_LIFT], steps);
    wave_add(&ctr[C_SEED_FAIL], fail);
}

// --------------------------------------------------------- level-line walk
// Lane state machine: each loop trip is one evaluation of P, P' followed by
// one Newton-on-log-P update, so lanes never wait for each other inside a
// segment.  Fine point s targets T_s = lambda_0 e^{2 i pi s / M}; the step
// towards it is Newton on log P, z += log(T_s / P) P / P' (an Euler step of
// the level-line flow lambda' = i P / P' of Section 4.1 with its correction).
__global__ void k_walk(plan_t pl, const cd *seeds, cd *starts, uint8_t *seg_flag,
                       unsigned long long *ctr)
{
    // a fine point (start or not) is accepted at |T/P - 1| < 2^-5 or when the
    // update is at rounding level: it only has to lie in the Newton basin of
    // the next target, and the next target is aimed from the actual value
    const double tol2 = 0x1p-10;
    const double dphi = 2.0 * M_PI / pl.M;
    unsigned long long steps = 0, pfail = 0;
    int64_t j = -1;        // current segment
    int64_t s = 0, send = 0;
    int it = 0;
    cd z = {0.0, 0.0};
    bool done = false;
    wave_queue wq = {0, 0};
    while (true) {
        bool need = !done && j < 0;
        uint64_t got = wave_take(wq, &ctr[C_SEG_NEXT], pl.chunk_seg, need);
        if (need) {
            if (got >= (uint64_t)pl.S) done = true;
            else { j = (int64_t)got; z = seeds[j]; s = j * pl.F + 1; send = j * pl.F + pl.F; it = 0; }
        }
        if (__ballot(!done) == 0) break;
        if (done) continue;
        cd P, dP;
        eval_q(pl.l, pl.N, z, P, dP);
        ++steps;
        int r = (int)(s % pl.M);
        cd T = {pl.level * c_cis_re[r], pl.level * c_cis_im[r]};
        cd w = cdiv(T, P);
        cd v = {w.re - 1.0, w.im};
        bool is_start = (s % pl.q) == 0;
        double a2 = cabs2(v);
        cd step = cdiv(P, dP);
        if (!cfinite(w) || !cfinite(step) || it > 24) {
            seg_flag[j] = 2;
            ++pfail;
            j = -1;
            continue;
        }
        cd u0 = clog_near1(w);
        cd h = cmul(u0, step);
        if (a2 < tol2 || cabs2(h) <= 0x1p-96 * fmax(cabs2(z), 0x1p-16)) {
            if (s == send) {
                // the walk must end on the next seed (phase check): a skipped
                // turn would land about 2 pi |P/P'| away
                cd e = csub(z, seeds[j + 1]);
                bool ok = cabs2(e) < 1e-2 * cabs2(step);
                seg_flag[j] = ok ? 0 : 1;
                pfail += !ok;
                j = -1;
                continue;
            }
            if (is_start) starts[s / pl.q] = z;
            // aim at the next fine point: log(T_{s+1}/P) = i dphi + log(T_s/P)
            ++s;
            it = 0;
            u0.im += dphi;
            z = cadd(z, cmul(u0, step));
        } else {
            ++it;
            z = cadd(z, h);
        }
    }
    wave_add(&ctr[C_STEPS_WALK], steps);
    wave_add(&ctr[C_PHASE_FAIL], pfail);
}

// ---------------------------------------------------------- Newton descent
// One lane per start, Newton map N_P (eq. Newton), cap max{20, I_N log d}
// (Algorithm S_par).  Discarded as divergent: non-finite, |z| > 8 (far from
// M, which lies in D(0,2) u {-2}), or a long-distance jump (step more than 8
// times the previous one after the third step, Section 6.4.3).  Converged
// when the step falls below tol * max(|z|, 2^-8); one more step is taken.
// MIXED precision: the descent starts in FP32 and a lane moves to FP64 once
// its FP32 step is below fp32_switch * |z| (or FP32 stalls / overflows).
__global__ void k_descend(plan_t pl, cd *roots, uint8_t *status, unsigned long long *ctr)
{
    unsigned long long steps = 0, steps32 = 0, nconv = 0, ndiv = 0, ntime = 0;
    int64_t k = -1;
    cd z = {0.0, 0.0};
    double prev = 0.0; // previous step (FP32: length; FP64: squared length)
    int it = 0;
    bool fin = false, done = false, f32 = false;
    const bool mixed = pl.precision == 1;
    const double tol2 = pl.tol_desc * pl.tol_desc;
    wave_queue wq = {0, 0};
    while (true) {
        bool need = !done && k < 0;
        uint64_t got = wave_take(wq, &ctr[C_START_NEXT], pl.chunk_start, need);
        if (need) {
            if (got >= (uint64_t)pl.NS) done = true;
            else { k = (int64_t)got; z = roots[k]; it = 0; prev = 0.0; fin = false; f32 = mixed; }
        }
        if (__ballot(!done) == 0) break;
        if (done) continue;
        uint8_t st = ST_NONE;
        if (f32) {
            cf c = {(float)z.re, (float)z.im}, P, dP;
            eval_q_f32(pl.l, pl.N, c, P, dP);
            ++steps32;
            float den = dP.re * dP.re + dP.im * dP.im;
            float sr = (P.re * dP.re + P.im * dP.im) / den;
            float si = (P.im * dP.re - P.re * dP.im) / den;
            float a = sqrtf(sr * sr + si * si);
            float ac = sqrtf(c.re * c.re + c.im * c.im);
            if (!isfinite(a) || !(den > 0.f) || a <= pl.fp32_switch * fmaxf(ac, 0.00390625f)) {
                // FP32 is done (or cannot resolve this point): FP64 takes
                // over from the current point without this step
                f32 = false;
                prev = prev * prev;
            } else {
                float zr = c.re - sr, zi = c.im - si;
                ++it;
                z = {(double)zr, (double)zi};
                float az = sqrtf(zr * zr + zi * zi);
                if (!isfinite(zr) || !isfinite(zi) || az > 8.f) st = ST_DIVERGED;
                else if (it > 3 && a > 8.f * (float)prev) st = ST_DIVERGED;
                else if (it >= pl.cap) st = ST_TIMEOUT;
                prev = a;
            }
        } else {
            cd P, dP;
            eval_q(pl.l, pl.N, z, P, dP);
            ++steps;
            cd d = cdiv(P, dP);
            z = csub(z, d);
            ++it;
            // squared lengths: |d|, |z| compared without square roots
            double a2 = cabs2(d);
            double az2 = cabs2(z);
            if (fin) st = ST_CONVERGED;
            else if (!isfinite(a2) || !cfinite(z) || az2 > 64.0) st = ST_DIVERGED;
            else if (it > 3 && a2 > 64.0 * prev) st = ST_DIVERGED;
            else if (a2 <= tol2 * fmax(az2, 0x1p-16)) fin = true;
            else if (it >= pl.cap) st = ST_TIMEOUT;
            prev = a2;
        }
        if (st != ST_NONE) {
            roots[k] = z;
            status[k] = st;
            nconv += st == ST_CONVERGED;
            ndiv += st == ST_DIVERGED;
            ntime += st == ST_TIMEOUT;
            k = -1;
        }
    }
    wave_add(&ctr[C_STEPS_DESC], steps);
    wave_add(&ctr[C_STEPS_FP32], steps32);
    wave_add(&ctr[C_CONVERGED], nconv);
    wave_add(&ctr[C_DIVERGED], ndiv);
    wave_add(&ctr[C_TIMEOUT], ntime);
}

// -------------------------------------------------------- nset collection
// Fold to the closed upper half plane, snap |Im| < tau/2 to the real axis,
// key by the real part (order-preserving uint64); non-converged go last.
__global__ void k_keys(plan_t pl, cd *roots, const uint8_t *status, uint64_t *keys, uint32_t *vals)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= pl.NS) return;
    uint64_t key = ~0ull;
    if (status[k] == ST_CONVERGED) {
        cd z = roots[k];
        z.im = fabs(z.im);
        if (z.im < 0.5 * pl.tau) z.im = 0.0;
        roots[k] = z;
        key = orderable(z.re);
    }
    keys[k] = key;
    vals[k] = (uint32_t)k;
}

// A sorted point is a duplicate when an earlier point lies within tau in both
// coordinates (the nset identification, the first point of a cluster kept).
__global__ void k_mark(plan_t pl, const cd *roots, const uint64_t *keys, const uint32_t *vals,
                       uint32_t *flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pl.NS) return;
    uint32_t f = 0;
    if (keys[i] != ~0ull) {
        cd zi = roots[vals[i]];
        f = 1;
        for (int64_t j = i - 1, c = 0; j >= 0 && c < 256; --j, ++c) {
            cd zj = roots[vals[j]];
            if (zi.re - zj.re >= pl.tau) break;
            if (fabs(zi.im - zj.im) < pl.tau) { f = 0; break; }
        }
    }
    flag[i] = f;
}

__global__ void k_scatter(plan_t pl, const cd *roots, const uint32_t *vals, const uint32_t *flag,
                          const uint32_t *pos, double *ore, double *oim, uint64_t capacity,
                          unsigned long long *ctr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nreal = 0;
    if (i < pl.NS) {
        if (flag[i]) {
            uint64_t p = pos[i];
            cd z = roots[vals[i]];
            if (p < capacity) { ore[p] = z.re; oim[p] = z.im; }
            nreal += z.im == 0.0;
        }
        if (i == pl.NS - 1) ctr[C_UNIQUE] = (unsigned long long)pos[i] + flag[i];
    }
    wave_add(&ctr[C_REAL], nreal);
}

// ---------------------------------------------------------- classification
// p_n: exact period = least k | n with p_k(root) = 0 (eq. def:hyp), tested by
// the Newton distance |p_k / p_k'| < tau.  tau is the identification radius,
// far below the least distance between roots of p_n (118.4 / 4^n, Section
// 6.3.2): a root of period n can sit that close to a root of period n/2 (the
// centre of a satellite next to its parent), so the scale of p_k alone would
// not do.  One orbit pass serves all divisors.
__global__ void k_classify(plan_t pl, const double *re, const double *im, int32_t *period,
                           int32_t *preperiod, uint8_t *flags, uint64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)count) return;
    cd c = {re[i], im[i]};
    int per = pl.n;
    if (pl.l == 0 && period) {
        orbit_state<double> s = {0.0, 0.0, 0.0, 0.0};
        const double thr = pl.tau;
        for (int k = 1; k < pl.n; ++k) {
            orbit_step(s, c.re, c.im);
            if (((pl.divmask_lo >> k) & 1u) && per == pl.n) {
                double a2 = s.zr * s.zr + s.zi * s.zi;
                double d2 = s.dr * s.dr + s.di * s.di;
                if (a2 < thr * thr * d2) per = k;
            }
        }
    }
    if (period) period[i] = per;
    if (preperiod) preperiod[i] = pl.l;
    if (flags) flags[i] = (im[i] == 0.0) ? 1 : 0;
}

} // namespace msplit
