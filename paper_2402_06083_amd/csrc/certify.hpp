// certify.hpp -- disk-arithmetic certificate of the roots on gfx950.
//
// Thm proofRoots: if f'(D(z0,R)) lies in a disk B' and R dist(0,B') > |f(z0)|,
// exactly one root of f lies in D(z0,R).  The enclosures come from the disk
// arithmetic of Thm diskArithmetic applied to the critical orbit
//   z_{k+1} = z_k^2 + c,  dz_{k+1} = 2 z_k dz_k + 1,  c in D(c0, R):
//   D(a,ra) + D(b,rb)  in D(a (+) b, ra + rb + ulp(a (+) b)/2)
//   D(a,ra) x D(b,rb)  in D(a (x) b, ra rb + ra|b| + rb|a| + R*),
//   R* = ulp(a (x) b)/2 + sum over the four real products u v of ulp(u v)/2,
// with ulp(x + iy) bounded by ulp(x) + ulp(y).  Centres are computed with
// separate IEEE multiplications and additions (no fused multiply-add), so the
// R* bound applies to each of them.  The GPU rounds to nearest only, so every radius
// expression is evaluated in round-to-nearest and then inflated by
// (1 + 2^-47) plus 2^-1000: each radius update is at most a few dozen
// operations, each off by at most 2^-53 relative (subnormal results by
// 2^-1075 absolute), which the inflation dominates.  This is a hardware-
// rounding certificate: it trusts the FP64 unit to round to nearest.
//
// Labels on the same disk: for p_n, a root of period k (k | n) is also a root
// of p_k -- Thm proofRoots is applied to p_k on the same disk -- and p_j has
// no zero on the disk for every strict divisor j of k (|p_j(D)| excludes 0).
// For q_{l,n} (Mis(l,n), eq. def:mis): q_{l-1,n} and q_{l,k} for every strict
// divisor k of n have no zero on the disk.
#pragma once
#include "common.hpp"
#include "kernels.hpp"
#include "tip.hpp"

namespace msplit {

// Contraction is switched off (DD_EXACT) wherever a rounding bound counts
// one rounding per written operation: the centres of the disks (explicit
// round-to-nearest operations) and the bounds below.  The radius recurrences
// of disk_orbit_step may fuse: they are sums of non-negative products, each
// inflated by up(), and a fused multiply-add rounds once where the separate
// operations round twice, so the inflation still covers the rounding.
//
// Rounding bound used below: a double r^ = fl(r) rounded to nearest obeys
// |r^ - r| <= ulp(r^)/2 <= u |r^| + eta with u = 2^-53 (normal results) and
// eta = 2^-1074 (covers a subnormal result), so the R* term of Thm
// diskArithmetic is bounded by u times the sum of the magnitudes of the
// rounded intermediate results, plus eta per operation.
constexpr double U53 = 0x1p-53;
constexpr double ETA = 0x1p-1074;

// x (1 + 2^-47) + 2^-1000: upper bound of a radius expression of at most a
// few dozen non-negative round-to-nearest operations
__device__ __forceinline__ double up(double x) { DD_EXACT return __dadd_rn(__dmul_rn(x, 1.0 + 0x1p-47), 0x1p-1000); }
__device__ __forceinline__ double dn(double x) { DD_EXACT return __dsub_rn(__dmul_rn(x, 1.0 - 0x1p-47), 0x1p-1000); }
// upper bound of |a|: sqrt(M^2 + m^2) <= M + m^2 / (2M) <= M + m / 2 for
// M = max(|re|, |im|) >= m = min(|re|, |im|) (at most 6% above |a|), written
// M + m / 2 = 3/4 (x + y) + 1/4 |x - y| (x = |re|, y = |im|: no max or min);
// its four roundings are covered by up()
__device__ __forceinline__ double abs_up(cd a)
{ DD_EXACT
    const double x = fabs(a.re), y = fabs(a.im);
    return up(__dadd_rn(__dmul_rn(0.75, __dadd_rn(x, y)), __dmul_rn(0.25, fabs(__dsub_rn(x, y)))));
}
// lower bound of |a|^2
__device__ __forceinline__ double abs2_dn(cd a)
{ DD_EXACT
    return dn(__dadd_rn(__dmul_rn(a.re, a.re), __dmul_rn(a.im, a.im)));
}
// bound of the rounding of a complex result a^ (both components)
__device__ __forceinline__ double rnd(cd a) { DD_EXACT return U53 * (fabs(a.re) + fabs(a.im)) + 2.0 * ETA; }

struct disk_step {
    cd Z, DZ;        // centres
    double e;        // radius of z_k at the exact point c0 (no radius on c)
    double rho, sig; // radii of z_k and dz_k over D(c0, R)
};

// One step of the orbit over disks: z <- z^2 + c, dz <- 2 z dz + 1, the centres
// computed with separate IEEE products and sums (no fused multiply-add); the
// radii (non-negative, inflated by up()) may use fused operations.
__device__ __forceinline__ void disk_orbit_step(disk_step &s, cd c, double R)
{
    const double x = s.Z.re, y = s.Z.im, u = s.DZ.re, v = s.DZ.im;
    const double xx = __dmul_rn(x, x), yy = __dmul_rn(y, y), xy = __dmul_rn(x, y);
    const cd sq = {__dsub_rn(xx, yy), __dadd_rn(xy, xy)}; // doubling is exact
    const cd Z1 = {__dadd_rn(sq.re, c.re), __dadd_rn(sq.im, c.im)};
    // rounding of the centre Z^2 + c: three products, one difference, two sums
    const double Rsq = U53 * (fabs(xx) + fabs(yy) + 2.0 * fabs(xy) + fabs(sq.re)) + rnd(Z1) + 6.0 * ETA;
    const double xu = __dmul_rn(x, u), yv = __dmul_rn(y, v), xv = __dmul_rn(x, v), yu = __dmul_rn(y, u);
    const cd pr = {__dsub_rn(xu, yv), __dadd_rn(xv, yu)};
    const cd DZ1 = {__dadd_rn(__dadd_rn(pr.re, pr.re), 1.0), __dadd_rn(pr.im, pr.im)};
    // rounding of 2 Z DZ + 1: four products and two sums (doubled), one sum
    const double Rpr = 2.0 * (U53 * (fabs(xu) + fabs(yv) + fabs(xv) + fabs(yu)) + rnd(pr) + 4.0 * ETA) +
                       U53 * fabs(DZ1.re) + ETA;
    const double aZ = abs_up(s.Z), aDZ = abs_up(s.DZ);
    // D(Z,e)^2 + c0
    const double e1 = up(s.e * s.e + 2.0 * s.e * aZ + Rsq);
    // D(Z,rho)^2 + D(c0,R)
    const double rho1 = up(s.rho * s.rho + 2.0 * s.rho * aZ + R + Rsq);
    // 2 D(Z,rho) D(DZ,sig) + 1
    const double sig1 = up(2.0 * (s.rho * s.sig + s.rho * aDZ + s.sig * aZ) + Rpr);
    s.Z = Z1;
    s.DZ = DZ1;
    s.e = e1;
    s.rho = rho1;
    s.sig = sig1;
}

struct cert_result { uint8_t flags; double R; };

// Strict divisors of the label lab of a root of p_n as a bit mask (bit k set
// when k | lab, k < lab; k < 32).  lab divides n, so they are among the
// strict divisors of n (divmask_n); lab = n, the label of almost every root,
// needs no division.
__device__ __forceinline__ uint32_t label_divmask(int lab, int n, uint32_t divmask_n)
{
    if (lab == n) return divmask_n;
    uint32_t m = 0u;
    for (uint32_t r = divmask_n; r; r &= r - 1u) {
        const int k = __builtin_ctz(r);
        if (k < lab && lab % k == 0) m |= 1u << k;
    }
    return m;
}

// The disk pass of a root of p_n of order N with label lab on D(c, R), then
// Thm proofRoots for p_n (and p_lab when lab != n).  UNI: every active lane
// of the wave certifies a root of the same p_N with label N, and N and dmask
// are wave-uniform, so the loop and the divisor tests are scalar branches and
// no state of step lab is kept.  P, dP: the centres of the last step, the
// plain values P(c), P'(c) (whether or not the test holds).
template <bool UNI>
__device__ __forceinline__ uint8_t certify_p_pass(int N, int lab, uint32_t dmask, cd c, double R, cd &P, cd &dP)
{ DD_EXACT
    disk_step t = {{0.0, 0.0}, {0.0, 0.0}, 0.0, 0.0, 0.0};
    cd Zk = {0, 0}, DZk = {0, 0};
    double ek = 0.0, sk = 0.0;
    bool label_ok = true;
#pragma unroll 2
    for (int kk = 1; kk <= N; ++kk) {
        disk_orbit_step(t, c, R);
        if (!UNI && kk == lab) { Zk = t.Z; DZk = t.DZ; ek = t.e; sk = t.sig; }
        // p_j, j a strict divisor of the label, has no zero on the disk
        if (kk < 32 && ((dmask >> kk) & 1u)) {
            const double r = t.rho;
            if (!(abs2_dn(t.Z) > up(r * r))) label_ok = false;
        }
    }
    P = t.Z;
    dP = t.DZ;
    const double Pup = up(abs_up(P) + up(t.e + rnd(P)));
    const double sP = up(t.sig + rnd(dP));
    // Thm proofRoots: R (|P'(c)| - sigma) > |P(c)|
    const double need = up(up(Pup / R) + sP);
    if (!(abs2_dn(dP) > up(need * need))) return 0;
    if (!UNI && lab != N) {
        // Thm proofRoots for p_lab on the same disk
        const double Pk = up(abs_up(Zk) + up(ek + rnd(Zk)));
        const double nk = up(up(Pk / R) + up(sk + rnd(DZk)));
        if (!(abs2_dn(DZk) > up(nk * nk))) label_ok = false;
    }
    return label_ok ? 2 | 4 : 2; // MSPLIT_R_CERTIFIED, MSPLIT_R_LABEL
}

// Certify c for P = q_{l,n} (l = 0: p_n) with label lab (p_n: period).
// The radius: R ~ 4 |P/P'| plus the rounding noise of a root, rounded up to a
// power of two; one fused pass carries the centres, the point radii e and
// the disk radii rho, sigma.  If the test fails, R grows by 16 (two more
// attempts).  p_n: the first pass takes R from the noise alone (a converged
// FP64 root has |P/P'| at rounding level, so this is almost always the same
// power of two) and needs no plain evaluation first; if it fails, R is taken
// from its centres P(c), P'(c) and the schedule above follows.  q_{l,n}: R
// from a plain evaluation.
// P_ONLY: a p_n-only instance (l = 0), without the registers of the q_{l,n}
// label tests.
template <bool P_ONLY = false>
__device__ cert_result certify_root(int l_arg, int n, int lab, uint32_t divmask_n, cd c)
{ DD_EXACT
    const int l = P_ONLY ? 0 : l_arg;
    const int N = l + n;
    cert_result res = {0, 0.0};
    if (!cfinite(c)) return res;
    const double noise = 64.0 * U53 * fmax(sqrt(cabs2(c)), 0x1p-8);
    // power of two above 4 |P/P'| + noise
    auto radius_for = [&](cd P0, cd dP0) {
        double R0 = 4.0 * sqrt(cabs2(P0) / cabs2(dP0)) + noise;
        if (!(R0 > 0x1p-1000) || !isfinite(R0)) R0 = 0x1p-1000;
        return ldexp(1.0, ilogb(R0) + 1);
    };
    if (l == 0) {
        const uint32_t dmask = label_divmask(lab, n, divmask_n);
        const int n0 = __builtin_amdgcn_readfirstlane(n);
        const bool uni = __ballot(n != n0 || lab != n) == 0;
        const uint32_t m0 = __builtin_amdgcn_readfirstlane(dmask);
        double R = ldexp(1.0, ilogb(noise) + 1);
        for (int attempt = 0; attempt < 4; ++attempt) {
            cd P0, dP0;
            const uint8_t f = uni ? certify_p_pass<true>(n0, n0, m0, c, R, P0, dP0)
                                  : certify_p_pass<false>(n, lab, dmask, c, R, P0, dP0);
            if (f) {
                res.flags = f;
                res.R = R;
                return res;
            }
            if (attempt == 0) {
                if (!cfinite(P0) || !cfinite(dP0)) return res;
                const double R1 = radius_for(P0, dP0);
                R = R1 > R ? R1 : 16.0 * R;
            } else {
                R *= 16.0;
            }
        }
        return res;
    }
    cd P0, dP0;
    eval_q(l, N, c, P0, dP0);
    if (!cfinite(P0) || !cfinite(dP0)) return res;
    double R = radius_for(P0, dP0);
    for (int attempt = 0; attempt < 3; ++attempt, R *= 16.0) {
        disk_step t = {{0.0, 0.0}, {0.0, 0.0}, 0.0, 0.0, 0.0};
        cd Zl = {0, 0}, DZl = {0, 0}, Zlm = {0, 0};
        double el = 0.0, rl = 0.0, sl = 0.0, rlm = 0.0;
        bool label_ok = true;
        for (int k = 0; k < N; ++k) {
            disk_orbit_step(t, c, R);
            const int kk = k + 1;
            if (kk == l - 1) { Zlm = t.Z; rlm = t.rho; }
            if (kk == l) { Zl = t.Z; DZl = t.DZ; el = t.e; rl = t.rho; sl = t.sig; }
            // q_{l,k} = z_{l+k} - z_l, k a strict divisor of n
            const int kd = kk - l;
            if (kd >= 1 && kd < n && ((divmask_n >> kd) & 1u)) {
                const cd d = {__dsub_rn(t.Z.re, Zl.re), __dsub_rn(t.Z.im, Zl.im)};
                const double r = up(t.rho + rl + rnd(d));
                if (!(abs2_dn(d) > up(r * r))) label_ok = false;
            }
            // q_{l-1,n} = z_{l-1+n} - z_{l-1}
            if (kk == l - 1 + n) {
                const cd d = {__dsub_rn(t.Z.re, Zlm.re), __dsub_rn(t.Z.im, Zlm.im)};
                const double r = up(t.rho + rlm + rnd(d));
                if (!(abs2_dn(d) > up(r * r))) label_ok = false;
            }
        }
        const cd P = {__dsub_rn(t.Z.re, Zl.re), __dsub_rn(t.Z.im, Zl.im)};
        const cd dP = {__dsub_rn(t.DZ.re, DZl.re), __dsub_rn(t.DZ.im, DZl.im)};
        const double Pup = up(abs_up(P) + up(t.e + el + rnd(P)));
        const double sP = up(t.sig + sl + rnd(dP));
        // Thm proofRoots: R (|P'(c)| - sigma) > |P(c)|
        const double need = up(up(Pup / R) + sP);
        if (abs2_dn(dP) > up(need * need)) {
            res.flags = 2; // MSPLIT_R_CERTIFIED
            res.R = R;
            if (lab != n) label_ok = false;
            if (label_ok) res.flags |= 4; // MSPLIT_R_LABEL
            return res;
        }
    }
    return res;
}

// ------------------------------------------------------- Newton basin
// Thm proofContract: the certified root z* lies in D(c, eta).  For
// eps > 3 eta, if P'(D(c, eps)) lies in a disk D(d, e') whose distance to 0
// exceeds twice its diameter (|d| > 5 e'), the Newton map sends D(c, eps)
// strictly into itself and D(c, eps) lies in the basin of z*.  eps is guessed
// from a plain orbit with the second derivative as the power of two below
// |P'| / (8 |P''|) (P' varies by about |P''| eps over the disk), capped at
// 1/4, and proven by the disk orbit of disk_orbit_step over D(c, eps);
// divided by 4 on failure, eight attempts (next to -2 the higher derivatives
// dominate and the guess can be 2^14 too large).  Returns eps, or 0.
__device__ __noinline__ double basin_radius(int l, int n, cd c, double eta)
{
    const int N = l + n;
    // z, z', z'' (z'' <- 2 (z'^2 + z z''), z' <- 2 z z' + 1, z <- z^2 + c)
    double zr = 0.0, zi = 0.0, dr = 0.0, di = 0.0, er = 0.0, ei = 0.0;
    double dlr = 0.0, dli = 0.0, elr = 0.0, eli = 0.0;
    for (int k = 1; k <= N; ++k) {
        const double ner = 2.0 * (dr * dr - di * di + zr * er - zi * ei);
        const double nei = 2.0 * (2.0 * dr * di + zr * ei + zi * er);
        const double ndr = 2.0 * (zr * dr - zi * di) + 1.0;
        const double ndi = 2.0 * (zr * di + zi * dr);
        const double nzr = zr * zr - zi * zi + c.re;
        const double nzi = 2.0 * zr * zi + c.im;
        zr = nzr; zi = nzi; dr = ndr; di = ndi; er = ner; ei = nei;
        if (k == l) { dlr = dr; dli = di; elr = er; eli = ei; }
    }
    const cd d1 = {dr - dlr, di - dli}, d2 = {er - elr, ei - eli};
    double eps = 0.125 * sqrt(cabs2(d1) / cabs2(d2));
    if (!(eps < 0.25)) eps = 0.25; // also for P'' = 0 and NaN
    eps = ldexp(1.0, ilogb(eps));  // power of two at most eps
    for (int attempt = 0; attempt < 8; ++attempt, eps *= 0.25) {
        if (!(eps > 3.0 * eta * (1.0 + 0x1p-40))) return 0.0;
        disk_step t = {{0.0, 0.0}, {0.0, 0.0}, 0.0, 0.0, 0.0};
        cd DZl = {0.0, 0.0};
        double sl = 0.0;
        for (int k = 0; k < N; ++k) {
            disk_orbit_step(t, c, eps);
            if (k + 1 == l) { DZl = t.DZ; sl = t.sig; }
        }
        cd d;
        double e1;
        {
            DD_EXACT
            d = {__dsub_rn(t.DZ.re, DZl.re), __dsub_rn(t.DZ.im, DZl.im)};
            e1 = up(t.sig + sl + rnd(d));
        }
        if (abs2_dn(d) > up(25.0 * up(e1 * e1))) return eps;
    }
    return 0.0;
}

// The basin radius of every certified output root (grid-stride over the
// output index space); a double-double root is taken at its FP64 part c with
// eta = R + |lo| (z* lies in D(c + lo, R)).
__global__ void k_basin(batch_args b, const double *re, const double *im, const double *re_lo,
                        const double *im_lo, uint8_t *flags, const double *radius, double *basin)
{
    unsigned long long *const wc = wave_ctr(b);
    const int64_t n_uniq = b.uniq_offs[b.T];
    type_count nb;
    type_cache tc;
    unsigned long long mbits = ~0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u0 = (int64_t)blockIdx.x * blockDim.x; u0 < n_uniq; u0 += stride) {
        const int64_t u = u0 + threadIdx.x;
        const int t = u < n_uniq ? cached_type(tc, b.uniq_offs, b.T, u) : nb.t;
        if (__ballot(u < n_uniq && t != nb.t)) {
            flush_count(wc, C_BASIN, nb);
            wave_reduce_by_key<RED_MIN>(wc, C_NCOUNTERS, C_MIN_BASIN_BITS, mbits != ~0ull ? nb.t : -1, mbits);
            mbits = ~0ull;
        }
        nb.t = t;
        if (u >= n_uniq) continue;
        const type_desc &td = b.types[t];
        const int64_t i = td.out_off + (u - b.uniq_offs[t]);
        double eps = 0.0;
        if (flags[i] & 2) {
            double eta = radius[i];
            if (re_lo && im_lo) {
                DD_EXACT
                eta = up(eta + up(fabs(re_lo[i]) + fabs(im_lo[i])));
            }
            eps = basin_radius(td.p.l, td.p.n, {re[i], im[i]}, eta);
        }
        basin[i] = eps;
        if (eps > 0.0) {
            flags[i] |= 16; // MSPLIT_R_BASIN
            nb.v += 1;
            const unsigned long long bits = (unsigned long long)__double_as_longlong(eps);
            mbits = bits < mbits ? bits : mbits;
        }
    }
    flush_count(wc, C_BASIN, nb);
    wave_reduce_by_key<RED_MIN>(wc, C_NCOUNTERS, C_MIN_BASIN_BITS, mbits != ~0ull ? nb.t : -1, mbits);
}

// ------------------------------------------------- double-double centres
// The same certificate for a double-double candidate c = hi + lo: the centres
// z_k run in double-double, the derivative centres and every radius in FP64.
// Each double-double operation on the centres (TwoSum / TwoProd based, with
// the final renormalisation) is within 2^-100 of the exact result relative to
// the magnitudes of its operands and result, so the R* term of the squaring
// step is bounded by U_DD (2|Z|^2 + |c| + |Z^2 + c|); the derivative
// recurrence uses Z.hi, and the neglected 2 |Z.lo| |DZ| joins its rounding.
constexpr double U_DD = 0x1p-100;

__device__ __forceinline__ double cdd_abs_up(cdd a)
{ DD_EXACT
    return up(abs_up({a.re.hi, a.im.hi}) + up(fabs(a.re.lo) + fabs(a.im.lo)));
}
// lower bound of |a| (0 when the bound is not positive)
__device__ __forceinline__ double cdd_abs_dn(cdd a)
{ DD_EXACT
    const double h = dn(sqrt(abs2_dn({a.re.hi, a.im.hi})));
    return fmax(0.0, dn(h - up(fabs(a.re.lo) + fabs(a.im.lo))));
}

struct disk_step_dd {
    cdd Z;
    cd DZ;
    double e, rho, sig;
};

__device__ __forceinline__ void disk_orbit_step_dd(disk_step_dd &s, cdd c, double aC, double R)
{ DD_EXACT
    const double aZ = cdd_abs_up(s.Z);
    const cdd Z1 = cdd_sqr_add(s.Z, c);
    const double Rsq = up(U_DD * up(2.0 * aZ * aZ + aC + cdd_abs_up(Z1)) + 8.0 * ETA);
    const double x = s.Z.re.hi, y = s.Z.im.hi, u = s.DZ.re, v = s.DZ.im;
    const double xu = __dmul_rn(x, u), yv = __dmul_rn(y, v), xv = __dmul_rn(x, v), yu = __dmul_rn(y, u);
    const cd pr = {__dsub_rn(xu, yv), __dadd_rn(xv, yu)};
    const cd DZ1 = {__dadd_rn(__dadd_rn(pr.re, pr.re), 1.0), __dadd_rn(pr.im, pr.im)};
    const double aDZ = abs_up(s.DZ);
    const double Rpr = up(2.0 * (U53 * (fabs(xu) + fabs(yv) + fabs(xv) + fabs(yu)) + rnd(pr) + 4.0 * ETA) +
                          U53 * fabs(DZ1.re) + ETA + 2.0 * up(fabs(s.Z.re.lo) + fabs(s.Z.im.lo)) * aDZ);
    const double e1 = up(s.e * s.e + 2.0 * s.e * aZ + Rsq);
    const double rho1 = up(s.rho * s.rho + 2.0 * s.rho * aZ + R + Rsq);
    const double sig1 = up(2.0 * (s.rho * s.sig + s.rho * aDZ + s.sig * aZ) + Rpr);
    s.Z = Z1;
    s.DZ = DZ1;
    s.e = e1;
    s.rho = rho1;
    s.sig = sig1;
}

// rounding bound of a double-double difference (relative U_DD)
__device__ __forceinline__ double rnd_dd(cdd a) { DD_EXACT return U_DD * cdd_abs_up(a) + 4.0 * ETA; }

__device__ __noinline__ cert_result certify_root_dd(int l, int n, int lab, uint32_t divmask_n, cdd c)
{ DD_EXACT
    const int N = l + n;
    cert_result res = {0, 0.0};
    const dd_step ns = dd_newton_step(l, N, c);
    const double s = sqrt(cdd_abs2_hi(ns.s));
    const double ac = sqrt(c.re.hi * c.re.hi + c.im.hi * c.im.hi);
    if (!isfinite(s) || !(ns.d2 > 0.0)) return res;
    double R0 = 4.0 * s + 64.0 * 0x1p-104 * fmax(ac, 0x1p-8);
    if (!(R0 > 0x1p-1000)) R0 = 0x1p-1000;
    double R = ldexp(1.0, ilogb(R0) + 1);
    const double aC = cdd_abs_up(c);
    const cdd zero = {{0.0, 0.0}, {0.0, 0.0}};
    for (int attempt = 0; attempt < 3; ++attempt, R *= 16.0) {
        disk_step_dd t = {zero, {0.0, 0.0}, 0.0, 0.0, 0.0};
        cdd Zl = zero, Zlm = zero, Zk = zero;
        cd DZl = {0, 0}, DZk = {0, 0};
        double el = 0.0, rl = 0.0, sl = 0.0, rlm = 0.0, ek = 0.0, sk = 0.0;
        bool label_ok = true;
        for (int k = 0; k < N; ++k) {
            disk_orbit_step_dd(t, c, aC, R);
            const int kk = k + 1;
            if (kk == l - 1) { Zlm = t.Z; rlm = t.rho; }
            if (kk == l) { Zl = t.Z; DZl = t.DZ; el = t.e; rl = t.rho; sl = t.sig; }
            if (l == 0) {
                if (kk == lab) { Zk = t.Z; DZk = t.DZ; ek = t.e; sk = t.sig; }
                if (kk < lab && lab % kk == 0 && !(cdd_abs_dn(t.Z) > t.rho)) label_ok = false;
            } else {
                const int kd = kk - l;
                if (kd >= 1 && kd < n && ((divmask_n >> kd) & 1u)) {
                    const cdd d = cdd_sub(t.Z, Zl);
                    if (!(cdd_abs_dn(d) > up(t.rho + rl + rnd_dd(d)))) label_ok = false;
                }
                if (kk == l - 1 + n) {
                    const cdd d = cdd_sub(t.Z, Zlm);
                    if (!(cdd_abs_dn(d) > up(t.rho + rlm + rnd_dd(d)))) label_ok = false;
                }
            }
        }
        const cdd P = cdd_sub(t.Z, Zl);
        const cd dP = {__dsub_rn(t.DZ.re, DZl.re), __dsub_rn(t.DZ.im, DZl.im)};
        const double Pup = up(cdd_abs_up(P) + up(t.e + el + rnd_dd(P)));
        const double sP = up(t.sig + sl + rnd(dP));
        const double need = up(up(Pup / R) + sP);
        if (abs2_dn(dP) > up(need * need)) {
            res.flags = 2;
            res.R = R;
            if (l == 0 && lab != n) {
                const double Pk = up(cdd_abs_up(Zk) + up(ek + rnd_dd(Zk)));
                const double nk = up(up(Pk / R) + up(sk + rnd(DZk)));
                if (!(abs2_dn(DZk) > up(nk * nk))) label_ok = false;
            }
            if (l > 0 && lab != n) label_ok = false;
            if (label_ok) res.flags |= 4;
            return res;
        }
    }
    return res;
}

// Grid-stride loop over the unique roots (compact index space of
// batch_args.uniq_offs, uniq_offs[T] roots, read on the device); counts and
// the largest radius stay in registers per type and are reduced once per
// wave at type changes and at the end.
// With low parts (re_lo, im_lo non-null) a candidate with a non-zero low
// part, or one the FP64 certificate cannot settle, gets the double-double
// certificate; MSPLIT_R_DD marks it.  With a hard list (list non-null)
// those candidates are appended to it for k_certify_dd instead, so that
// this kernel keeps the registers of the FP64 certificate alone.
template <bool HARD_LIST, bool P_ONLY = false>
__global__ void __launch_bounds__(256) k_certify(batch_args b, const double *re, const double *im, const double *re_lo,
                          const double *im_lo, const int32_t *period, uint8_t *flags, double *radius, uint32_t *list)
{
    const int64_t n_uniq = b.uniq_offs[b.T];
    unsigned long long *const wc = wave_ctr(b);
    type_count nc, nl;
    type_cache tc;
    unsigned long long rbits = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u0 = (int64_t)blockIdx.x * blockDim.x; u0 < n_uniq; u0 += stride) {
        const int64_t u = u0 + threadIdx.x;
        const int t = u < n_uniq ? cached_type(tc, b.uniq_offs, b.T, u) : nc.t;
        if (__ballot(u < n_uniq && t != nc.t)) {
            flush_count(wc, C_CERTIFIED, nc);
            flush_count(wc, C_LABEL, nl);
            // non-negative doubles order like their bit patterns
            wave_reduce_by_key<RED_MAX>(wc, C_NCOUNTERS, C_MAX_RAD_BITS, rbits ? nc.t : -1, rbits);
            rbits = 0;
        }
        nc.t = nl.t = t;
        bool hard = false;
        if (u < n_uniq) {
            const type_desc &td = b.types[t];
            const int64_t i = td.out_off + (u - b.uniq_offs[t]);
            const cd c = {re[i], im[i]};
            const int lab = period ? period[i] : td.p.n;
            const cd lo = re_lo && im_lo ? cd{re_lo[i], im_lo[i]} : cd{0.0, 0.0};
            const bool has_lo = lo.re != 0.0 || lo.im != 0.0;
            cert_result r = {0, 0.0};
            if (!has_lo) r = certify_root<P_ONLY>(td.p.l, td.p.n, lab, td.p.divmask_lo, c);
            const bool use_dd = re_lo && im_lo && (has_lo || !(r.flags & 2));
            hard = HARD_LIST && use_dd;
            if (!hard) {
                if (use_dd) r = certify_root_dd(td.p.l, td.p.n, lab, td.p.divmask_lo, {{c.re, lo.re}, {c.im, lo.im}});
                flags[i] = (c.im == 0.0 && lo.im == 0.0 ? 1 : 0) | r.flags | (use_dd ? 8 : 0);
                radius[i] = r.R;
                nc.v += (r.flags & 2) != 0;
                nl.v += (r.flags & 4) != 0;
                if (r.flags & 2) {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(r.R);
                    rbits = bits > rbits ? bits : rbits;
                }
            }
        }
        if (HARD_LIST) wave_append(list, &b.gctr[G_HARD_CERT], hard, (uint32_t)u);
    }
    flush_count(wc, C_CERTIFIED, nc);
    flush_count(wc, C_LABEL, nl);
    wave_reduce_by_key<RED_MAX>(wc, C_NCOUNTERS, C_MAX_RAD_BITS, rbits ? nc.t : -1, rbits);
}

// The double-double certificates of the hard list of k_certify<true>.
// An FP64 root whose certificate fails (no low part) is first polished by
// double-double Newton steps on the certified polynomial (its rounding error,
// not its position, may be what the disk test cannot absorb next to a close
// root); when the polished point is certified it replaces the root in the
// output (high and low parts, MSPLIT_R_DD).
__global__ void k_certify_dd(batch_args b, double *re, double *im, double *re_lo, double *im_lo,
                             const int32_t *period, uint8_t *flags, double *radius, const uint32_t *list)
{
    unsigned long long *const wc = wave_ctr(b);
    const int64_t n = (int64_t)b.gctr[G_HARD_CERT];
    type_count nc, nl;
    type_cache tc;
    unsigned long long rbits = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < n; k0 += stride) {
        const int64_t k = k0 + threadIdx.x;
        const int64_t u = k < n ? (int64_t)list[k] : -1;
        const int t = u >= 0 ? cached_type(tc, b.uniq_offs, b.T, u) : nc.t;
        if (__ballot(u >= 0 && t != nc.t)) {
            flush_count(wc, C_CERTIFIED, nc);
            flush_count(wc, C_LABEL, nl);
            wave_reduce_by_key<RED_MAX>(wc, C_NCOUNTERS, C_MAX_RAD_BITS, rbits ? nc.t : -1, rbits);
            rbits = 0;
        }
        nc.t = nl.t = t;
        if (u < 0) continue;
        const type_desc &td = b.types[t];
        const int64_t i = td.out_off + (u - b.uniq_offs[t]);
        cd c = {re[i], im[i]}, lo = {re_lo[i], im_lo[i]};
        const int lab = period ? period[i] : td.p.n;
        cert_result r = certify_root_dd(td.p.l, td.p.n, lab, td.p.divmask_lo, {{c.re, lo.re}, {c.im, lo.im}});
        if (!(r.flags & 2) && lo.re == 0.0 && lo.im == 0.0) {
            cdd z = {{c.re, 0.0}, {c.im, 0.0}};
            for (int s = 0; s < 4; ++s) {
                const dd_step st = dd_newton_step(td.p.l, td.p.N, z);
                if (!isfinite(st.s.re.hi) || !isfinite(st.s.im.hi)) break;
                z = cdd_sub(z, st.s);
            }
            const cert_result r2 = certify_root_dd(td.p.l, td.p.n, lab, td.p.divmask_lo, z);
            if (r2.flags & 2) {
                r = r2;
                c = {z.re.hi, z.im.hi};
                lo = {z.re.lo, z.im.lo};
                re[i] = c.re;
                im[i] = c.im;
                re_lo[i] = lo.re;
                im_lo[i] = lo.im;
            }
        }
        flags[i] = (c.im == 0.0 && lo.im == 0.0 ? 1 : 0) | r.flags | 8;
        radius[i] = r.R;
        nc.v += (r.flags & 2) != 0;
        nl.v += (r.flags & 4) != 0;
        if (r.flags & 2) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(r.R);
            rbits = bits > rbits ? bits : rbits;
        }
    }
    flush_count(wc, C_CERTIFIED, nc);
    flush_count(wc, C_LABEL, nl);
    wave_reduce_by_key<RED_MAX>(wc, C_NCOUNTERS, C_MAX_RAD_BITS, rbits ? nc.t : -1, rbits);
}

// Thm certif, global part, on each type's list (sorted by real part):
// certified disks must be pairwise disjoint and disjoint from their
// conjugates unless centred on the real axis; with the quarter-separation
// reading every pair satisfies |z_i - z_j| >= 4 max(R_i, R_j) and every
// non-real root Im z >= 2 R.  Every pair closer than 4 (R_i + R_max) in real
// part is checked.  Also a statistic: the least distance found between a
// root and its conjugate or one of the next 8 roots in real order (an upper
// bound of the least distance; the closest pairs of p_n, the leftmost real
// roots, are adjacent in that order).  radius == nullptr: only the statistic.
// With low parts the distances are taken on hi + lo (the list is ordered by
// the real part to 2^-46, so closer roots may come in either order).
__global__ void __launch_bounds__(256) k_separation(batch_args b, const double *re, const double *im,
                                                    const double *re_lo, const double *im_lo, const double *radius)
{
    // blocks loop over tiles of 256 roots of the output index space; a tile
    // and the SEP_HALO roots after it are staged in LDS (the scan of a root
    // reads up to 8 successors, more only where disks are large), the rest
    // of a long scan reads global memory
    constexpr int SEP_HALO = 8, NT = 256 + SEP_HALO;
    __shared__ double sx[NT], sy[NT], sxl[NT], syl[NT], sR[NT];
    __shared__ int stp[NT];
    const int64_t n_uniq = b.uniq_offs[b.T];
    unsigned long long *const wc = wave_ctr(b);
    type_count bad;
    type_cache tc, th;
    unsigned long long sbits = ~0ull;
    const bool lo = re_lo && im_lo;
    for (int64_t u0 = (int64_t)blockIdx.x * 256; u0 < n_uniq; u0 += (int64_t)gridDim.x * 256) {
        for (int k = threadIdx.x; k < NT; k += 256) {
            const int64_t u = u0 + k;
            int t = -1;
            if (u < n_uniq) {
                type_cache &c = k < 256 ? tc : th;
                t = cached_type(c, b.uniq_offs, b.T, u);
                const int64_t i = b.types[t].out_off + (u - c.lo);
                sx[k] = re[i];
                sy[k] = im[i];
                sxl[k] = lo ? re_lo[i] : 0.0;
                syl[k] = lo ? im_lo[i] : 0.0;
                sR[k] = radius ? radius[i] : 0.0;
            }
            stp[k] = t;
        }
        __syncthreads();
        const int64_t u = u0 + threadIdx.x;
        const int t = u < n_uniq ? stp[threadIdx.x] : bad.t;
        if (__ballot(u < n_uniq && t != bad.t)) {
            flush_count(wc, C_OVERLAP, bad);
            wave_reduce_by_key<RED_MIN>(wc, C_NCOUNTERS, C_MIN_SEP_BITS, sbits != ~0ull ? bad.t : -1, sbits);
            sbits = ~0ull;
        }
        bad.t = t;
        if (u < n_uniq) {
            const type_desc &td = b.types[t];
            const int64_t u_end = tc.hi; // the type's roots end there (tc holds type t: u < n_uniq)
            const double rmax =
                radius ? __longlong_as_double((long long)b.ctr[(int64_t)t * C_NCOUNTERS + C_MAX_RAD_BITS]) : 0.0;
            const int k0 = threadIdx.x;
            const double xi = sx[k0], yi = sy[k0], Ri = sR[k0], xl = sxl[k0], yl = syl[k0];
            const double yt = yi + yl;
            double best = yt > 0.0 ? 2.0 * yt : INFINITY;
            if (radius && (yi != 0.0 || yl != 0.0) && !(yt >= 2.0 * Ri)) bad.v += 1;
            bool pair_bad = false;
            for (int64_t j = u + 1, c = 0; j < u_end; ++j, ++c) {
                const int64_t k = j - u0;
                double xj, yj, xlj, ylj, Rj;
                if (k < NT) {
                    xj = sx[k];
                    yj = sy[k];
                    xlj = sxl[k];
                    ylj = syl[k];
                    Rj = sR[k];
                } else {
                    const int64_t ij = td.out_off + (j - tc.lo);
                    xj = re[ij];
                    yj = im[ij];
                    xlj = lo ? re_lo[ij] : 0.0;
                    ylj = lo ? im_lo[ij] : 0.0;
                    Rj = radius ? radius[ij] : 0.0;
                }
                const double dx = (xj - xi) + (xlj - xl);
                // the list is ordered by real part only to the key resolution
                // 2^-KEY_RES: a closer root may follow a farther one by that much
                const bool need_pair = radius && dx <= 4.0 * (Ri + rmax) + 0x1p-45;
                if (!need_pair && (dx > best || c >= 8)) break;
                const double dy = (yj - yi) + (ylj - yl);
                const double d = sqrt(dx * dx + dy * dy);
                best = fmin(best, d);
                if (radius && !(d >= 4.0 * fmax(Ri, Rj) * (1.0 + 1e-15))) pair_bad = true;
            }
            bad.v += pair_bad;
            if (isfinite(best)) {
                const unsigned long long bits = (unsigned long long)__double_as_longlong(best);
                sbits = bits < sbits ? bits : sbits;
            }
        }
        __syncthreads();
    }
    flush_count(wc, C_OVERLAP, bad);
    wave_reduce_by_key<RED_MIN>(wc, C_NCOUNTERS, C_MIN_SEP_BITS, sbits != ~0ull ? bad.t : -1, sbits);
}

// ---------------------------------------------------------- classification
// Threads run over the collected index space (coll_offs[T] roots, read on
// the device).  keep[u] selects the
// roots of the output set, cls[u] is the period (p_n) or n (q_{l,n}).
//
// q_{l,n}: a candidate near a centre Hyp(k), k | n, may be a descent stalled
// inside the rounding-noise ball of that multiple root (Thm fact_mis), where
// q evaluates to noise -- even to an exact zero, which passes as converged --
// and neither the step ratio nor any fixed distance tells it from a genuine
// root.  q ~ C d^eta at distance d from a root of multiplicity
// eta = eta_l(k) = floor((l-1)/k) + 2, so the ball has radius about
// eps^(1/eta): 1e-4 in FP64 for eta = 4, 0.2 for the centre 0 of q_{20,2}
// (eta = 21).  Thm proofRoots settles it: it certifies exactly one root
// counted with multiplicity, which a multiple root never passes, so a
// candidate within max(NEAR_CENTRE, 2^(-50/eta)) of a centre is kept only
// when the certificate (FP64, else double-double) holds on it.
constexpr double NEAR_CENTRE = 1e-3;



__device__ __forceinline__ double near_centre_radius(int l, int kmin)
{
    const int eta = (l - 1) / kmin + 2;
    return fmax(NEAR_CENTRE, exp2(-50.0 / eta));
}

// FP64 pass: every FP64 candidate whose classification FP64 settles; the
// double-double candidates and the q candidates near a centre go to a hard
// list for k_classify_hard (their certificates and double-double orbits kept
// out of this kernel's registers).
// One thread per collected root; the grid covers an upper bound of their
// number (blocks past it return at once).
__global__ void __launch_bounds__(256) k_classify(batch_args b, const cd *uz, const uint8_t *uz_dd, uint32_t *keep,
                                                  int32_t *cls, int labels, uint32_t *list)
{
    __shared__ int64_t offs[MAX_TYPES + 1];
    const int64_t n = b.coll_offs[b.T];
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((int64_t)blockIdx.x * blockDim.x >= n) return; // whole blocks
    for (int i = threadIdx.x; i <= b.T; i += blockDim.x) offs[i] = b.coll_offs[i];
    __syncthreads();
    bool hard = false;
    if (u < n) {
        const int t = find_type_lds(offs, b.T, u);
        const plan_t &pl = b.types[t].p;
        const cd c = uz[u];
        const bool dd = uz_dd[u];
        uint32_t k = 1;
        int per = pl.n;
        if (pl.l == 0) {
            if (dd) hard = labels != 0;
            else if (labels) per = classify_p(pl.n, pl.divmask_lo, pl.tau, c);
        } else if (dd) {
            hard = true;
        } else {
            double hmin2 = INFINITY;
            int kmin = pl.n;
            const bool kq = classify_q(pl.l, pl.n, pl.divmask_lo, pl.tau, c, hmin2, kmin);
            // s_{l,n} (el < 0) has simple roots only: no stall next to a centre
            const double w = near_centre_radius(pl.l, kmin);
            hard = kq && pl.el > 0 && hmin2 < w * w;
            k = kq ? 1u : 0u;
        }
        if (!hard) {
            keep[u] = k;
            cls[u] = per;
        }
    }
    wave_append(list, &b.gctr[G_HARD_CLS], hard, (uint32_t)u);
}

__global__ void k_classify_hard(batch_args b, const cd *uz, const cd *uz_lo, const uint8_t *uz_dd, uint32_t *keep,
                                int32_t *cls, const uint32_t *list)
{
    const int64_t n = (int64_t)b.gctr[G_HARD_CLS];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const int64_t u = list[j];
        const int t = find_type(b.coll_offs, b.T, u);
        const plan_t &pl = b.types[t].p;
        const cd c = uz[u];
        const bool dd = uz_dd[u];
        const cd lo = dd ? uz_lo[u] : cd{0.0, 0.0};
        const cdd cc = {{c.re, lo.re}, {c.im, lo.im}};
        uint32_t k = 1;
        int per = pl.n;
        if (pl.l == 0) {
            per = classify_p_dd(pl.n, pl.divmask_lo, pl.tau_dd, cc);
        } else {
            double hmin2 = INFINITY;
            int kmin = pl.n;
            bool kq = dd ? classify_q_dd(pl.l, pl.n, pl.divmask_lo, pl.tau_dd, cc, hmin2, kmin)
                         : classify_q(pl.l, pl.n, pl.divmask_lo, pl.tau, c, hmin2, kmin);
            // cheap first: the step ratio of Thm fact_mis in double-double
            const bool multiple = pl.el > 0; // q_{l,n}; s_{l,n} has simple roots only
            if (multiple && kq && !dd && hmin2 < 1e-12 && stalled_at_multiple_root(pl.l, pl.n, kmin, c)) kq = false;
            const double w = near_centre_radius(pl.l, kmin);
            if (multiple && kq && hmin2 < w * w) {
                cert_result r = {0, 0.0};
                if (!dd) r = certify_root(pl.l, pl.n, pl.n, pl.divmask_lo, c);
                if (!(r.flags & 2)) r = certify_root_dd(pl.l, pl.n, pl.n, pl.divmask_lo, cc);
                kq = (r.flags & 2) != 0;
            }
            k = kq ? 1u : 0u;
        }
        keep[u] = k;
        cls[u] = per;
    }
}

} // namespace msplit
