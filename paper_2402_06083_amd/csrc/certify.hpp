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
// R* bound applies verbatim.  The GPU rounds to nearest only, so every radius
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

namespace msplit {

__device__ __forceinline__ double ulp64(double x)
{
    double a = fabs(x);
    if (!(a >= 2.2250738585072014e-308)) return 4.9406564584124654e-324;
    return ldexp(1.0, ilogb(a) - 52);
}
__device__ __forceinline__ double up(double x) { return __dadd_rn(__dmul_rn(x, 1.0 + 0x1p-47), 0x1p-1000); }
__device__ __forceinline__ double dn(double x) { return __dsub_rn(__dmul_rn(x, 1.0 - 0x1p-47), 0x1p-1000); }
// upper bound of |a|
__device__ __forceinline__ double abs_up(cd a)
{
    return up(sqrt(up(__dadd_rn(__dmul_rn(a.re, a.re), __dmul_rn(a.im, a.im)))));
}
// lower bound of |a|^2
__device__ __forceinline__ double abs2_dn(cd a)
{
    return dn(__dadd_rn(__dmul_rn(a.re, a.re), __dmul_rn(a.im, a.im)));
}
__device__ __forceinline__ double hulp(cd a) { return 0.5 * (ulp64(a.re) + ulp64(a.im)); }

struct disk_step {
    cd Z, DZ;  // centres
    double e;  // radius of z_k at the exact point c0 (R = 0)
    double rho, sig; // radii of z_k and dz_k over D(c0, R)
};

// one step of the disk orbit; Rin = radius of c
__device__ __forceinline__ void disk_orbit_step(disk_step &s, cd c, double Rin)
{
    const double x = s.Z.re, y = s.Z.im, u = s.DZ.re, v = s.DZ.im;
    // centre of z^2
    double xx = __dmul_rn(x, x), yy = __dmul_rn(y, y), xy = __dmul_rn(x, y);
    cd sq = {__dsub_rn(xx, yy), __dadd_rn(xy, xy)};
    double Rsq = hulp(sq) + 0.5 * (ulp64(xx) + ulp64(yy) + 2.0 * ulp64(xy));
    // centre of z * dz
    double xu = __dmul_rn(x, u), yv = __dmul_rn(y, v), xv = __dmul_rn(x, v), yu = __dmul_rn(y, u);
    cd pr = {__dsub_rn(xu, yv), __dadd_rn(xv, yu)};
    double Rpr = hulp(pr) + 0.5 * (ulp64(xu) + ulp64(yv) + ulp64(xv) + ulp64(yu));
    cd Z1 = {__dadd_rn(sq.re, c.re), __dadd_rn(sq.im, c.im)};
    cd DZ1 = {__dadd_rn(__dadd_rn(pr.re, pr.re), 1.0), __dadd_rn(pr.im, pr.im)};
    const double aZ = abs_up(s.Z), aDZ = abs_up(s.DZ);
    // D(Z,e)^2 + c0
    double e1 = up(s.e * s.e + 2.0 * s.e * aZ + Rsq + hulp(Z1));
    // D(Z,rho)^2 + D(c0,R)
    double rho1 = up(s.rho * s.rho + 2.0 * s.rho * aZ + Rsq + Rin + hulp(Z1));
    // 2 D(Z,rho) D(DZ,sig) + 1 (doubling is exact)
    double sig1 = up(2.0 * (s.rho * s.sig + s.rho * aDZ + s.sig * aZ + Rpr) + hulp(DZ1));
    s.Z = Z1;
    s.DZ = DZ1;
    s.e = e1;
    s.rho = rho1;
    s.sig = sig1;
}

struct cert_result { uint8_t flags; double R; };

// Certify c for P = q_{l,n} (l = 0: p_n) with label lab (p_n: period).
__device__ cert_result certify_root(int l, int n, int lab, uint32_t divmask_n, cd c)
{
    const int N = l + n;
    // pass A: centre values and point radii
    disk_step s = {{0.0, 0.0}, {0.0, 0.0}, 0.0, 0.0, 0.0};
    cd Zl = {0, 0}, DZl = {0, 0};
    double el = 0.0;
    cd Zk = {0, 0}, DZk = {0, 0};
    double ek = 0.0;
    for (int k = 0; k < N; ++k) {
        disk_orbit_step(s, c, 0.0);
        if (k + 1 == l) { Zl = s.Z; DZl = s.DZ; el = s.e; }
        if (l == 0 && k + 1 == lab) { Zk = s.Z; DZk = s.DZ; ek = s.e; }
    }
    cd P = {__dsub_rn(s.Z.re, Zl.re), __dsub_rn(s.Z.im, Zl.im)};
    cd dP = {__dsub_rn(s.DZ.re, DZl.re), __dsub_rn(s.DZ.im, DZl.im)};
    const double Pup = up(abs_up(P) + up(s.e + el + hulp(P)));
    const double dlow = sqrt(abs2_dn(dP));
    cert_result res = {0, 0.0};
    if (!(dlow > 0.0) || !isfinite(Pup)) return res;
    double R0 = 4.0 * Pup / dlow;
    if (!(R0 > 0x1p-1000)) R0 = 0x1p-1000;
    double R = ldexp(1.0, ilogb(R0) + 1); // power of two above R0
    for (int attempt = 0; attempt < 3; ++attempt, R *= 16.0) {
        // pass B: radii over D(c, R)
        disk_step t = {{0.0, 0.0}, {0.0, 0.0}, 0.0, 0.0, 0.0};
        cd Zl1 = {0, 0};
        double rl = 0.0, sl = 0.0, rlm = 0.0;
        cd Zlm = {0, 0};
        double sk = 0.0;
        bool label_ok = true;
        for (int k = 0; k < N; ++k) {
            disk_orbit_step(t, c, R);
            const int kk = k + 1;
            if (kk == l - 1) { Zlm = t.Z; rlm = t.rho; }
            if (kk == l) { Zl1 = t.Z; rl = t.rho; sl = t.sig; }
            if (l == 0) {
                if (kk == lab) sk = t.sig;
                // p_j, j a strict divisor of the label, has no zero on the disk
                if (kk < lab && lab % kk == 0) {
                    double r = t.rho;
                    if (!(abs2_dn(t.Z) > up(r * r))) label_ok = false;
                }
            } else {
                // q_{l,k} = z_{l+k} - z_l, k a strict divisor of n
                int kd = kk - l;
                if (kd >= 1 && kd < n && ((divmask_n >> kd) & 1u)) {
                    cd d = {__dsub_rn(t.Z.re, Zl1.re), __dsub_rn(t.Z.im, Zl1.im)};
                    double r = up(t.rho + rl + hulp(d));
                    if (!(abs2_dn(d) > up(r * r))) label_ok = false;
                }
                // q_{l-1,n} = z_{l-1+n} - z_{l-1}
                if (kk == l - 1 + n) {
                    cd d = {__dsub_rn(t.Z.re, Zlm.re), __dsub_rn(t.Z.im, Zlm.im)};
                    double r = up(t.rho + rlm + hulp(d));
                    if (!(abs2_dn(d) > up(r * r))) label_ok = false;
                }
            }
        }
        const double sP = up(t.sig + sl + hulp(dP));
        const double tneed = up(up(Pup / R) + sP);
        if (abs2_dn(dP) > up(tneed * tneed)) {
            res.flags = 2; // MSPLIT_R_CERTIFIED
            res.R = R;
            if (l == 0 && lab != n) {
                // Thm proofRoots for p_lab on the same disk
                double Pk = up(abs_up(Zk) + up(ek + hulp(Zk)));
                double need = up(up(Pk / R) + up(sk + hulp(DZk)));
                if (!(abs2_dn(DZk) > up(need * need))) label_ok = false;
            }
            if (l > 0 && lab != n) label_ok = false;
            if (label_ok) res.flags |= 4; // MSPLIT_R_LABEL
            return res;
        }
    }
    return res;
}

__global__ void k_certify(int l, int n, uint32_t divmask_n, const double *re, const double *im,
                          const int32_t *period, uint8_t *flags, double *radius, uint64_t count,
                          unsigned long long *ctr, int ctr_cert, int ctr_label, int ctr_maxrad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nc = 0, nl = 0;
    if (i < (int64_t)count) {
        cd c = {re[i], im[i]};
        int lab = period ? period[i] : n;
        cert_result r = certify_root(l, n, lab, divmask_n, c);
        uint8_t f = (im[i] == 0.0 ? 1 : 0) | r.flags;
        if (flags) flags[i] = f;
        if (radius) radius[i] = r.R;
        nc += (r.flags & 2) != 0;
        nl += (r.flags & 4) != 0;
        if (r.flags & 2) atomicMax(&ctr[ctr_maxrad], (unsigned long long)__double_as_longlong(r.R));
    }
    wave_add(&ctr[ctr_cert], nc);
    wave_add(&ctr[ctr_label], nl);
}

// Thm certif, global part, on a list sorted by real part: certified disks
// must be pairwise disjoint and disjoint from their conjugates unless centred
// on the real axis; with the quarter-separation reading every pair satisfies
// |z_i - z_j| >= 4 max(R_i, R_j) and every non-real root Im z >= 2 R.
// Also the least distance among the roots and their conjugates, scanning the
// neighbours in real order (at most 64 of them).
__global__ void k_separation(const double *re, const double *im, const double *radius, uint64_t count,
                             double rmax, unsigned long long *ctr, int ctr_overlap, int ctr_minsep)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long bad = 0;
    if (i < (int64_t)count) {
        const double xi = re[i], yi = im[i], Ri = radius ? radius[i] : 0.0;
        double best = yi > 0.0 ? 2.0 * yi : INFINITY;
        if (radius && yi != 0.0 && !(yi >= 2.0 * Ri)) bad = 1;
        // every pair closer than 4 (R_i + R_max) in real part is checked; the
        // nearest-neighbour scan for the statistic stops after 64 points
        for (int64_t j = i + 1, c = 0; j < (int64_t)count; ++j, ++c) {
            double dx = re[j] - xi;
            bool need_pair = radius && dx <= 4.0 * (Ri + rmax);
            if (!need_pair && (dx > best || c >= 64)) break;
            double dy = im[j] - yi;
            double d = sqrt(dx * dx + dy * dy);
            best = fmin(best, d);
            if (radius) {
                double Rj = radius[j];
                if (!(d >= 4.0 * fmax(Ri, Rj) * (1.0 + 1e-15))) bad = 1;
            }
        }
        if (isfinite(best)) atomicMin(&ctr[ctr_minsep], (unsigned long long)__double_as_longlong(best));
    }
    wave_add(&ctr[ctr_overlap], bad);
}

// Same scan, reading the largest certificate radius from the counter slot
// that k_certify filled (no host round trip between the two kernels).
__global__ void k_separation_rmax(const double *re, const double *im, const double *radius, uint64_t count,
                                  unsigned long long *ctr, int ctr_maxrad, int ctr_overlap, int ctr_minsep)
{
    const double rmax = __longlong_as_double((long long)ctr[ctr_maxrad]);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long bad = 0;
    if (i < (int64_t)count) {
        const double xi = re[i], yi = im[i], Ri = radius[i];
        double best = yi > 0.0 ? 2.0 * yi : INFINITY;
        if (yi != 0.0 && !(yi >= 2.0 * Ri)) bad = 1;
        for (int64_t j = i + 1, c = 0; j < (int64_t)count; ++j, ++c) {
            double dx = re[j] - xi;
            bool need_pair = dx <= 4.0 * (Ri + rmax);
            if (!need_pair && (dx > best || c >= 64)) break;
            double dy = im[j] - yi;
            double d = sqrt(dx * dx + dy * dy);
            best = fmin(best, d);
            double Rj = radius[j];
            if (!(d >= 4.0 * fmax(Ri, Rj) * (1.0 + 1e-15))) bad = 1;
        }
        if (isfinite(best)) atomicMin(&ctr[ctr_minsep], (unsigned long long)__double_as_longlong(best));
    }
    wave_add(&ctr[ctr_overlap], bad);
}

} // namespace msplit
