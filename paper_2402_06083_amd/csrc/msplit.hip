// msplit.hip -- C ABI of libmsplit (see include/msplit.h) and the host side of
// the splitting pipeline on gfx950.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <vector>

#include "msplit.h"
#include "kernels.hpp"
#include "certify.hpp"

using namespace msplit;

namespace {

// ------------------------------------------------------------ combinatorics
// Moebius function and the counts of Thm countingHyp (eq. HypCount) and
// eq. MisCount, used for the completeness check of a split.
int mobius(int n)
{
    int r = 1;
    for (int p = 2; p * p <= n; ++p) {
        if (n % p) continue;
        n /= p;
        if (n % p == 0) return 0;
        r = -r;
    }
    return n > 1 ? -r : r;
}

int64_t hyp_count(int n)
{
    int64_t s = 0;
    for (int k = 1; k <= n; ++k)
        if (n % k == 0) s += (int64_t)mobius(n / k) * ((int64_t)1 << (k - 1));
    return s;
}

int64_t mis_count(int l, int n)
{
    if (l == 1) return 0;
    if (l == 0) return hyp_count(n);
    int64_t phi = ((l - 1) % n == 0) ? (((int64_t)1 << (l - 1)) - 1) : ((int64_t)1 << (l - 1));
    return phi * hyp_count(n);
}

uint32_t divisor_mask(int n)
{
    uint32_t m = 0;
    for (int k = 1; k < n && k < 32; ++k)
        if (n % k == 0) m |= 1u << k;
    return m;
}

const msplit_options *defaults()
{
    static msplit_options o = {sizeof(msplit_options), MSPLIT_FP64, 0.0, 0, 0, 0, 0.0, 0, 0, 0.0};
    return &o;
}

bool valid_type(int l, int n) { return n >= 1 && l >= 0 && l != 1 && l + n <= 30; }

// ------------------------------------------------------------------- plan
plan_t make_plan(int l, int n, const msplit_options *o)
{
    plan_t p;
    memset(&p, 0, sizeof(p));
    p.l = l;
    p.n = n;
    p.N = l + n;
    p.D = (int64_t)1 << (p.N - 1);
    p.level = o->level > 0 ? o->level : (l == 0 ? 5.0 : 100.0);
    p.M = o->points_per_turn ? (int)o->points_per_turn : 8;
    p.q = p.M / 4;
    const int64_t half = (int64_t)p.M * p.D / 2; // fine points, upper half
    int64_t F = o->seg_points;
    if (!F) {
        // about 2^17 segments to fill the chip, 8..128 fine points each
        F = half >> 17;
        F = std::max<int64_t>(8, std::min<int64_t>(128, F));
    }
    F = std::min<int64_t>(F, half);
    // power of two, multiple of q
    int64_t f2 = 1;
    while (f2 * 2 <= F) f2 *= 2;
    F = std::max<int64_t>(f2, p.q);
    p.F = F;
    p.S = half / F;
    p.NS = 2 * p.D + 1;
    double IN = o->cap_factor > 0 ? o->cap_factor : (l == 0 ? 1.0 : 2.6);
    double capf = ceil(IN * log((double)p.D));
    int floor_cap = o->min_cap ? (int)o->min_cap : 20;
    p.cap = std::max(floor_cap, (int)capf);
    // identification radius: far below the least root distance of p_N
    // (118.4 / 4^N, Section 6.3.2) and far above the FP64 error of a root
    double sep = 118.4 * pow(4.0, -(double)p.N);
    p.tau = std::min(1e-12, sep / 32.0);
    p.tol_desc = 0x1p-46;
    p.divmask_lo = divisor_mask(n);
    p.precision = o->precision;
    p.fp32_switch = o->fp32_switch > 0 ? (float)o->fp32_switch : 0x1p-14f;
    // work-queue chunks: about four chunks per wave of a full persistent grid
    auto chunk_for = [](int64_t items) {
        int64_t waves = 256 * 8 * 4;
        int64_t c = items / (waves * 4);
        return (uint32_t)std::max<int64_t>(64, std::min<int64_t>(1024, c));
    };
    p.chunk_seg = chunk_for(p.S);
    p.chunk_start = chunk_for(p.NS);
    return p;
}

// ------------------------------------------------------------- workspace
struct layout {
    size_t ctr, seeds, starts, status, segf, keys, keys2, vals, vals2, flag, pos, temp, total;
    size_t temp_bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

hipError_t rocprim_temp(const plan_t &p, size_t &bytes)
{
    size_t sort_b = 0, scan_b = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, sort_b, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (uint32_t *)nullptr, (uint32_t *)nullptr, (size_t)p.NS, 0, 64);
    if (e != hipSuccess) return e;
    e = rocprim::exclusive_scan(nullptr, scan_b, (uint32_t *)nullptr, (uint32_t *)nullptr, 0u, (size_t)p.NS,
                                rocprim::plus<uint32_t>());
    if (e != hipSuccess) return e;
    bytes = std::max(sort_b, scan_b);
    return hipSuccess;
}

layout make_layout(const plan_t &p, size_t temp_bytes)
{
    layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.ctr = take(sizeof(unsigned long long) * C_NCOUNTERS);
    L.seeds = take(sizeof(cd) * (p.S + 1));
    L.starts = take(sizeof(cd) * p.NS);
    L.status = take(p.NS);
    L.segf = take(p.S);
    L.keys = take(8 * p.NS);
    L.keys2 = take(8 * p.NS);
    L.vals = take(4 * p.NS);
    L.vals2 = take(4 * p.NS);
    L.flag = take(4 * p.NS);
    L.pos = take(4 * p.NS);
    L.temp_bytes = temp_bytes;
    L.temp = take(temp_bytes);
    L.total = off;
    return L;
}

// -------------------------------------------------------------- launches
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_nan(cd *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = {__longlong_as_double(0x7ff8000000000000ll), __longlong_as_double(0x7ff8000000000000ll)};
}
__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int device_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// persistent grid: enough waves to fill every SIMD several times
unsigned persistent_blocks(int64_t work, int bs)
{
    int64_t cap = (int64_t)device_cus() * 8;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (work + bs - 1) / bs));
}

struct call_ctx {
    hipStream_t stream;
    msplit_stats *stats;
    int err = MSPLIT_OK;
    bool check(hipError_t e)
    {
        if (e != hipSuccess) {
            if (stats) stats->hip_error = (int32_t)e;
            err = MSPLIT_E_DEVICE;
            return false;
        }
        return true;
    }
};

#define CHK(x)                      \
    do {                            \
        if (!ctx.check((x))) return ctx.err; \
    } while (0)

void set_cis(int M, hipStream_t stream)
{
    static int cached = -1;
    if (cached == M) return;
    double re[64], im[64];
    for (int s = 0; s < 64; ++s) {
        double t = 2.0 * M_PI * (double)(s % M) / (double)M;
        re[s] = cos(t);
        im[s] = sin(t);
        // exact values at the quarter turns
        if (4 * (s % M) == 0) { re[s] = 1; im[s] = 0; }
        if (4 * (s % M) == M) { re[s] = 0; im[s] = 1; }
        if (4 * (s % M) == 2 * M) { re[s] = -1; im[s] = 0; }
        if (4 * (s % M) == 3 * M) { re[s] = 0; im[s] = -1; }
    }
    (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(c_cis_re), re, sizeof(re), 0, hipMemcpyHostToDevice, stream);
    (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(c_cis_im), im, sizeof(im), 0, hipMemcpyHostToDevice, stream);
    (void)hipStreamSynchronize(stream);
    cached = M;
}

__global__ void k_unzip(const cd *z, double *re, double *im, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { re[i] = z[i].re; im[i] = z[i].im; }
}

// The whole split of one type.  Returns a status; *count is always written.
int split_one(int l, int n, const msplit_options *opts, void *workspace, uint64_t ws_bytes, msplit_roots *out,
              uint64_t *count, msplit_stats *stats, void *stream_v, bool starts_only = false,
              double *sre = nullptr, double *sim = nullptr, uint64_t scap = 0)
{
    if (count) *count = 0;
    if (!count || !workspace) return MSPLIT_E_ARG;
    if (!starts_only && !out) return MSPLIT_E_ARG;
    if (starts_only && (!sre || !sim)) return MSPLIT_E_ARG;
    if (!valid_type(l, n)) return MSPLIT_E_ARG;
    if (!opts) opts = defaults();
    if (opts->struct_size && opts->struct_size != sizeof(msplit_options)) return MSPLIT_E_ARG;
    if (opts->precision < 0 || opts->precision > 1) return MSPLIT_E_UNSUPPORTED;
    if (opts->points_per_turn && (opts->points_per_turn % 4 || opts->points_per_turn > 64)) return MSPLIT_E_ARG;
    if (stats) memset(stats, 0, sizeof(*stats));
    plan_t p = make_plan(l, n, opts);
    // FP64 keys separate the roots only while the identification radius
    // stays well above the FP64 rounding of a root
    if (p.tau < 0x1p-50) return MSPLIT_E_PRECISION;
    if (l != 0) return MSPLIT_E_UNSUPPORTED;
    hipStream_t stream = (hipStream_t)stream_v;
    call_ctx ctx{stream, stats};
    size_t temp_bytes = 0;
    CHK(rocprim_temp(p, temp_bytes));
    layout L = make_layout(p, temp_bytes);
    if (ws_bytes < L.total) return MSPLIT_E_WORKSPACE;
    char *ws = (char *)workspace;
    unsigned long long *ctr = (unsigned long long *)(ws + L.ctr);
    cd *seeds = (cd *)(ws + L.seeds);
    cd *starts = (cd *)(ws + L.starts);
    uint8_t *status = (uint8_t *)(ws + L.status);
    uint8_t *segf = (uint8_t *)(ws + L.segf);
    uint64_t *keys = (uint64_t *)(ws + L.keys), *keys2 = (uint64_t *)(ws + L.keys2);
    uint32_t *vals = (uint32_t *)(ws + L.vals), *vals2 = (uint32_t *)(ws + L.vals2);
    uint32_t *flag = (uint32_t *)(ws + L.flag), *pos = (uint32_t *)(ws + L.pos);
    void *temp = ws + L.temp;
    const int bs = opts->block_size ? (int)opts->block_size : 256;
    if (bs % 64 || bs > 1024) return MSPLIT_E_ARG;

    set_cis(p.M, stream);
    // events: [0] start, [1] seeds, [2] walk, [3] descend, [4] collect,
    // [5] classify, [6] certify (end)
    hipEvent_t ev[7];
    for (int i = 0; i < 7; ++i) CHK(hipEventCreate(&ev[i]));
    struct ev_guard {
        hipEvent_t *e;
        ~ev_guard() { for (int i = 0; i < 7; ++i) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    CHK(hipEventRecord(ev[0], stream));

    // counters: zero, min-separation slot at +inf
    k_fill_u64<<<1, 64, 0, stream>>>(ctr, C_NCOUNTERS, 0ull);
    k_fill_u64<<<1, 1, 0, stream>>>(ctr + C_MIN_SEP_BITS, 1, 0x7ff0000000000000ull);
    k_fill_nan<<<blocks_for(p.NS, 256), 256, 0, stream>>>(starts, p.NS);
    k_fill_u8<<<blocks_for(p.NS, 256), 256, 0, stream>>>(status, p.NS, ST_NONE);
    // seeds (lift from the circle |p_1| = lambda_0)
    k_seeds<<<blocks_for(p.S + 1, bs), bs, 0, stream>>>(p, seeds, starts, ctr);
    CHK(hipEventRecord(ev[1], stream));
    // level-line walk
    k_walk<<<persistent_blocks(p.S, bs), bs, 0, stream>>>(p, seeds, starts, segf, ctr);
    CHK(hipEventRecord(ev[2], stream));
    if (starts_only) {
        if (scap < (uint64_t)p.NS) return MSPLIT_E_CAPACITY;
        k_unzip<<<blocks_for(p.NS, 256), 256, 0, stream>>>(starts, sre, sim, p.NS);
        CHK(hipGetLastError());
        unsigned long long h[C_NCOUNTERS];
        CHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream));
        CHK(hipStreamSynchronize(stream));
        *count = (uint64_t)p.NS;
        if (stats) {
            stats->starts = (uint64_t)p.NS;
            stats->phase_fail = h[C_PHASE_FAIL] + h[C_SEED_FAIL];
            stats->steps_lift = h[C_STEPS_LIFT];
            stats->steps_walk = h[C_STEPS_WALK];
            float a = 0.f, b = 0.f;
            (void)hipEventElapsedTime(&a, ev[0], ev[1]);
            (void)hipEventElapsedTime(&b, ev[1], ev[2]);
            stats->ms_stage[0] = a;
            stats->ms_stage[1] = b;
            stats->ms_device = a + b;
        }
        return (h[C_PHASE_FAIL] + h[C_SEED_FAIL]) ? MSPLIT_E_INCOMPLETE : MSPLIT_OK;
    }
    // descents
    k_descend<<<persistent_blocks(p.NS, bs), bs, 0, stream>>>(p, starts, status, ctr);
    CHK(hipEventRecord(ev[3], stream));
    // nset collection
    k_keys<<<blocks_for(p.NS, 256), 256, 0, stream>>>(p, starts, status, keys, vals);
    size_t tb = temp_bytes;
    CHK(rocprim::radix_sort_pairs(temp, tb, keys, keys2, vals, vals2, (size_t)p.NS, 0, 64, stream));
    k_mark<<<blocks_for(p.NS, 256), 256, 0, stream>>>(p, starts, keys2, vals2, flag);
    tb = temp_bytes;
    CHK(rocprim::exclusive_scan(temp, tb, flag, pos, 0u, (size_t)p.NS, rocprim::plus<uint32_t>(), stream));
    k_scatter<<<blocks_for(p.NS, 256), 256, 0, stream>>>(p, starts, vals2, flag, pos, out->re, out->im,
                                                          out->capacity, ctr);
    CHK(hipEventRecord(ev[4], stream));
    CHK(hipGetLastError());
    unsigned long long h[C_NCOUNTERS];
    CHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream));
    CHK(hipStreamSynchronize(stream));
    const uint64_t uniq = h[C_UNIQUE];
    *count = uniq;
    if (uniq > out->capacity) return MSPLIT_E_CAPACITY;
    // classification
    if (uniq) {
        if (out->re_lo)
            k_fill_u64<<<blocks_for((int64_t)uniq, 256), 256, 0, stream>>>((unsigned long long *)out->re_lo, uniq, 0ull);
        if (out->im_lo)
            k_fill_u64<<<blocks_for((int64_t)uniq, 256), 256, 0, stream>>>((unsigned long long *)out->im_lo, uniq, 0ull);
        k_classify<<<blocks_for((int64_t)uniq, 256), 256, 0, stream>>>(
            p, out->re, out->im, (opts->flags & MSPLIT_F_NO_LABEL) ? nullptr : out->period, out->preperiod,
            out->flags, uniq);
        if (out->radius)
            k_fill_u64<<<blocks_for((int64_t)uniq, 256), 256, 0, stream>>>((unsigned long long *)out->radius, uniq, 0ull);
    }
    CHK(hipEventRecord(ev[5], stream));
    // certificate
    const bool cert = (opts->flags & MSPLIT_F_CERTIFY) != 0;
    if (cert && uniq) {
        if (!out->radius || !out->flags) return MSPLIT_E_ARG;
        k_certify<<<blocks_for((int64_t)uniq, 128), 128, 0, stream>>>(
            l, n, p.divmask_lo, out->re, out->im, (opts->flags & MSPLIT_F_NO_LABEL) ? nullptr : out->period,
            out->flags, out->radius, uniq, ctr, C_CERTIFIED, C_LABEL, C_MAX_RAD_BITS);
        // the separation scan needs the largest radius
        k_separation_rmax<<<blocks_for((int64_t)uniq, 256), 256, 0, stream>>>(
            out->re, out->im, out->radius, uniq, ctr, C_MAX_RAD_BITS, C_OVERLAP, C_MIN_SEP_BITS);
    } else if (uniq) {
        k_separation<<<blocks_for((int64_t)uniq, 256), 256, 0, stream>>>(out->re, out->im, nullptr, uniq, 0.0,
                                                                          ctr, C_OVERLAP, C_MIN_SEP_BITS);
    }
    CHK(hipEventRecord(ev[6], stream));
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream));
    CHK(hipStreamSynchronize(stream));
    float ms = 0.f, mss[6] = {0, 0, 0, 0, 0, 0};
    (void)hipEventElapsedTime(&ms, ev[0], ev[6]);
    for (int i = 0; i < 6; ++i) (void)hipEventElapsedTime(&mss[i], ev[i], ev[i + 1]);

    const uint64_t total = h[C_REAL] + 2 * (uniq - h[C_REAL]);
    const uint64_t expected = (uint64_t)p.D;
    if (stats) {
        stats->starts = (uint64_t)p.NS;
        stats->converged = h[C_CONVERGED];
        stats->diverged = h[C_DIVERGED];
        stats->timeouts = h[C_TIMEOUT];
        stats->unique = uniq;
        stats->n_real = h[C_REAL];
        stats->total = total;
        stats->expected = expected;
        stats->missing = expected > total ? expected - total : 0;
        stats->phase_fail = h[C_PHASE_FAIL] + h[C_SEED_FAIL];
        stats->certified = h[C_CERTIFIED];
        stats->label_proven = h[C_LABEL];
        stats->overlaps = h[C_OVERLAP];
        stats->steps_lift = h[C_STEPS_LIFT];
        stats->steps_walk = h[C_STEPS_WALK];
        stats->steps_desc = h[C_STEPS_DESC];
        stats->steps_fp32 = h[C_STEPS_FP32];
        memcpy(&stats->min_sep, &h[C_MIN_SEP_BITS], 8);
        memcpy(&stats->max_radius, &h[C_MAX_RAD_BITS], 8);
        stats->ms_device = ms;
        for (int i = 0; i < 6; ++i) stats->ms_stage[i] = mss[i];
    }
    if (total != expected) return MSPLIT_E_INCOMPLETE;
    return MSPLIT_OK;
}

} // namespace

// ===================================================================== C ABI
extern "C" {

const char *msplit_strerror(int status)
{
    switch (status) {
    case MSPLIT_OK: return "ok";
    case MSPLIT_E_ARG: return "invalid argument";
    case MSPLIT_E_CAPACITY: return "output capacity too small";
    case MSPLIT_E_WORKSPACE: return "workspace too small";
    case MSPLIT_E_DEVICE: return "HIP error";
    case MSPLIT_E_INCOMPLETE: return "fewer roots than the exact count";
    case MSPLIT_E_PRECISION: return "precision cannot separate the roots";
    case MSPLIT_E_UNSUPPORTED: return "not supported by this build";
    default: return "unknown status";
    }
}

uint64_t msplit_expected_count(int l, int n, int primitive_only)
{
    if (!valid_type(l, n) && !(l == 0 && n >= 1 && n <= 62)) return 0;
    if (l == 0) return primitive_only ? (uint64_t)hyp_count(n) : ((uint64_t)1 << (n - 1));
    return (uint64_t)mis_count(l, n);
}

int msplit_workspace_size(int l, int n, const msplit_options *opts, uint64_t *bytes)
{
    if (!bytes || !valid_type(l, n)) return MSPLIT_E_ARG;
    if (!opts) opts = defaults();
    plan_t p = make_plan(l, n, opts);
    size_t tb = 0;
    if (rocprim_temp(p, tb) != hipSuccess) return MSPLIT_E_DEVICE;
    *bytes = make_layout(p, tb).total;
    return MSPLIT_OK;
}

int msplit_hyperbolic(int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                      msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream)
{
    return split_one(0, n, opts, workspace, workspace_bytes, out, count, stats, stream);
}

int msplit_misiurewicz(int l, int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                       msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream)
{
    if (l < 2) {
        if (count) *count = 0;
        return MSPLIT_E_ARG;
    }
    return split_one(l, n, opts, workspace, workspace_bytes, out, count, stats, stream);
}

int msplit_starts(int l, int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes, double *re,
                  double *im, uint64_t capacity, uint64_t *count, msplit_stats *stats, void *stream)
{
    return split_one(l, n, opts, workspace, workspace_bytes, nullptr, count, stats, stream, true, re, im, capacity);
}

int msplit_certify(int l, int n, msplit_roots *roots, uint64_t count, void *workspace, uint64_t workspace_bytes,
                   msplit_stats *stats, void *stream_v)
{
    if (!roots || !workspace || !roots->re || !roots->im || !roots->flags || !roots->radius) return MSPLIT_E_ARG;
    if (!valid_type(l, n)) return MSPLIT_E_ARG;
    if (workspace_bytes < 256) return MSPLIT_E_WORKSPACE;
    if (stats) memset(stats, 0, sizeof(*stats));
    hipStream_t stream = (hipStream_t)stream_v;
    call_ctx ctx{stream, stats};
    unsigned long long *ctr = (unsigned long long *)workspace;
    k_fill_u64<<<1, 64, 0, stream>>>(ctr, C_NCOUNTERS, 0ull);
    k_fill_u64<<<1, 1, 0, stream>>>(ctr + C_MIN_SEP_BITS, 1, 0x7ff0000000000000ull);
    if (count) {
        k_certify<<<blocks_for((int64_t)count, 128), 128, 0, stream>>>(
            l, n, divisor_mask(n), roots->re, roots->im, roots->period, roots->flags, roots->radius, count, ctr,
            C_CERTIFIED, C_LABEL, C_MAX_RAD_BITS);
    }
    unsigned long long h[C_NCOUNTERS];
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream));
    CHK(hipStreamSynchronize(stream));
    double rmax;
    memcpy(&rmax, &h[C_MAX_RAD_BITS], 8);
    if (count)
        k_separation<<<blocks_for((int64_t)count, 256), 256, 0, stream>>>(roots->re, roots->im, roots->radius,
                                                                           count, rmax, ctr, C_OVERLAP,
                                                                           C_MIN_SEP_BITS);
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream));
    CHK(hipStreamSynchronize(stream));
    if (stats) {
        stats->certified = h[C_CERTIFIED];
        stats->label_proven = h[C_LABEL];
        stats->overlaps = h[C_OVERLAP];
        memcpy(&stats->min_sep, &h[C_MIN_SEP_BITS], 8);
        memcpy(&stats->max_radius, &h[C_MAX_RAD_BITS], 8);
    }
    return MSPLIT_OK;
}

int msplit_batch_workspace_size(const int32_t *ln_pairs, int npairs, const msplit_options *opts, uint64_t *bytes)
{
    if (!ln_pairs || npairs <= 0 || !bytes) return MSPLIT_E_ARG;
    uint64_t mx = 0;
    for (int i = 0; i < npairs; ++i) {
        uint64_t b = 0;
        int r = msplit_workspace_size(ln_pairs[2 * i], ln_pairs[2 * i + 1], opts, &b);
        if (r) return r;
        mx = std::max(mx, b);
    }
    *bytes = mx;
    return MSPLIT_OK;
}

int msplit_batch(const int32_t *ln_pairs, int npairs, const msplit_options *opts, void *workspace,
                 uint64_t workspace_bytes, msplit_roots *out, const uint64_t *caps, uint64_t *counts,
                 msplit_stats *stats, void *stream)
{
    if (!ln_pairs || npairs <= 0 || !out || !caps || !counts) return MSPLIT_E_ARG;
    uint64_t off = 0;
    int first_err = MSPLIT_OK;
    for (int i = 0; i < npairs; ++i) {
        msplit_roots o = *out;
        o.re = out->re + off;
        o.im = out->im + off;
        o.re_lo = out->re_lo ? out->re_lo + off : nullptr;
        o.im_lo = out->im_lo ? out->im_lo + off : nullptr;
        o.period = out->period ? out->period + off : nullptr;
        o.preperiod = out->preperiod ? out->preperiod + off : nullptr;
        o.flags = out->flags ? out->flags + off : nullptr;
        o.radius = out->radius ? out->radius + off : nullptr;
        o.capacity = caps[i];
        int r = split_one(ln_pairs[2 * i], ln_pairs[2 * i + 1], opts, workspace, workspace_bytes, &o, &counts[i],
                          stats ? &stats[i] : nullptr, stream);
        if (r && first_err == MSPLIT_OK) first_err = r;
        if (r == MSPLIT_E_ARG || r == MSPLIT_E_DEVICE || r == MSPLIT_E_WORKSPACE) return r;
        off += caps[i];
    }
    return first_err;
}

} // extern "C"
