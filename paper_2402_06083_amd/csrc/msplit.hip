// msplit.hip -- C ABI of libmsplit (see include/msplit.h) and the host side of
// the splitting pipeline on gfx950.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <cstring>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "msplit.h"
#include "kernels.hpp"
#include "certify.hpp"
#include "sort.hpp"
#include "stream.hpp"

using namespace msplit;

// The workspace of msplit_hyperbolic_static: a device array of fixed size in
// the library, so that the call allocates nothing.  Each device holds its
// own copy until the process ends.  In host code the name is a stand-in, not
// a device address: the address comes from hipGetSymbolAddress, taken once
// per device (scratch_of_device).
static __device__ __align__(256) unsigned char scratch[MSPLIT_STATIC_SCRATCH_BYTES];

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
    // MSPLIT_F_SIMPLE: Mis(l,n) from the simple roots of s_{l,n} = p_{N-1} +
    // p_{l-1} = q_{l,n} / q_{l-1,n} (eq. polySimple), half the degree of q_{l,n}
    const bool simple = l >= 2 && (o->flags & MSPLIT_F_SIMPLE);
    p.el = simple ? -(l - 1) : l;
    p.eN = simple ? p.N - 1 : p.N;
    p.D = (int64_t)1 << (p.eN - 1);
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
    // power of two, multiple of q, at least 2 (a segment is walked from both
    // ends to its middle point)
    int64_t f2 = 1;
    while (f2 * 2 <= F) f2 *= 2;
    F = std::max<int64_t>(f2, std::max<int64_t>(p.q, 2));
    p.F = F;
    p.S = half / F;
    p.seg0 = 0;
    p.nseg = p.S;
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
    // double-double route next to -2 (Section 6.3.2): the real Misiurewicz
    // parameters at the left end of M pair up closer than FP64 resolves from
    // order about 18 on (their gap shrinks like 8^-N); a generous tip radius
    // keeps every FP64 root outside it far from its neighbours
    p.x_tip = (l >= 2 && p.N >= 14) ? 0x1p-14 : 0.0;
    if (l == 0 && p.N >= 25) {
        // p_n beyond FP64 separation (118.4 / 4^n, Section 6.3.2, nears the
        // FP64 spacing at n = 25): FP64 keeps tau = 2^-44 away from -2 and
        // the tip goes to double-double.  The closest pairs there are a
        // centre of period n/2 and its satellite of period n (Section 6.3.2),
        // whose gap grows about linearly with the distance x to -2, measured
        // at 6e-8 x for n = 26 and halving with each further order; the tip
        // covers every x where that gap is below 128 tau, and at least the
        // region where the spacing of the real roots, about
        // 4 pi sqrt(x / 2) / 2^n, is below 128 tau.
        p.tau = 0x1p-44;
        // from order 28 the left end of the level line (about -2 - 14.7 / 4^n)
        // is closer to -2 than the FP64 spacing: re-solve the starts there
        // (the FP64 walk failed over the last 320 starts at order 30 and the
        // last 1088 at order 31: a tip four times larger per order beyond 30)
        if (p.N >= 28) p.tip_starts = (int)std::min<int64_t>(p.NS, (int64_t)4096 << (2 * std::max(0, p.N - 30)));
        const double a = 128.0 * p.tau * ldexp(1.0, p.N) / (4.0 * M_PI);
        const double x_sat = 128.0 * p.tau / (6e-8 * ldexp(1.0, 26 - p.N));
        p.x_tip = std::max(2.0 * a * a, x_sat);
    }
    p.tau_dd = 0x1p-90;
    p.divmask_lo = divisor_mask(n);
    p.precision = o->precision;
    p.fp32_switch = o->fp32_switch > 0 ? (float)o->fp32_switch : 0x1p-14f;
    return p;
}

// work-queue chunk: about four chunks per wave of a full persistent grid
uint32_t chunk_for(int64_t items)
{
    const int64_t waves = 256 * 8 * 4;
    const int64_t c = items / (waves * 4);
    return (uint32_t)std::max<int64_t>(64, std::min<int64_t>(1024, c));
}

// ------------------------------------------------------------------ batch
struct batch_plan {
    int T = 0;
    std::vector<int> slot;          // processing position -> caller index
    std::vector<type_desc> td;      // in processing order
    std::vector<int64_t> seed_offs, seg_offs, start_offs; // T + 1
    int64_t n_seeds = 0, n_segs = 0, n_starts = 0;
    int64_t n_tip = 0; // starts re-solved in double-double, all types
};

// Types in decreasing order N (then caller order) so that the persistent
// queues end on the cheapest items.
int make_batch(const int32_t *ln, int npairs, const msplit_options *o, const uint64_t *out_offs,
               const uint64_t *caps, batch_plan &bp)
{
    if (npairs <= 0 || npairs > MAX_TYPES) return MSPLIT_E_ARG;
    bp.T = npairs;
    bp.slot.resize(npairs);
    std::iota(bp.slot.begin(), bp.slot.end(), 0);
    std::stable_sort(bp.slot.begin(), bp.slot.end(), [&](int a, int b) {
        return ln[2 * a] + ln[2 * a + 1] > ln[2 * b] + ln[2 * b + 1];
    });
    bp.td.resize(npairs);
    bp.seed_offs.assign(npairs + 1, 0);
    bp.seg_offs.assign(npairs + 1, 0);
    bp.start_offs.assign(npairs + 1, 0);
    for (int t = 0; t < npairs; ++t) {
        const int c = bp.slot[t];
        const int l = ln[2 * c], n = ln[2 * c + 1];
        if (!valid_type(l, n)) return MSPLIT_E_ARG;
        type_desc &d = bp.td[t];
        memset(&d, 0, sizeof(d));
        d.p = make_plan(l, n, o);
        d.seed_off = bp.seed_offs[t];
        d.seg_off = bp.seg_offs[t];
        d.start_off = bp.start_offs[t];
        d.out_off = out_offs ? (int64_t)out_offs[c] : 0;
        d.tip_lo_off = bp.n_tip;
        bp.n_tip += d.p.tip_starts;
        d.cap = caps ? caps[c] : 0;
        bp.seed_offs[t + 1] = bp.seed_offs[t] + d.p.nseg + 1;
        bp.seg_offs[t + 1] = bp.seg_offs[t] + d.p.nseg;
        bp.start_offs[t + 1] = bp.start_offs[t] + d.p.NS;
    }
    bp.n_seeds = bp.seed_offs[npairs];
    bp.n_segs = bp.seg_offs[npairs];
    bp.n_starts = bp.start_offs[npairs];
    return MSPLIT_OK;
}

// ------------------------------------------------------------- workspace
struct layout {
    size_t gctr, ctr, spread, isz, cis, types, offs, rtile, seeds, starts, status, iters, segf, flag0, pos0, keys,
        vals, keys2, vals2, zs, zs_lo, roots, roots_lo, tip_lo, flag, pos, counts, part, mid, total;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// device sizes (int64 slots): the starts, the prekeys tiles (whose survivor
// counts are scanned), the digit counts scanned between the sweeps of the sort
enum { SZ_STARTS = 0, SZ_COUNTS, SZ_PKTILES, SZ_N = 4 };

// tiles of the sort: every segment (type) rounds up to whole tiles
int64_t sort_tiles_max(int64_t n, int T) { return n / RS_TILE + T + 1; }

layout make_layout(const batch_plan &bp)
{
    layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    const size_t T = (size_t)bp.T, NS = (size_t)bp.n_starts;
    const int64_t n_counts = sort_tiles_max(bp.n_starts, bp.T) * RS_BINS;
    const int64_t n_part = std::max<int64_t>(bp.n_starts, n_counts) / SC_TILE + 2;
    L.gctr = take(sizeof(unsigned long long) * G_NCOUNTERS);
    L.ctr = take(sizeof(unsigned long long) * C_NCOUNTERS * T);
    L.spread = take(sizeof(unsigned long long) * C_NCOUNTERS * T * CTR_SPREAD);
    L.isz = take(sizeof(int64_t) * SZ_N);
    L.cis = take(sizeof(double) * 128);
    L.types = take(sizeof(type_desc) * T);
    L.offs = take(sizeof(int64_t) * 8 * (T + 1));
    L.rtile = take(sizeof(int64_t) * (T + 1));
    L.seeds = take(sizeof(cd) * bp.n_seeds);
    L.starts = take(sizeof(cd) * NS);
    L.status = take(NS);
    L.iters = take(NS);
    L.segf = take(2 * (size_t)bp.n_segs); // one flag per walk (two per segment)
    L.flag0 = take(4 * NS);
    L.pos0 = take(4 * NS);
    L.keys = take(8 * NS);
    L.vals = take(4 * NS);
    L.keys2 = take(8 * NS);
    L.zs = take(sizeof(cd) * NS);
    // the walks' meeting points live in zs (free until the collection) when
    // they fit there (segments of at least 4 q fine points), else apart
    const size_t mid_bytes = sizeof(walk_mid) * (size_t)bp.n_segs;
    L.mid = mid_bytes <= sizeof(cd) * NS ? L.zs : take(mid_bytes);
    L.zs_lo = take(sizeof(cd) * NS);
    L.roots = take(sizeof(cd) * NS);
    L.roots_lo = take(sizeof(cd) * NS);
    L.tip_lo = take(sizeof(cd) * (size_t)std::max<int64_t>(bp.n_tip, 1));
    L.vals2 = take(4 * NS);
    L.flag = take(4 * NS);
    L.pos = take(4 * NS);
    L.counts = take(4 * (size_t)n_counts);
    L.part = take(4 * (size_t)n_part);
    L.total = off;
    return L;
}

// -------------------------------------------------------------- launches
// counters: zero; per-type minimum-separation slot at +inf (every copy);
// the device sizes that are known before the call
__device__ __forceinline__ unsigned long long ctr_identity(int slot)
{
    return slot == C_MIN_SEP_BITS || slot == C_MIN_BASIN_BITS ? 0x7ff0000000000000ull : 0ull;
}
__global__ void k_init_counters(unsigned long long *gctr, unsigned long long *ctr, unsigned long long *spread, int T,
                                int64_t *isz, int64_t n_starts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < G_NCOUNTERS) gctr[i] = 0;
    if (i < T * C_NCOUNTERS) ctr[i] = ctr_identity(i % C_NCOUNTERS);
    if (i < T * C_NCOUNTERS * CTR_SPREAD) spread[i] = ctr_identity(i % C_NCOUNTERS);
    if (isz && i < SZ_N)
        isz[i] = i == SZ_STARTS ? n_starts : i == SZ_PKTILES ? (n_starts + PK_TILE - 1) / PK_TILE : 0;
}
// ctr = the copies combined: sums, except the largest radius (max) and the
// least separation and least basin radius (min); non-negative doubles order like their bit
// patterns.  One wave per counter, lane k reading copy k.
static_assert(CTR_SPREAD == 64, "one lane per counter copy");
__global__ void k_fold_counters(unsigned long long *ctr, const unsigned long long *spread, int T)
{
    const int n = T * C_NCOUNTERS;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return; // whole waves
    const int slot = i % C_NCOUNTERS;
    unsigned long long a = spread[(size_t)lane * n + i];
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(a, d, 64);
        if (slot == C_MAX_RAD_BITS) a = o > a ? o : a;
        else if (slot == C_MIN_SEP_BITS || slot == C_MIN_BASIN_BITS) a = o < a ? o : a;
        else a += o;
    }
    if (lane == 0) ctr[i] = a;
}
unsigned fold_blocks(int T) { return (unsigned)((T * C_NCOUNTERS + 3) / 4); }

__global__ void k_unzip(const cd *z, double *re, double *im, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { re[i] = z[i].re; im[i] = z[i].im; }
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

unsigned blocks_for(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// persistent grid: enough waves to fill every SIMD several times
unsigned persistent_blocks(int64_t work, int bs)
{
    int64_t cap = (int64_t)device_cus() * 8;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (work + bs - 1) / bs));
}

// exclusive scan of *n_dev (at most n_max) u32 values, in == out allowed
void scan_u32(const uint32_t *in, uint32_t *out, const int64_t *n_dev, int64_t n_max, uint32_t *part,
              hipStream_t st)
{
    const int64_t tiles = std::max<int64_t>(1, (n_max + SC_TILE - 1) / SC_TILE);
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, (int64_t)device_cus() * 8);
    k_scan_reduce<<<grid, SC_BLOCK, 0, st>>>(in, n_dev, part);
    k_scan_down<<<grid, SC_BLOCK, 0, st>>>(in, out, n_dev, part);
}

// segmented sort (segments seg[0..T], on the device, seg[0] = 0) of at most
// n_max pairs on key bits [0, bits); the sorted pairs end in (*k, *v)
void sort_pairs(uint64_t **k, uint32_t **v, uint64_t *k2, uint32_t *v2, const int64_t *seg, int64_t *tile, int T,
                int bits, int64_t n_max, uint32_t *counts, int64_t *n_counts, uint32_t *part, hipStream_t st)
{
    k_rs_tiles<<<1, 64, 0, st>>>(seg, T, tile, n_counts);
    const int64_t tmax = sort_tiles_max(n_max, T);
    // the upsweep holds little LDS: 8 blocks per CU; the downsweep's LDS
    // allows fewer, and 4 per CU measured best
    const unsigned grid_up = (unsigned)std::min<int64_t>(tmax, (int64_t)device_cus() * 8);
    const unsigned grid_down = (unsigned)std::min<int64_t>(tmax, (int64_t)device_cus() * 4);
    const rs_segs s = {seg, tile, T};
    uint64_t *ka = *k, *kb = k2;
    uint32_t *va = *v, *vb = v2;
    for (int shift = 0; shift < bits; shift += 8) {
        k_rs_upsweep<<<grid_up, SC_BLOCK, 0, st>>>(ka, s, shift, counts);
        scan_u32(counts, counts, n_counts, tmax * RS_BINS, part, st);
        k_rs_downsweep<<<grid_down, SC_BLOCK, 0, st>>>(ka, va, kb, vb, s, shift, counts);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *k = ka;
    *v = va;
}

struct call_ctx {
    msplit_stats *stats;
    int nstats;
    int err = MSPLIT_OK;
    bool check(hipError_t e)
    {
        if (e != hipSuccess) {
            for (int i = 0; i < nstats && stats; ++i) stats[i].hip_error = (int32_t)e;
            err = MSPLIT_E_DEVICE;
            return false;
        }
        return true;
    }
};

#define CHK(x)                               \
    do {                                     \
        if (!ctx.check((x))) return ctx.err; \
    } while (0)

struct events {
    hipEvent_t e[7];
    int made = 0;
    ~events() { for (int i = 0; i < made; ++i) (void)hipEventDestroy(e[i]); }
};

// One call of the pipeline: the plan, the workspace carve-up and the kernel
// arguments, all prepared on the host before anything is enqueued.
struct batch_call {
    batch_plan bp;
    layout L;
    msplit_options o;
    msplit_roots out;
    int bs = 256;
    bool cert = false, labels = true, any_tip = false, basin = false, conj = false;
    batch_args ba;
    char *ws = nullptr;
    int64_t out_max = 0;
    std::vector<int64_t> offs; // host copy of the item offsets (uploaded once)
    std::vector<unsigned long long> h;
};

template <typename P>
P *ws_at(const batch_call &c, size_t off) { return (P *)(c.ws + off); }

// Options of a call (no device work).
int check_options(batch_call &c, const msplit_options *opts, const msplit_roots *out, bool starts_only)
{
    if (!starts_only && (!out || !out->re || !out->im)) return MSPLIT_E_ARG;
    if (opts->struct_size && opts->struct_size != sizeof(msplit_options)) return MSPLIT_E_ARG;
    if (opts->precision < 0 || opts->precision > 2) return MSPLIT_E_ARG;
    // M: a power of two, 4 .. 64 (the walk takes phase indices and starts by masks)
    if (opts->points_per_turn && (opts->points_per_turn < 4 || opts->points_per_turn > 64 ||
                                  (opts->points_per_turn & (opts->points_per_turn - 1))))
        return MSPLIT_E_ARG;
    c.bs = opts->block_size ? (int)opts->block_size : 256;
    if (c.bs % 64 || c.bs > 256) return MSPLIT_E_ARG;
    c.o = *opts;
    if (out) c.out = *out; else memset(&c.out, 0, sizeof(c.out));
    // double-double roots need their low parts
    if (!starts_only && opts->precision == MSPLIT_DD && (!out->re_lo || !out->im_lo)) return MSPLIT_E_ARG;
    c.cert = !starts_only && (opts->flags & MSPLIT_F_CERTIFY) != 0;
    if (c.cert && (!out->radius || !out->flags)) return MSPLIT_E_ARG;
    c.labels = !(opts->flags & MSPLIT_F_NO_LABEL);
    c.basin = c.cert && (opts->flags & MSPLIT_F_BASIN) && out->basin;
    c.conj = !starts_only && (opts->flags & MSPLIT_F_CONJUGATES) != 0;
    return MSPLIT_OK;
}

// Limits of the plan: the identification radius against FP64 keys, 32-bit
// item indices, one M per call.
int check_plan(const batch_plan &bp)
{
    for (int t = 0; t < bp.T; ++t) {
        // FP64 keys separate the roots only while the identification radius
        // stays well above the FP64 rounding of a root
        if (bp.td[t].p.tau < 0x1p-50) return MSPLIT_E_PRECISION;
    }
    if (bp.n_starts >= ((int64_t)1 << 32)) return MSPLIT_E_UNSUPPORTED;
    // every type of one call shares M (the cis table)
    for (int t = 1; t < bp.T; ++t)
        if (bp.td[t].p.M != bp.td[0].p.M) return MSPLIT_E_ARG;
    return MSPLIT_OK;
}

// Kernel arguments over the workspace carved by c.L (no device work).
void setup_args(batch_call &c, char *ws)
{
    const batch_plan &bp = c.bp;
    c.ws = ws;
    const int T = bp.T;
    c.offs.assign(8 * (T + 1), 0);
    std::copy(bp.seed_offs.begin(), bp.seed_offs.end(), c.offs.begin());
    std::copy(bp.seg_offs.begin(), bp.seg_offs.end(), c.offs.begin() + (T + 1));
    std::copy(bp.start_offs.begin(), bp.start_offs.end(), c.offs.begin() + 2 * (T + 1));
    int64_t *doffs = ws_at<int64_t>(c, c.L.offs);
    batch_args &ba = c.ba;
    ba.types = ws_at<type_desc>(c, c.L.types);
    ba.seed_offs = doffs;
    ba.seg_offs = doffs + (T + 1);
    ba.start_offs = doffs + 2 * (T + 1);
    ba.uniq_offs = doffs + 3 * (T + 1);
    ba.coll_offs = doffs + 4 * (T + 1);
    ba.kept_offs = doffs + 5 * (T + 1);
    ba.surv_offs = doffs + 6 * (T + 1);
    // the FP32 pass's index space (MIXED): the starts of the types it runs on
    int64_t *v32 = c.offs.data() + 7 * (T + 1);
    for (int t = 0; t < T; ++t)
        v32[t + 1] = v32[t] + (c.o.precision == MSPLIT_MIXED && fp32_eligible(bp.td[t].p.el, bp.td[t].p.eN)
                                   ? bp.start_offs[t + 1] - bp.start_offs[t] : 0);
    ba.fp32_offs = doffs + 7 * (T + 1);
    ba.n_fp32 = v32[T];
    // about one evaluation per start: one static chunk per wave, no atomics
    ba.chunk_fp32 = (uint32_t)std::max<int64_t>(64, std::min<int64_t>(4096, (ba.n_fp32 + 8191) / 8192));
    ba.cis = ws_at<double>(c, c.L.cis);
    ba.dphi = 2.0 * M_PI / bp.td[0].p.M;
    ba.x_tip_max = 0.0;
    for (int t = 0; t < T; ++t) ba.x_tip_max = std::max(ba.x_tip_max, bp.td[t].p.x_tip);
    ba.T = T;
    ba.n_seeds = bp.n_seeds;
    ba.n_segs = bp.n_segs;
    ba.n_starts = bp.n_starts;
    ba.chunk_seg = chunk_for(2 * bp.n_segs); // two walks per segment
    ba.chunk_start = chunk_for(bp.n_starts);
    ba.gctr = ws_at<unsigned long long>(c, c.L.gctr);
    ba.ctr = ws_at<unsigned long long>(c, c.L.ctr);
    ba.spread = ws_at<unsigned long long>(c, c.L.spread);
    c.any_tip = false;
    for (int t = 0; t < T; ++t) c.any_tip = c.any_tip || bp.td[t].p.x_tip > 0.0;
    c.out_max = 0;
    for (int t = 0; t < T; ++t) c.out_max += (int64_t)std::min<uint64_t>(bp.td[t].cap, (uint64_t)bp.td[t].p.D);
    c.h.assign((size_t)T * C_NCOUNTERS, 0ull);
}

// Validation, plan and layout; no device work.
int prepare(batch_call &c, const int32_t *ln, int npairs, const msplit_options *opts, void *workspace,
            uint64_t ws_bytes, const msplit_roots *out, const uint64_t *out_offs, const uint64_t *caps,
            bool starts_only)
{
    if (!workspace || !ln) return MSPLIT_E_ARG;
    if (!opts) opts = defaults();
    int r = check_options(c, opts, out, starts_only);
    if (r) return r;
    r = make_batch(ln, npairs, opts, out_offs, caps, c.bp);
    if (r) return r;
    r = check_plan(c.bp);
    if (r) return r;
    c.L = make_layout(c.bp);
    if (ws_bytes < c.L.total) return MSPLIT_E_WORKSPACE;
    setup_args(c, (char *)workspace);
    return MSPLIT_OK;
}

// One item of a streamed split (a chunk of the level line, or a partition of
// the candidates: collect_only, no seeds and no segments) on a given layout.
void plan_item(batch_plan &bp, const plan_t &p, int64_t out_off, uint64_t cap, bool collect_only)
{
    bp.T = 1;
    bp.slot.assign(1, 0);
    bp.td.resize(1);
    type_desc &d = bp.td[0];
    memset(&d, 0, sizeof(d));
    d.p = p;
    if (collect_only) d.p.tip_starts = 0;
    d.out_off = out_off;
    d.cap = cap;
    const int64_t nseed = collect_only ? 0 : p.nseg + 1, nseg = collect_only ? 0 : p.nseg;
    bp.seed_offs = {0, nseed};
    bp.seg_offs = {0, nseg};
    bp.start_offs = {0, p.NS};
    bp.n_seeds = nseed;
    bp.n_segs = nseg;
    bp.n_starts = p.NS;
    bp.n_tip = d.p.tip_starts;
}

// Type descriptors and item offsets to the workspace (the other offset
// tables are set on the device by every call).
hipError_t upload_tables(const batch_call &c, hipStream_t stream)
{
    hipError_t e = hipMemcpyAsync((void *)c.ba.types, c.bp.td.data(), sizeof(type_desc) * c.bp.T,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)c.ba.seed_offs, c.offs.data(), sizeof(int64_t) * c.offs.size(),
                           hipMemcpyHostToDevice, stream);
    return e;
}

// The level line: counters, seeds, walk (events ev[0..2] when non-null).
void enqueue_level_line(const batch_call &c, hipStream_t stream, hipEvent_t *ev)
{
    const batch_plan &bp = c.bp;
    const batch_args &ba = c.ba;
    const int T = bp.T, bs = c.bs;
    cd *seeds = ws_at<cd>(c, c.L.seeds), *starts = ws_at<cd>(c, c.L.starts);
    cd *tip_lo = ws_at<cd>(c, c.L.tip_lo);
    if (ev) (void)hipEventRecord(ev[0], stream);
    k_init_counters<<<blocks_for((int64_t)T * C_NCOUNTERS * CTR_SPREAD + G_NCOUNTERS, 256), 256, 0, stream>>>(
        ba.gctr, ba.ctr, ba.spread, T, ws_at<int64_t>(c, c.L.isz), bp.n_starts);
    k_cis<<<1, 64, 0, stream>>>(bp.td[0].p.M, (double *)ba.cis);
    // seeds: lift from the circle |p_1| = lambda_0
    // (and the descent's first iterates, in roots)
    cd *first = ws_at<cd>(c, c.L.roots);
    k_seeds<<<persistent_blocks(bp.n_seeds, bs), bs, 0, stream>>>(ba, seeds, starts, first);
    if (ev) (void)hipEventRecord(ev[1], stream);
    // level-line walk
    k_walk<<<persistent_blocks(2 * bp.n_segs, bs), bs, 0, stream>>>(ba, seeds, starts, ws_at<uint8_t>(c, c.L.segf),
                                                                    ws_at<walk_mid>(c, c.L.mid), first);
    // segments whose walk failed its phase check: starts lifted again in
    // double-double (the list lives in flag0, free until the descents)
    uint32_t *failed = ws_at<uint32_t>(c, c.L.flag0);
    k_failed_list<<<blocks_for(std::max<int64_t>(bp.n_segs, 1), 256), 256, 0, stream>>>(
        ba, ws_at<uint8_t>(c, c.L.segf), ws_at<walk_mid>(c, c.L.mid), failed);
    k_relift_failed<<<device_cus() * 4, 64, 0, stream>>>(ba, failed, starts, first);
    if (bp.n_tip > 0)
        k_lift_tip_starts<<<blocks_for(bp.n_tip, 64), 64, 0, stream>>>(ba, starts, tip_lo, bp.n_tip, first);
    if (ev) (void)hipEventRecord(ev[2], stream);
}

// The workspace arrays of the root stages, from the layout.
struct pipe_bufs {
    int64_t *isz, *rtile;
    cd *starts, *zs, *zs_lo, *roots, *roots_lo, *tip_lo;
    uint8_t *status, *iters;
    uint32_t *flag0, *pos0, *vals, *vals2, *flag, *pos, *rcounts, *part;
    uint64_t *keys, *keys2;
};

pipe_bufs bufs_of(const batch_call &c)
{
    pipe_bufs B;
    B.isz = ws_at<int64_t>(c, c.L.isz);
    B.rtile = ws_at<int64_t>(c, c.L.rtile);
    B.starts = ws_at<cd>(c, c.L.starts);
    B.status = ws_at<uint8_t>(c, c.L.status);
    B.iters = ws_at<uint8_t>(c, c.L.iters);
    B.flag0 = ws_at<uint32_t>(c, c.L.flag0);
    B.pos0 = ws_at<uint32_t>(c, c.L.pos0);
    B.keys = ws_at<uint64_t>(c, c.L.keys);
    B.keys2 = ws_at<uint64_t>(c, c.L.keys2);
    B.zs = ws_at<cd>(c, c.L.zs);
    B.zs_lo = ws_at<cd>(c, c.L.zs_lo);
    B.roots = ws_at<cd>(c, c.L.roots);
    B.roots_lo = ws_at<cd>(c, c.L.roots_lo);
    B.tip_lo = ws_at<cd>(c, c.L.tip_lo);
    B.vals = ws_at<uint32_t>(c, c.L.vals);
    B.vals2 = ws_at<uint32_t>(c, c.L.vals2);
    B.flag = ws_at<uint32_t>(c, c.L.flag);
    B.pos = ws_at<uint32_t>(c, c.L.pos);
    B.rcounts = ws_at<uint32_t>(c, c.L.counts);
    B.part = ws_at<uint32_t>(c, c.L.part);
    return B;
}

// Where the collection leaves the identified roots, and the buffers it frees.
struct collected {
    cd *uz, *uz_lo;
    uint8_t *uz_dd;
    uint64_t *fkeys;         // the sort's spare key buffer
    uint32_t *svals, *fvals; // its value buffers (free once gathered)
};

// Descents from the starts (MIXED: an FP32 pass first), then the
// double-double route: the routed starts (next to -2, or stalled at the
// FP64 precision floor) descend again from their starting points (the list
// lives in flag0 until the collection).
void enqueue_descents(const batch_call &c, const pipe_bufs &B, hipStream_t stream)
{
    const batch_plan &bp = c.bp;
    const batch_args &ba = c.ba;
    const int bs = c.bs;
    // the FP64 descent continues from roots: the first iterates written with
    // the starts, or the FP32 pass's results after the steps in iters (for
    // the types the FP32 pass runs on; without such a type it is skipped)
    const int nb = persistent_blocks(bp.n_starts, bs);
    // the FP64 descent's queue: every wave starts on its static chunk, the
    // counter hands out the chunks after them
    const unsigned long long q0 = (unsigned long long)nb * (bs / 64) * ba.chunk_start;
    if (c.o.precision == MSPLIT_DD) {
        // every descent in double-double, from its starting point (Section
        // 6.4.3: the high-precision tier for the whole job)
        k_list_all<<<blocks_for(bp.n_starts, 256), 256, 0, stream>>>(ba, B.flag0);
        k_descend_dd<<<device_cus() * 4, 256, 0, stream>>>(ba, B.flag0, B.starts, B.tip_lo, B.roots, B.roots_lo,
                                                           B.status, 1);
        return;
    }
    if (ba.n_fp32 > 0) {
        k_descend32<<<persistent_blocks(ba.n_fp32, bs), bs, 0, stream>>>(ba, B.roots, B.status, B.iters);
        k_set_counter<<<1, 64, 0, stream>>>(&ba.gctr[G_START_NEXT2], q0);
        if (c.any_tip) k_descend<true, true><<<nb, bs, 0, stream>>>(ba, B.roots, B.roots, B.status, B.iters);
        else k_descend<false, true><<<nb, bs, 0, stream>>>(ba, B.roots, B.roots, B.status, B.iters);
    } else {
        k_set_counter<<<1, 64, 0, stream>>>(&ba.gctr[G_START_NEXT], q0);
        if (c.any_tip) k_descend<true, false><<<nb, bs, 0, stream>>>(ba, B.roots, B.roots, B.status, B.iters);
        else k_descend<false, false><<<nb, bs, 0, stream>>>(ba, B.roots, B.roots, B.status, B.iters);
    }
    if (c.any_tip) {
        // (iters holds the descent's tip flags here)
        k_route_tip<<<persistent_blocks(bp.n_starts, ROUTE_ITEMS), 256, 0, stream>>>(ba, B.roots, B.status, B.iters,
                                                                                      B.flag0);
        k_descend_dd<<<device_cus() * 4, 256, 0, stream>>>(ba, B.flag0, B.starts, B.tip_lo, B.roots, B.roots_lo,
                                                           B.status, 0);
    }
}

// nset collection of the descents' results (roots, roots_lo, status):
// local identification (window: PREKEY_WINDOW, or 0 for candidates that are
// already identified), compaction, sort, global identification, and the
// identified roots in the collected index space (type-major, by real part).
collected enqueue_collect(const batch_call &c, const pipe_bufs &B, hipStream_t stream, int window)
{
    const batch_plan &bp = c.bp;
    const batch_args &ba = c.ba;
    const int T = bp.T;
    const unsigned gs = persistent_blocks(bp.n_starts, 256);
    // one tile of PK_TILE starts per block: the blocks balance over the CUs;
    // the survivors go tile-local to the sort's spare buffers, their counts
    // to flag0, whose scan (pos0) places them
    const int64_t pk_tiles = std::max<int64_t>((bp.n_starts + PK_TILE - 1) / PK_TILE, 1);
    k_prekeys<<<pk_tiles, COLLECT_BLOCK, 0, stream>>>(ba, B.roots, B.roots_lo, B.status, B.keys2, B.vals2, B.flag0,
                                                      window);
    scan_u32(B.flag0, B.pos0, B.isz + SZ_PKTILES, pk_tiles, B.part, stream);
    k_compact<<<(unsigned)std::min<int64_t>(pk_tiles, (int64_t)device_cus() * 16), COLLECT_BLOCK, 0, stream>>>(
        ba, B.keys2, B.vals2, B.flag0, B.pos0, B.keys, B.vals);
    uint64_t *skeys = B.keys;
    uint32_t *svals = B.vals;
    sort_pairs(&skeys, &svals, B.keys2, B.vals2, ba.surv_offs, B.rtile, T, KEY_BITS, bp.n_starts, B.rcounts,
               B.isz + SZ_COUNTS, B.part, stream);
    collected C;
    C.fkeys = skeys == B.keys ? B.keys2 : B.keys;
    C.fvals = svals == B.vals ? B.vals2 : B.vals;
    C.svals = svals;
    k_gather<<<gs, 256, 0, stream>>>(ba, B.roots, B.roots_lo, skeys, svals, B.zs, B.zs_lo, B.iters);
    k_mark<<<gs, 256, 0, stream>>>(ba, skeys, B.zs, B.zs_lo, B.iters, B.flag);
    scan_u32(B.flag, B.pos, ba.surv_offs + T, bp.n_starts, B.part, stream);
    k_type_bounds<<<1, 256, 0, stream>>>(ba, B.flag, B.pos);
    // the starts, the descent results and their status are no longer needed
    // once gathered
    C.uz = B.starts;
    C.uz_lo = B.roots_lo;
    C.uz_dd = B.status;
    k_scatter<<<gs, 256, 0, stream>>>(ba, B.flag, B.pos, B.zs, B.zs_lo, B.iters, C.uz, C.uz_lo, C.uz_dd);
    return C;
}

// Classification: period labels (p_n), type Mis(l,n) (q_{l,n}); the kept
// roots go to the caller's slices.  flag0/pos0 and the sort's spare buffers
// are free here.  key_lo > 0: collected roots with a key below key_lo are
// not emitted (the look-back margin of a partition of streamed candidates).
void enqueue_classify(const batch_call &c, const pipe_bufs &B, const collected &C, hipStream_t stream,
                      uint64_t key_lo = 0)
{
    const batch_plan &bp = c.bp;
    const batch_args &ba = c.ba;
    const msplit_roots &out = c.out;
    const int T = bp.T;
    const unsigned gs = persistent_blocks(bp.n_starts, 256);
    uint32_t *keep = B.flag0, *kpos = B.pos0;
    int32_t *cls = (int32_t *)C.fvals;
    uint32_t *hard = C.svals;
    k_classify<<<blocks_for(bp.n_starts, 256), 256, 0, stream>>>(ba, C.uz, C.uz_dd, keep, cls, c.labels ? 1 : 0,
                                                                 hard);
    k_classify_hard<<<device_cus() * 4, 256, 0, stream>>>(ba, C.uz, C.uz_lo, C.uz_dd, keep, cls, hard);
    if (key_lo) k_drop_below<<<gs, 256, 0, stream>>>(ba, C.uz, keep, key_lo);
    scan_u32(keep, kpos, ba.coll_offs + T, bp.n_starts, B.part, stream);
    k_kept_bounds<<<1, 256, 0, stream>>>(ba, keep, kpos);
    k_emit<<<gs, 256, 0, stream>>>(ba, C.uz, C.uz_lo, C.uz_dd, keep, kpos, cls, out.re, out.im, out.re_lo, out.im_lo,
                                   c.labels ? out.period : nullptr, out.preperiod, out.flags);
}

// Certificate, separation and Newton basins over the output index space
// (uniq_offs: min(kept, capacity) roots per type, on the device); n_max
// bounds the number of roots (grid sizes), hard_c is a list of n_max slots.
// p_only: every type is some p_n (the certificate's p_n-only instance).
void enqueue_certify(const batch_args &ba, const msplit_roots &out, bool cert, bool labels, bool basin, int T,
                     int64_t n_max, uint32_t *hard_c, hipStream_t stream, bool p_only = false)
{
    if (n_max <= 0) return;
    if (cert) {
        // one root per thread: the blocks balance over the CUs (a persistent
        // grid held 4 waves per SIMD and ended on its slowest blocks)
        const int32_t *lab = labels ? out.period : nullptr;
        if (out.re_lo && out.im_lo) {
            if (p_only)
                k_certify<true, true><<<blocks_for(n_max, 256), 256, 0, stream>>>(
                    ba, out.re, out.im, out.re_lo, out.im_lo, lab, out.flags, out.radius, hard_c);
            else
                k_certify<true><<<blocks_for(n_max, 256), 256, 0, stream>>>(
                    ba, out.re, out.im, out.re_lo, out.im_lo, lab, out.flags, out.radius, hard_c);
            k_certify_dd<<<device_cus() * 2, 128, 0, stream>>>(ba, out.re, out.im, out.re_lo, out.im_lo, lab,
                                                               out.flags, out.radius, hard_c);
        } else {
            k_certify<false><<<blocks_for(n_max, 256), 256, 0, stream>>>(
                ba, out.re, out.im, nullptr, nullptr, lab, out.flags, out.radius, nullptr);
        }
        // k_separation reads the largest radius of each type
        k_fold_counters<<<fold_blocks(T), 256, 0, stream>>>(ba.ctr, ba.spread, T);
        k_separation<<<persistent_blocks(n_max, 256), 256, 0, stream>>>(ba, out.re, out.im, out.re_lo, out.im_lo,
                                                                        out.radius);
        // Newton basins of the certified roots (Thm proofContract)
        if (basin)
            k_basin<<<persistent_blocks(n_max, 128), 128, 0, stream>>>(ba, out.re, out.im, out.re_lo, out.im_lo,
                                                                       out.flags, out.radius, out.basin);
    } else {
        k_separation<<<persistent_blocks(n_max, 256), 256, 0, stream>>>(ba, out.re, out.im, out.re_lo, out.im_lo,
                                                                        nullptr);
    }
}

// MSPLIT_F_CONJUGATES: every output slice expanded in place to all the roots
// (the conjugate before each non-real root), through a staging copy in
// buffers of the workspace that are free once the roots are emitted (at
// most D/2 + D/16 roots per type, within the NS = 2D + 1 slots of each).
void enqueue_conjugates(const batch_call &c, const pipe_bufs &B, hipStream_t stream)
{
    const batch_plan &bp = c.bp;
    const batch_args &ba = c.ba;
    const msplit_roots &o = c.out;
    conj_stage s;
    s.re = (double *)B.zs;
    s.im = (double *)B.zs + bp.n_starts;
    s.re_lo = (double *)B.zs_lo;
    s.im_lo = (double *)B.zs_lo + bp.n_starts;
    s.radius = (double *)B.keys;
    s.basin = (double *)B.keys2;
    s.period = (int32_t *)B.vals;
    s.preperiod = (int32_t *)B.vals2;
    s.flags = (uint8_t *)B.flag0;
    const unsigned gs = persistent_blocks(c.out_max, 256);
    k_conj_stage<<<gs, 256, 0, stream>>>(ba, o.re, o.im, o.re_lo, o.im_lo, o.period, o.preperiod, o.flags,
                                          c.cert ? o.radius : nullptr, c.basin ? o.basin : nullptr, s, B.flag);
    scan_u32(B.flag, B.pos, ba.uniq_offs + bp.T, std::max<int64_t>(c.out_max, 1), B.part, stream);
    k_conj_scatter<<<gs, 256, 0, stream>>>(ba, s, B.pos, o.re, o.im, o.re_lo, o.im_lo, o.period, o.preperiod,
                                            o.flags, c.cert ? o.radius : nullptr, c.basin ? o.basin : nullptr);
}

// Descents, collection, classification, certificate (events ev[3..6]).
// Every size after the level line is computed and read on the device.
void enqueue_roots(const batch_call &c, hipStream_t stream, hipEvent_t *ev)
{
    const pipe_bufs B = bufs_of(c);
    enqueue_descents(c, B, stream);
    if (ev) (void)hipEventRecord(ev[3], stream);
    const collected C = enqueue_collect(c, B, stream, PREKEY_WINDOW);
    if (ev) (void)hipEventRecord(ev[4], stream);
    enqueue_classify(c, B, C, stream);
    if (ev) (void)hipEventRecord(ev[5], stream);
    bool p_only = true;
    for (const type_desc &d : c.bp.td) p_only = p_only && d.p.l == 0;
    enqueue_certify(c.ba, c.out, c.cert, c.labels, c.basin, c.bp.T, c.out_max, (uint32_t *)C.fkeys, stream, p_only);
    if (c.conj) enqueue_conjugates(c, B, stream);
    k_fold_counters<<<fold_blocks(c.bp.T), 256, 0, stream>>>(c.ba.ctr, c.ba.spread, c.bp.T);
    if (ev) (void)hipEventRecord(ev[6], stream);
}

// Counters to the host (one synchronisation), per-type counts and stats.
int finish(batch_call &c, hipStream_t stream, uint64_t *counts, msplit_stats *stats, call_ctx &ctx, float ms,
           const float *mss)
{
    CHK(hipMemcpyAsync(c.h.data(), c.ba.ctr, sizeof(unsigned long long) * c.h.size(), hipMemcpyDeviceToHost,
                       stream));
    CHK(hipStreamSynchronize(stream));
    const batch_plan &bp = c.bp;
    const int T = bp.T;
    auto H = [&](int t, int slot) { return c.h[(size_t)t * C_NCOUNTERS + slot]; };
    int status_all = MSPLIT_OK;
    for (int t = 0; t < T; ++t) {
        // roots written: the upper half plane, or all of them with their
        // conjugates (MSPLIT_F_CONJUGATES)
        const uint64_t u = H(t, C_KEPT), nr = H(t, C_REAL);
        const uint64_t w = c.conj ? nr + 2 * (u - nr) : u;
        counts[bp.slot[t]] = w;
        if (w > bp.td[t].cap) status_all = MSPLIT_E_CAPACITY;
    }
    if (stats) memset(stats, 0, sizeof(msplit_stats) * T);
    for (int t = 0; t < T; ++t) {
        const int ci = bp.slot[t];
        const plan_t &p = bp.td[t].p;
        const uint64_t uniq = H(t, C_KEPT), nreal = H(t, C_REAL);
        const uint64_t total = nreal + 2 * (uniq - nreal);
        // p_n: all 2^(n-1) roots; q_{l,n}: |Mis(l,n)| (eq. MisCount)
        const uint64_t expected = p.l == 0 ? (uint64_t)p.D : (uint64_t)mis_count(p.l, p.n);
        if (total != expected && status_all == MSPLIT_OK) status_all = MSPLIT_E_INCOMPLETE;
        if (!stats) continue;
        msplit_stats &s = stats[ci];
        s.starts = (uint64_t)p.NS;
        s.converged = H(t, C_CONVERGED);
        s.diverged = H(t, C_DIVERGED);
        s.timeouts = H(t, C_TIMEOUT);
        s.unique = uniq;
        s.n_real = nreal;
        s.total = total;
        s.expected = expected;
        s.missing = expected > total ? expected - total : 0;
        s.phase_fail = H(t, C_PHASE_FAIL) + H(t, C_SEED_FAIL);
        s.certified = H(t, C_CERTIFIED);
        s.label_proven = H(t, C_LABEL);
        s.overlaps = H(t, C_OVERLAP);
        s.steps_lift = H(t, C_STEPS_LIFT);
        s.steps_walk = H(t, C_STEPS_WALK);
        s.steps_desc = H(t, C_STEPS_DESC);
        s.steps_fp32 = H(t, C_STEPS_FP32);
        s.sorted = H(t, C_SURVIVORS);
        s.discarded = H(t, C_UNIQUE) - uniq;
        s.dd_routed = H(t, C_DD_ROUTED);
        s.steps_dd = H(t, C_STEPS_DD);
        s.mark_capped = (int32_t)std::min<uint64_t>(H(t, C_MARK_CAPPED), 0x7fffffff);
        unsigned long long ms_bits = H(t, C_MIN_SEP_BITS), mr_bits = H(t, C_MAX_RAD_BITS);
        unsigned long long mb_bits = H(t, C_MIN_BASIN_BITS);
        memcpy(&s.min_sep, &ms_bits, 8);
        memcpy(&s.max_radius, &mr_bits, 8);
        s.basin = H(t, C_BASIN);
        memcpy(&s.min_basin, &mb_bits, 8);
        if (!s.basin) s.min_basin = 0.0;
        s.ms_device = ms;
        for (int i = 0; i < 6; ++i) s.ms_stage[i] = mss ? mss[i] : 0.f;
    }
    return status_all;
}

// The split of a list of types (in caller order ln[2i], ln[2i+1]); roots of
// type i go to out at out_offs[i] with capacity caps[i].  counts[i] and
// stats[i] are written for every type.  starts_only: stop after the level
// line and copy the starts of the single type to sre / sim.
// timed = false: no events (stage and device times stay 0), for the entry
// point that creates nothing.
int run_batch(const int32_t *ln, int npairs, const msplit_options *opts, void *workspace, uint64_t ws_bytes,
              msplit_roots *out, const uint64_t *out_offs, const uint64_t *caps, uint64_t *counts,
              msplit_stats *stats, void *stream_v, bool starts_only = false, double *sre = nullptr,
              double *sim = nullptr, uint64_t scap = 0, bool timed = true)
{
    for (int i = 0; i < npairs && counts; ++i) counts[i] = 0;
    if (!counts) return MSPLIT_E_ARG;
    if (starts_only && (!sre || !sim || npairs != 1)) return MSPLIT_E_ARG;
    if (stats && npairs > 0) memset(stats, 0, sizeof(msplit_stats) * npairs);
    batch_call c;
    int r = prepare(c, ln, npairs, opts, workspace, ws_bytes, out, out_offs, caps, starts_only);
    if (r) return r;
    if (starts_only && scap < (uint64_t)c.bp.td[0].p.NS) return MSPLIT_E_CAPACITY;
    hipStream_t stream = (hipStream_t)stream_v;
    call_ctx ctx{stats, npairs};
    CHK(upload_tables(c, stream));
    events ev;
    for (int i = 0; i < 7 && timed; ++i) {
        CHK(hipEventCreate(&ev.e[i]));
        ev.made = i + 1;
    }
    enqueue_level_line(c, stream, timed ? ev.e : nullptr);
    CHK(hipGetLastError());
    if (starts_only) {
        const plan_t &p = c.bp.td[0].p;
        k_unzip<<<blocks_for(p.NS, 256), 256, 0, stream>>>(ws_at<cd>(c, c.L.starts), sre, sim, p.NS);
        k_fold_counters<<<fold_blocks(c.bp.T), 256, 0, stream>>>(c.ba.ctr, c.ba.spread, c.bp.T);
        CHK(hipGetLastError());
        CHK(hipMemcpyAsync(c.h.data(), c.ba.ctr, sizeof(unsigned long long) * c.h.size(), hipMemcpyDeviceToHost,
                           stream));
        CHK(hipStreamSynchronize(stream));
        counts[0] = (uint64_t)p.NS;
        float a = 0.f, b = 0.f;
        (void)hipEventElapsedTime(&a, ev.e[0], ev.e[1]);
        (void)hipEventElapsedTime(&b, ev.e[1], ev.e[2]);
        const uint64_t phase_fail = c.h[C_PHASE_FAIL] + c.h[C_SEED_FAIL];
        if (stats) {
            stats->starts = (uint64_t)p.NS;
            stats->phase_fail = phase_fail;
            stats->steps_lift = c.h[C_STEPS_LIFT];
            stats->steps_walk = c.h[C_STEPS_WALK];
            stats->ms_stage[0] = a;
            stats->ms_stage[1] = b;
            stats->ms_device = a + b;
        }
        // a failed walk is repaired by the double-double lift of its starts;
        // a lift that did not converge is not
        return c.h[C_SEED_FAIL] ? MSPLIT_E_INCOMPLETE : MSPLIT_OK;
    }
    enqueue_roots(c, stream, timed ? ev.e : nullptr);
    CHK(hipGetLastError());
    float ms = 0.f, mss[6] = {0, 0, 0, 0, 0, 0};
    if (timed) {
        CHK(hipEventSynchronize(ev.e[6]));
        (void)hipEventElapsedTime(&ms, ev.e[0], ev.e[6]);
        for (int i = 0; i < 6; ++i) (void)hipEventElapsedTime(&mss[i], ev.e[i], ev.e[i + 1]);
    }
    return finish(c, stream, counts, stats, ctx, ms, mss);
}

// --------------------------------------------------------------- streaming
// One type too large for a single pass (stream.hpp): chunks of the level line
// (seeds, walk, descents, identification within the chunk) append their
// roots to an accumulation; partitions of the accumulation by real part are
// identified, classified and emitted in key order; the certificate runs over
// the whole output.  Workspace: the accumulation and its tables, then one
// region shared by the chunk calls, the partition calls and the certificate.
struct stream_plan {
    plan_t p;               // the whole type
    int64_t segs_per_chunk = 0, nchunks = 0, chunk_starts_max = 0;
    int64_t acc_cap = 0;    // accumulated roots
    int64_t part_cap = 0;   // candidates of one partition
    layout LA, LB;          // a chunk call, a partition call
    size_t acc_off = 0, acc_lo_off = 0, acc_dd_off = 0, tab_off = 0, work_off = 0, hard_off = 0, total = 0;
};

constexpr int64_t STREAM_DEFAULT_CHUNK = (int64_t)1 << 28;

bool valid_stream_type(int l, int n) { return n >= 1 && l >= 0 && l != 1 && l + n <= 33; }

// The chunk item c of the level line (segments [c s, c s + s), the last
// chunk up to S with the left end and the tip starts).
plan_t chunk_item(const stream_plan &z, int64_t c)
{
    plan_t q = z.p;
    q.seg0 = c * z.segs_per_chunk;
    const bool last = c == z.nchunks - 1;
    q.nseg = last ? z.p.S - q.seg0 : z.segs_per_chunk;
    q.NS = q.nseg * (z.p.F / z.p.q) + (last ? 1 : 0);
    if (!last) q.tip_starts = 0;
    return q;
}

int make_stream_plan(int l, int n, const msplit_options *o, uint64_t chunk_starts, stream_plan &z)
{
    if (!valid_stream_type(l, n)) return MSPLIT_E_ARG;
    z.p = make_plan(l, n, o);
    const plan_t &p = z.p;
    if (p.tau < 0x1p-50) return MSPLIT_E_PRECISION;
    const int64_t per_seg = p.F / p.q; // starts per segment
    int64_t C = chunk_starts ? (int64_t)chunk_starts : STREAM_DEFAULT_CHUNK;
    if (C < 4 * per_seg || C >= ((int64_t)1 << 31)) return MSPLIT_E_ARG;
    z.segs_per_chunk = std::max<int64_t>(1, C / per_seg);
    z.nchunks = (p.S + z.segs_per_chunk - 1) / z.segs_per_chunk;
    // the last chunk carries the tip starts: fold a short remainder into the
    // chunk before it
    if (z.nchunks > 1 && (p.S - (z.nchunks - 1) * z.segs_per_chunk) * per_seg < 2 * (int64_t)p.tip_starts + 2)
        z.nchunks -= 1;
    if (z.nchunks > STREAM_MAX_CHUNKS) return MSPLIT_E_ARG;
    int64_t longest = 0, longest_seg = 0;
    for (int64_t c = std::max<int64_t>(0, z.nchunks - 2); c < z.nchunks; ++c) {
        longest = std::max(longest, chunk_item(z, c).NS);
        longest_seg = std::max(longest_seg, chunk_item(z, c).nseg);
    }
    z.chunk_starts_max = longest;
    if (longest >= ((int64_t)1 << 32)) return MSPLIT_E_UNSUPPORTED;
    // upper-half roots: D / 2 plus half the real ones (6.3% of the roots of
    // p_16, fewer from there on), and the repeats between chunks (the roots
    // reached from both sides of a chunk boundary)
    z.acc_cap = p.D / 2 + p.D / 16 + 65536;
    z.part_cap = std::max<int64_t>(1 << 16, longest / 2);
    batch_plan ba_, bb_;
    plan_item(ba_, chunk_item(z, z.nchunks - 1), 0, 0, false);
    ba_.n_starts = longest;
    ba_.n_seeds = longest_seg + 1;
    ba_.n_segs = longest_seg;
    z.LA = make_layout(ba_);
    plan_t pb = p;
    pb.NS = z.part_cap;
    plan_item(bb_, pb, 0, 0, true);
    z.LB = make_layout(bb_);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o2 = off; off += align256(bytes); return o2; };
    z.acc_off = take(sizeof(cd) * (size_t)z.acc_cap);
    z.acc_lo_off = take(sizeof(cd) * (size_t)z.acc_cap);
    z.acc_dd_off = take((size_t)z.acc_cap);
    z.tab_off = take(sizeof(int64_t) * (4 * (STREAM_MAX_CHUNKS + 1)) + sizeof(unsigned long long) * STREAM_HIST_BINS);
    z.work_off = off;
    // the certificate's hard list after the partition layout's tables
    z.hard_off = z.LB.seeds;
    const size_t work = std::max({z.LA.total, z.LB.total, z.hard_off + align256(4 * (size_t)z.acc_cap)});
    z.total = z.work_off + work;
    return MSPLIT_OK;
}

struct stream_events {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~stream_events()
    {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
    float ms(int i, int j) const
    {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e[i], e[j]);
        return t;
    }
};

int run_stream(int l, int n, const msplit_options *opts, uint64_t chunk_starts, void *workspace, uint64_t ws_bytes,
               msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream_v)
{
    if (count) *count = 0;
    if (!count || !out || !workspace) return MSPLIT_E_ARG;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (!opts) opts = defaults();
    stream_plan z;
    int r = make_stream_plan(l, n, opts, chunk_starts, z);
    if (r) return r;
    if (ws_bytes < z.total) return MSPLIT_E_WORKSPACE;
    {
        batch_call probe;
        r = check_options(probe, opts, out, false);
        if (r) return r;
        if (probe.conj) return MSPLIT_E_UNSUPPORTED;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    call_ctx ctx{stats, 1};
    char *ws = (char *)workspace;
    cd *acc = (cd *)(ws + z.acc_off), *acc_lo = (cd *)(ws + z.acc_lo_off);
    uint8_t *acc_dd = (uint8_t *)(ws + z.acc_dd_off);
    int64_t *chunk_offs = (int64_t *)(ws + z.tab_off);
    int64_t *sl = chunk_offs + (STREAM_MAX_CHUNKS + 1);
    int64_t *pre = sl + 2 * (STREAM_MAX_CHUNKS + 1);
    unsigned long long *hist = (unsigned long long *)(pre + (STREAM_MAX_CHUNKS + 1));
    char *work = ws + z.work_off;
    const plan_t &p = z.p;
    // stage times from events on the stream, read after each synchronisation
    stream_events ev;
    for (hipEvent_t &x : ev.e) CHK(hipEventCreate(&x));
    float ms_stage[6] = {0, 0, 0, 0, 0, 0};
    auto H = [](const batch_call &c, int slot) { return c.h[slot]; };
    uint64_t sum[C_NCOUNTERS] = {0};
    auto add = [&](const batch_call &c, std::initializer_list<int> slots) {
        for (int s2 : slots) sum[s2] += H(c, s2);
    };
    auto counters_to_host = [&](batch_call &c) -> bool {
        k_fold_counters<<<fold_blocks(1), 256, 0, stream>>>(c.ba.ctr, c.ba.spread, 1);
        return ctx.check(hipGetLastError()) &&
               ctx.check(hipMemcpyAsync(c.h.data(), c.ba.ctr, sizeof(unsigned long long) * c.h.size(),
                                        hipMemcpyDeviceToHost, stream)) &&
               ctx.check(hipStreamSynchronize(stream));
    };

    // chunks of the level line
    std::vector<int64_t> h_chunk_offs(z.nchunks + 1, 0);
    int64_t acc_n = 0;
    for (int64_t ci = 0; ci < z.nchunks; ++ci) {
        batch_call c;
        r = check_options(c, opts, out, false);
        if (r) return r;
        c.cert = c.basin = false;
        plan_item(c.bp, chunk_item(z, ci), 0, 0, false);
        r = check_plan(c.bp);
        if (r) return r;
        c.L = z.LA;
        setup_args(c, work);
        CHK(upload_tables(c, stream));
        enqueue_level_line(c, stream, ev.e); // records e[0], e[1], e[2]
        const pipe_bufs B = bufs_of(c);
        enqueue_descents(c, B, stream);
        CHK(hipEventRecord(ev.e[3], stream));
        const collected C = enqueue_collect(c, B, stream, PREKEY_WINDOW);
        k_append<<<persistent_blocks(c.bp.n_starts, 256), 256, 0, stream>>>(c.ba, C.uz, C.uz_lo, C.uz_dd, acc, acc_lo,
                                                                            acc_dd, acc_n, z.acc_cap);
        CHK(hipEventRecord(ev.e[4], stream));
        if (!counters_to_host(c)) return ctx.err;
        for (int i = 0; i < 4; ++i) ms_stage[i] += ev.ms(i, i + 1);
        const int64_t u = (int64_t)H(c, C_UNIQUE);
        add(c, {C_CONVERGED, C_DIVERGED, C_TIMEOUT, C_PHASE_FAIL, C_SEED_FAIL, C_STEPS_LIFT, C_STEPS_WALK,
                C_STEPS_DESC, C_STEPS_FP32, C_DD_ROUTED, C_STEPS_DD, C_SURVIVORS, C_UNIQUE, C_MARK_CAPPED});
        if (acc_n + u > z.acc_cap) return MSPLIT_E_WORKSPACE;
        acc_n += u;
        h_chunk_offs[ci + 1] = acc_n;
    }

    // partitions of the accumulation by real part: bins of the key histogram,
    // greedily, each with the bin below it (the look-back margin) within the
    // partition capacity
    CHK(hipMemcpyAsync(chunk_offs, h_chunk_offs.data(), sizeof(int64_t) * h_chunk_offs.size(),
                       hipMemcpyHostToDevice, stream));
    k_fill_u64<<<blocks_for(STREAM_HIST_BINS, 256), 256, 0, stream>>>(hist, STREAM_HIST_BINS, 0ull);
    k_key_hist<<<device_cus(), 256, 0, stream>>>(acc, acc_n, hist);
    std::vector<unsigned long long> hh(STREAM_HIST_BINS);
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(hh.data(), hist, sizeof(unsigned long long) * STREAM_HIST_BINS, hipMemcpyDeviceToHost,
                       stream));
    CHK(hipStreamSynchronize(stream));
    // bounds[k]: first bin of partition k; a partition holds its bins and,
    // as its look-back margin, at most the bin before its first
    std::vector<int> bounds = {0};
    {
        uint64_t cur = 0;
        for (int bin = 0; bin < STREAM_HIST_BINS; ++bin) {
            if (bin > bounds.back() && cur + hh[bin] > (uint64_t)z.part_cap) {
                bounds.push_back(bin);
                cur = hh[bin - 1];
            }
            cur += hh[bin];
            if (cur > (uint64_t)z.part_cap) return MSPLIT_E_WORKSPACE; // one bin beyond a partition
        }
        bounds.push_back(STREAM_HIST_BINS);
    }
    const uint64_t win = 1ull + (uint64_t)ceil(p.tau * 0x1p46); // key_window of the identification radius
    int64_t out_n = 0;
    for (size_t k = 0; k + 1 < bounds.size(); ++k) {
        const uint64_t lo = (uint64_t)bounds[k] << STREAM_HIST_SHIFT;
        const uint64_t hi = bounds[k + 1] == STREAM_HIST_BINS ? ~0ull : (uint64_t)bounds[k + 1] << STREAM_HIST_SHIFT;
        const uint64_t lo_w = lo > win ? lo - win : 0;
        CHK(hipEventRecord(ev.e[0], stream));
        k_slices<<<blocks_for(2 * z.nchunks, 256), 256, 0, stream>>>(acc, chunk_offs, (int)z.nchunks, lo_w, hi, sl);
        k_slice_prefix<<<1, 64, 0, stream>>>(sl, (int)z.nchunks, pre);
        int64_t m = 0;
        CHK(hipGetLastError());
        CHK(hipMemcpyAsync(&m, pre + z.nchunks, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        CHK(hipStreamSynchronize(stream));
        if (m > z.part_cap) return MSPLIT_E_WORKSPACE;
        if (m == 0) continue;
        batch_call c;
        r = check_options(c, opts, out, false);
        if (r) return r;
        c.cert = c.basin = false;
        plan_t pk = p;
        pk.NS = m;
        const uint64_t cap = out->capacity > (uint64_t)out_n ? out->capacity - (uint64_t)out_n : 0;
        plan_item(c.bp, pk, out_n, cap, true);
        c.L = z.LB;
        setup_args(c, work);
        CHK(upload_tables(c, stream));
        const pipe_bufs B = bufs_of(c);
        k_init_counters<<<blocks_for((int64_t)C_NCOUNTERS * CTR_SPREAD + G_NCOUNTERS, 256), 256, 0, stream>>>(
            c.ba.gctr, c.ba.ctr, c.ba.spread, 1, B.isz, m);
        k_select<<<persistent_blocks(m, 256), 256, 0, stream>>>(acc, acc_lo, acc_dd, sl, pre, (int)z.nchunks, m,
                                                                B.roots, B.roots_lo, B.status);
        const collected C = enqueue_collect(c, B, stream, 0);
        CHK(hipEventRecord(ev.e[1], stream));
        enqueue_classify(c, B, C, stream, lo);
        CHK(hipEventRecord(ev.e[2], stream));
        if (!counters_to_host(c)) return ctx.err;
        ms_stage[3] += ev.ms(0, 1);
        ms_stage[4] += ev.ms(1, 2);
        const int64_t kept = (int64_t)H(c, C_KEPT);
        add(c, {C_KEPT, C_REAL, C_MARK_CAPPED});
        if ((uint64_t)(out_n + kept) > out->capacity) {
            out_n += kept;
            *count = (uint64_t)out_n;
            return MSPLIT_E_CAPACITY;
        }
        out_n += kept;
    }

    // certificate and separation over the whole output
    batch_call c;
    r = check_options(c, opts, out, false);
    if (r) return r;
    {
        plan_t pc = p;
        pc.NS = 0;
        plan_item(c.bp, pc, 0, (uint64_t)out_n, true);
        c.L = z.LB;
        setup_args(c, work);
        CHK(hipEventRecord(ev.e[0], stream));
        CHK(upload_tables(c, stream));
        const int64_t uo[2] = {0, out_n};
        CHK(hipMemcpyAsync(c.ba.uniq_offs, uo, sizeof(uo), hipMemcpyHostToDevice, stream));
        k_init_counters<<<blocks_for((int64_t)C_NCOUNTERS * CTR_SPREAD + G_NCOUNTERS, 256), 256, 0, stream>>>(
            c.ba.gctr, c.ba.ctr, c.ba.spread, 1, nullptr, 0);
        enqueue_certify(c.ba, c.out, c.cert, c.labels, c.basin, 1, out_n, (uint32_t *)(work + z.hard_off), stream,
                        p.l == 0);
        CHK(hipEventRecord(ev.e[1], stream));
        if (!counters_to_host(c)) return ctx.err;
        ms_stage[5] += ev.ms(0, 1);
    }
    *count = (uint64_t)out_n;
    const uint64_t uniq = (uint64_t)out_n, nreal = sum[C_REAL];
    const uint64_t total = nreal + 2 * (uniq - nreal);
    const uint64_t expected = p.l == 0 ? (uint64_t)p.D : (uint64_t)mis_count(p.l, p.n);
    if (stats) {
        msplit_stats &s = *stats;
        s.starts = (uint64_t)(2 * p.D + 1);
        s.converged = sum[C_CONVERGED];
        s.diverged = sum[C_DIVERGED];
        s.timeouts = sum[C_TIMEOUT];
        s.unique = uniq;
        s.n_real = nreal;
        s.total = total;
        s.expected = expected;
        s.missing = expected > total ? expected - total : 0;
        s.phase_fail = sum[C_PHASE_FAIL] + sum[C_SEED_FAIL];
        s.certified = H(c, C_CERTIFIED);
        s.label_proven = H(c, C_LABEL);
        s.overlaps = H(c, C_OVERLAP);
        s.steps_lift = sum[C_STEPS_LIFT];
        s.steps_walk = sum[C_STEPS_WALK];
        s.steps_desc = sum[C_STEPS_DESC];
        s.steps_fp32 = sum[C_STEPS_FP32];
        s.sorted = sum[C_SURVIVORS];
        s.discarded = sum[C_UNIQUE] - uniq;
        s.dd_routed = sum[C_DD_ROUTED];
        s.steps_dd = sum[C_STEPS_DD];
        s.mark_capped = (int32_t)std::min<uint64_t>(sum[C_MARK_CAPPED], 0x7fffffff);
        unsigned long long ms_bits = H(c, C_MIN_SEP_BITS), mr_bits = H(c, C_MAX_RAD_BITS),
                           mb_bits = H(c, C_MIN_BASIN_BITS);
        memcpy(&s.min_sep, &ms_bits, 8);
        memcpy(&s.max_radius, &mr_bits, 8);
        s.basin = H(c, C_BASIN);
        memcpy(&s.min_basin, &mb_bits, 8);
        if (!s.basin) s.min_basin = 0.0;
        float all = 0.f;
        for (int i = 0; i < 6; ++i) {
            s.ms_stage[i] = ms_stage[i];
            all += ms_stage[i];
        }
        s.ms_device = all;
    }
    return total == expected ? MSPLIT_OK : MSPLIT_E_INCOMPLETE;
}

// A batch captured as one hipGraph: every kernel of a call from the counter
// initialisation to the certificate (the sizes they need are on the
// device, so the capture holds no host round trip).  The type tables are
// uploaded before each launch, outside the graph.
struct graph_state {
    batch_call c;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~graph_state()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Capture the call on the stream (kernels only: the runtime does not time
// events recorded inside a graph, so a launch reports its total time).
hipError_t capture(graph_state &g, hipStream_t stream)
{
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    enqueue_level_line(g.c, stream, nullptr);
    enqueue_roots(g.c, stream, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t e_launch = hipGetLastError();
    e = hipStreamEndCapture(stream, &graph);
    if (e == hipSuccess && e_launch != hipSuccess) e = e_launch;
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return e;
    }
    g.graph = graph;
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        g.graph = nullptr;
        g.exec = nullptr;
    }
    return e;
}

} // namespace

// ===================================================================== C ABI
namespace {

// Address of this device's copy of the static scratch array: looked up once
// per device, with that device current, and kept.
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_at[SCRATCH_DEVICES];

hipError_t scratch_of_device(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_at[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_at[dev] = p;
    }
    *ptr = scratch_at[dev];
    return hipSuccess;
}

} // namespace

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

int msplit_batch_workspace_size(const int32_t *ln_pairs, int npairs, const msplit_options *opts, uint64_t *bytes)
{
    if (!ln_pairs || npairs <= 0 || !bytes) return MSPLIT_E_ARG;
    if (!opts) opts = defaults();
    batch_plan bp;
    int r = make_batch(ln_pairs, npairs, opts, nullptr, nullptr, bp);
    if (r) return r;
    *bytes = make_layout(bp).total;
    return MSPLIT_OK;
}

int msplit_workspace_size(int l, int n, const msplit_options *opts, uint64_t *bytes)
{
    if (!bytes || !valid_type(l, n)) return MSPLIT_E_ARG;
    const int32_t ln[2] = {l, n};
    return msplit_batch_workspace_size(ln, 1, opts, bytes);
}

int msplit_hyperbolic(int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                      msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream)
{
    if (count) *count = 0;
    if (!count || !out) return MSPLIT_E_ARG;
    const int32_t ln[2] = {0, n};
    const uint64_t off = 0, cap = out->capacity;
    return run_batch(ln, 1, opts, workspace, workspace_bytes, out, &off, &cap, count, stats, stream);
}

int msplit_hyperbolic_static(int n, const msplit_options *opts, msplit_roots *out, uint64_t *count,
                             msplit_stats *stats, void *stream)
{
    if (count) *count = 0;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (!count || !out) return MSPLIT_E_ARG;
    uint64_t need = 0;
    int r = msplit_workspace_size(0, n, opts, &need);
    if (r) return r;
    if (need > MSPLIT_STATIC_SCRATCH_BYTES) return MSPLIT_E_WORKSPACE;
    void *ws = nullptr;
    const hipError_t e = scratch_of_device(&ws);
    if (e != hipSuccess) {
        if (stats) stats->hip_error = (int32_t)e;
        return MSPLIT_E_DEVICE;
    }
    const int32_t ln[2] = {0, n};
    const uint64_t off = 0, cap = out->capacity;
    return run_batch(ln, 1, opts, ws, MSPLIT_STATIC_SCRATCH_BYTES, out, &off, &cap, count, stats, stream, false,
                     nullptr, nullptr, 0, false);
}

int msplit_misiurewicz(int l, int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                       msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream)
{
    if (count) *count = 0;
    if (!count || !out || l < 2) return MSPLIT_E_ARG;
    const int32_t ln[2] = {l, n};
    const uint64_t off = 0, cap = out->capacity;
    return run_batch(ln, 1, opts, workspace, workspace_bytes, out, &off, &cap, count, stats, stream);
}

int msplit_starts(int l, int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes, double *re,
                  double *im, uint64_t capacity, uint64_t *count, msplit_stats *stats, void *stream)
{
    if (count) *count = 0;
    if (!count) return MSPLIT_E_ARG;
    const int32_t ln[2] = {l, n};
    return run_batch(ln, 1, opts, workspace, workspace_bytes, nullptr, nullptr, nullptr, count, stats, stream, true,
                     re, im, capacity);
}

int msplit_batch(const int32_t *ln_pairs, int npairs, const msplit_options *opts, void *workspace,
                 uint64_t workspace_bytes, msplit_roots *out, const uint64_t *caps, uint64_t *counts,
                 msplit_stats *stats, void *stream)
{
    if (!ln_pairs || npairs <= 0 || !out || !caps || !counts) return MSPLIT_E_ARG;
    std::vector<uint64_t> offs(npairs, 0);
    for (int i = 1; i < npairs; ++i) offs[i] = offs[i - 1] + caps[i - 1];
    return run_batch(ln_pairs, npairs, opts, workspace, workspace_bytes, out, offs.data(), caps, counts, stats,
                     stream);
}

int msplit_stream_workspace_size(int l, int n, const msplit_options *opts, uint64_t chunk_starts, uint64_t *bytes)
{
    if (!bytes) return MSPLIT_E_ARG;
    stream_plan z;
    int r = make_stream_plan(l, n, opts ? opts : defaults(), chunk_starts, z);
    if (r) return r;
    *bytes = z.total;
    return MSPLIT_OK;
}

int msplit_split_streamed(int l, int n, const msplit_options *opts, uint64_t chunk_starts, void *workspace,
                          uint64_t workspace_bytes, msplit_roots *out, uint64_t *count, msplit_stats *stats,
                          void *stream)
{
    return run_stream(l, n, opts, chunk_starts, workspace, workspace_bytes, out, count, stats, stream);
}

int msplit_certify(int l, int n, msplit_roots *roots, uint64_t count, void *workspace, uint64_t workspace_bytes,
                   msplit_stats *stats, void *stream_v)
{
    if (!roots || !workspace || !roots->re || !roots->im || !roots->flags || !roots->radius) return MSPLIT_E_ARG;
    if (!valid_type(l, n)) return MSPLIT_E_ARG;
    if (stats) memset(stats, 0, sizeof(*stats));
    // one type, the candidates as its unique roots
    batch_plan bp;
    const int32_t ln[2] = {l, n};
    const uint64_t off = 0;
    int r = make_batch(ln, 1, defaults(), &off, &count, bp);
    if (r) return r;
    const size_t ctr_bytes = align256(sizeof(unsigned long long) * (G_NCOUNTERS + C_NCOUNTERS));
    const size_t spread_bytes = align256(sizeof(unsigned long long) * C_NCOUNTERS * CTR_SPREAD);
    const size_t need = ctr_bytes + spread_bytes + align256(sizeof(type_desc)) + align256(sizeof(int64_t) * 8);
    static_assert(align256(sizeof(unsigned long long) * (G_NCOUNTERS + C_NCOUNTERS)) +
                          align256(sizeof(unsigned long long) * C_NCOUNTERS * CTR_SPREAD) +
                          align256(sizeof(type_desc)) + align256(sizeof(int64_t) * 8) <=
                      MSPLIT_CERTIFY_WORKSPACE,
                  "certify workspace");
    if (workspace_bytes < need) return MSPLIT_E_WORKSPACE;
    hipStream_t stream = (hipStream_t)stream_v;
    call_ctx ctx{stats, 1};
    char *ws = (char *)workspace;
    unsigned long long *gctr = (unsigned long long *)ws;
    unsigned long long *ctr = gctr + G_NCOUNTERS;
    unsigned long long *spread = (unsigned long long *)(ws + ctr_bytes);
    type_desc *dtypes = (type_desc *)(ws + ctr_bytes + spread_bytes);
    int64_t *doffs = (int64_t *)((char *)dtypes + align256(sizeof(type_desc)));
    const int64_t uo[2] = {0, (int64_t)count};
    CHK(hipMemcpyAsync(dtypes, bp.td.data(), sizeof(type_desc), hipMemcpyHostToDevice, stream));
    CHK(hipMemcpyAsync(doffs, uo, sizeof(uo), hipMemcpyHostToDevice, stream));
    batch_args ba;
    memset(&ba, 0, sizeof(ba));
    ba.types = dtypes;
    ba.seed_offs = ba.seg_offs = ba.start_offs = ba.uniq_offs = doffs;
    ba.T = 1;
    ba.gctr = gctr;
    ba.ctr = ctr;
    ba.spread = spread;
    k_init_counters<<<blocks_for((int64_t)C_NCOUNTERS * CTR_SPREAD + G_NCOUNTERS, 256), 256, 0, stream>>>(
        gctr, ctr, spread, 1, nullptr, 0);
    if (count) {
        k_certify<false><<<blocks_for((int64_t)count, 256), 256, 0, stream>>>(
            ba, roots->re, roots->im, roots->re_lo, roots->im_lo, roots->period, roots->flags, roots->radius,
            nullptr);
        k_fold_counters<<<fold_blocks(1), 256, 0, stream>>>(ctr, spread, 1);
        k_separation<<<persistent_blocks((int64_t)count, 256), 256, 0, stream>>>(
            ba, roots->re, roots->im, roots->re_lo, roots->im_lo, roots->radius);
        if (roots->basin)
            k_basin<<<persistent_blocks((int64_t)count, 128), 128, 0, stream>>>(
                ba, roots->re, roots->im, roots->re_lo, roots->im_lo, roots->flags, roots->radius, roots->basin);
    }
    k_fold_counters<<<fold_blocks(1), 256, 0, stream>>>(ctr, spread, 1);
    CHK(hipGetLastError());
    unsigned long long h[C_NCOUNTERS];
    CHK(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream));
    CHK(hipStreamSynchronize(stream));
    if (stats) {
        stats->certified = h[C_CERTIFIED];
        stats->label_proven = h[C_LABEL];
        stats->overlaps = h[C_OVERLAP];
        memcpy(&stats->min_sep, &h[C_MIN_SEP_BITS], 8);
        memcpy(&stats->max_radius, &h[C_MAX_RAD_BITS], 8);
        stats->basin = h[C_BASIN];
        memcpy(&stats->min_basin, &h[C_MIN_BASIN_BITS], 8);
        if (!stats->basin) stats->min_basin = 0.0;
    }
    return MSPLIT_OK;
}

struct msplit_graph {
    graph_state g;
};

int msplit_batch_graph(const int32_t *ln_pairs, int npairs, const msplit_options *opts, void *workspace,
                       uint64_t workspace_bytes, msplit_roots *out, const uint64_t *caps, void *stream_v,
                       msplit_graph **graph)
{
    if (graph) *graph = nullptr;
    if (!ln_pairs || npairs <= 0 || !out || !caps || !graph || !stream_v) return MSPLIT_E_ARG;
    std::vector<uint64_t> offs(npairs, 0);
    for (int i = 1; i < npairs; ++i) offs[i] = offs[i - 1] + caps[i - 1];
    msplit_graph *G = new (std::nothrow) msplit_graph;
    if (!G) return MSPLIT_E_ARG;
    graph_state &g = G->g;
    int r = prepare(g.c, ln_pairs, npairs, opts, workspace, workspace_bytes, out, offs.data(), caps, false);
    if (r) {
        delete G;
        return r;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    hipError_t e = hipEventCreate(&g.e0);
    if (e == hipSuccess) e = hipEventCreate(&g.e1);
    if (e == hipSuccess) e = capture(g, stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete G;
        return MSPLIT_E_DEVICE;
    }
    *graph = G;
    return MSPLIT_OK;
}

int msplit_graph_launch(msplit_graph *G, uint64_t *counts, msplit_stats *stats, void *stream_v)
{
    if (!G || !counts || !stream_v) return MSPLIT_E_ARG;
    graph_state &g = G->g;
    const int T = g.c.bp.T;
    for (int i = 0; i < T; ++i) counts[i] = 0;
    hipStream_t stream = (hipStream_t)stream_v;
    call_ctx ctx{stats, T};
    CHK(upload_tables(g.c, stream));
    CHK(hipEventRecord(g.e0, stream));
    CHK(hipGraphLaunch(g.exec, stream));
    CHK(hipEventRecord(g.e1, stream));
    CHK(hipEventSynchronize(g.e1));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, g.e0, g.e1));
    return finish(g.c, stream, counts, stats, ctx, ms, nullptr);
}

void msplit_graph_destroy(msplit_graph *G) { delete G; }

} // extern "C"
