// common.hpp -- device helpers shared by the kernels of libmsplit (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msplit {

// ---------------------------------------------------------------- complex
struct cd { double re, im; };
struct cf { float re, im; };

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ double cabs2(cd a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabs(cd a) { return sqrt(cabs2(a)); }
// a / b through one reciprocal of |b|^2, after scaling both by the same
// power of two so that |b|^2 cannot overflow or underflow: near escaping
// iterates |P'| exceeds 1e154 while |P| does not, and an unscaled |P'|^2
// would turn the Newton step P/P' into an exact zero.  (The same common
// factor cancellation the paper applies to its FP80 steps, Section 6.3.2.)
// b = 0 or a non-finite b yields a non-finite quotient.
__device__ __forceinline__ cd cdiv(cd a, cd b)
{
    const double m = fmax(fabs(b.re), fabs(b.im));
    const double s = ldexp(1.0, -ilogb(m));
    const cd bs = {b.re * s, b.im * s}, as = {a.re * s, a.im * s};
    const double r = 1.0 / cabs2(bs);
    return {(as.re * bs.re + as.im * bs.im) * r, (as.im * bs.re - as.re * bs.im) * r};
}
__device__ __forceinline__ bool cfinite(cd a) { return isfinite(a.re) && isfinite(a.im); }

// a / b for the Newton updates: the hardware reciprocal of |b|^2 refined by
// one Newton-Raphson step (relative error ~1e-16: the iteration needs no
// correctly rounded quotient), with the power-of-two scaling of cdiv only
// when |b|^2 leaves [2^-1000, 2^1000].
__device__ __forceinline__ cd cdiv_fast(cd a, cd b)
{
    const double d2 = cabs2(b);
    if (!(d2 >= 0x1p-1000 && d2 <= 0x1p1000)) return cdiv(a, b);
    double r = __builtin_amdgcn_rcp(d2);
    r = fma(fma(-d2, r, 1.0), r, r);
    return {(a.re * b.re + a.im * b.im) * r, (a.im * b.re - a.re * b.im) * r};
}

// Approximation u(w) of log w for the Newton iteration on log P (the step
// z += u(T/P) P/P').  It only has to be exact at the fixed point w = 1 and
// close enough elsewhere to keep the iteration contracting, so no
// transcendental function is evaluated:
//   |w - 1| < 1/8 : log1p series up to v^7 (relative error < 3e-7);
//   |y| <= 0.8    : 2 atanh(y) = 2 (y + y^3/3 + ... + y^9/9), y = (w-1)/(w+1)
//                   (relative error about 1e-3 at |y| = 0.67);
//   otherwise     : u = w - 1, i.e. the plain Newton map with target,
//                   z += (T - P)/P' (Section 4.1, L(P; z, T)).
__device__ __forceinline__ cd clog_near1(cd w)
{
    const cd v = {w.re - 1.0, w.im};
    const double a2 = cabs2(v);
    if (a2 < (1.0 / 64.0)) {
        // v - v^2/2 + v^3/3 - ... - v^6/6 + v^7/7 (Horner)
        cd acc = {1.0 / 7.0, 0.0};
        acc = cadd(cmul(acc, v), {-1.0 / 6.0, 0.0});
        acc = cadd(cmul(acc, v), {0.2, 0.0});
        acc = cadd(cmul(acc, v), {-0.25, 0.0});
        acc = cadd(cmul(acc, v), {1.0 / 3.0, 0.0});
        acc = cadd(cmul(acc, v), {-0.5, 0.0});
        acc = cadd(cmul(acc, v), {1.0, 0.0});
        return cmul(acc, v);
    }
    const cd y = cdiv(v, {w.re + 1.0, w.im});
    if (cabs2(y) > 0.64) return v;
    const cd y2 = cmul(y, y);
    cd acc = {1.0 / 9.0, 0.0};
    acc = cadd(cmul(acc, y2), {1.0 / 7.0, 0.0});
    acc = cadd(cmul(acc, y2), {0.2, 0.0});
    acc = cadd(cmul(acc, y2), {1.0 / 3.0, 0.0});
    acc = cadd(cmul(acc, y2), {1.0, 0.0});
    const cd r = cmul(acc, y);
    return {2.0 * r.re, 2.0 * r.im};
}

// The approximation of log w in the level-line walk, without branches (the
// lanes of a wave sit at every distance from their targets): the log1p
// series to four terms, v - v^2/2 + v^3/3 - v^4/4, v = w - 1 (error about
// |v|^5 / 5: 6e-3 at |v| = 1/2, 2e-5 at |v| = 1/4), exact with slope 1 at
// w = 1; beyond |v| = 1/2 (a prediction gone far) u = v, the plain Newton
// map with target.  The walk aims each update from the nearer target, so
// |v| stays below 1/4 at almost every evaluation.
__device__ __forceinline__ cd clog_series(cd w)
{
    const cd v = {w.re - 1.0, w.im};
    cd acc = {v.re * -0.25 + 1.0 / 3.0, v.im * -0.25};
    acc = cadd(cmul(acc, v), {-0.5, 0.0});
    acc = cadd(cmul(acc, v), {1.0, 0.0});
    const cd u = cmul(acc, v);
    return cabs2(v) <= 0.25 ? u : v;
}

// ---------------------------------------------------------------- orbit
// Critical orbit p_0 = 0, p_{k+1} = p_k^2 + c and p'_{k+1} = 2 p_k p'_k + 1
// (Section 2, eq. defFundMap; the derivative is the chain rule of the same
// recurrence).  q_{l,n} = p_{l+n} - p_l; l = 0 gives p_n since p_0 = 0.
template <typename T>
struct orbit_state { T zr, zi, dr, di; };

template <typename T>
__device__ __forceinline__ void orbit_step(orbit_state<T> &s, T cr, T ci)
{
    // dz <- 2 z dz + 1 with the old z, then z <- z^2 + c
    T tr = s.zr * s.dr - s.zi * s.di;
    T ti = s.zr * s.di + s.zi * s.dr;
    T nr = s.zr * s.zr - s.zi * s.zi + cr;
    T ni = (s.zr + s.zr) * s.zi + ci;
    s.dr = tr + tr + T(1);
    s.di = ti + ti;
    s.zr = nr;
    s.zi = ni;
}

// The evaluation runs the same recurrence on u_k = 2 p_k (a scaling by 2,
// exact in binary floating point): u_{k+1} = u_k^2 / 2 + 2c and
// p'_{k+1} = u_k p'_k + 1.  Written with fused multiply-adds, one step is 2
// multiplications and 6 FMAs -- 8 vector instructions for the 16 real flops
// of the plain step, the FMA peak rate -- against 11 for the plain form
// (which needs 2 z and 2 (z dz) as separate doublings).
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
struct orbit2_state { T ur, ui, dr, di; }; // u = 2 p_k, d = p_k'

template <typename T>
__device__ __forceinline__ void orbit2_step(orbit2_state<T> &s, T c4r, T c2i)
{
    const T ur = T(0.5) * fmat(s.ur, s.ur, fmat(-s.ui, s.ui, c4r));
    const T ui = fmat(s.ur, s.ui, c2i);
    const T dr = fmat(s.ur, s.dr, fmat(-s.ui, s.di, T(1)));
    const T di = fmat(s.ur, s.di, s.ui * s.dr);
    s.ur = ur;
    s.ui = ui;
    s.dr = dr;
    s.di = di;
}

// P = q_{l,n}(c), dP = q_{l,n}'(c), N = l + n >= 1 (l = 0: p_N).  The orbit
// starts from its first iterate, p_1 = c and p_1' = 1 (exact), so an
// evaluation of order N takes N - 1 steps; p_N needs no subtraction.  A
// negative l selects a sum: P = z_N + z_{-l}, the simplified polynomial
// s_{a+1,n} = p_{a+n} + p_a (eq. polySimple) for l = -a, N = a + n.
template <typename T, typename C>
__device__ __forceinline__ void eval_q_t(int l, int N, C c, C &P, C &dP)
{
    const T c4r = T(4) * c.re, c2i = T(2) * c.im;
    orbit2_state<T> s = {T(2) * c.re, c2i, T(1), T(0)};
    if (l == 0) {
        // N - 1 steps: an odd one first, then pairs (a loop of two steps with
        // no remainder: no register copies between the loop and the rest)
        if ((N - 1) & 1) orbit2_step(s, c4r, c2i);
        for (int j = (N - 1) >> 1; j > 0; --j) {
            orbit2_step(s, c4r, c2i);
            orbit2_step(s, c4r, c2i);
        }
        P = {T(0.5) * s.ur, T(0.5) * s.ui};
        dP = {s.dr, s.di};
        return;
    }
    const int la = l < 0 ? -l : l;
    int k = 1;
    for (; k < la; ++k) orbit2_step(s, c4r, c2i);
    // the subtracted term, negated for the sum (no sign kept live in the loop)
    orbit2_state<T> sl = s;
    if (l < 0) sl = {-s.ur, -s.ui, -s.dr, -s.di};
#pragma unroll 2
    for (; k < N; ++k) orbit2_step(s, c4r, c2i);
    P = {T(0.5) * (s.ur - sl.ur), T(0.5) * (s.ui - sl.ui)};
    dP = {s.dr - sl.dr, s.di - sl.di};
}

__device__ __forceinline__ void eval_q(int l, int N, cd c, cd &P, cd &dP) { eval_q_t<double>(l, N, c, P, dP); }

// Same evaluation; when every active lane of the wave has the same (l, N)
// the trip counts are made wave-uniform (scalar loop control).
__device__ __forceinline__ void eval_q_wave(int l, int N, cd c, cd &P, cd &dP)
{
    const int l0 = __builtin_amdgcn_readfirstlane(l), N0 = __builtin_amdgcn_readfirstlane(N);
    if (__ballot(l != l0 || N != N0) == 0) eval_q(l0, N0, c, P, dP);
    else eval_q(l, N, c, P, dP);
}

__device__ __forceinline__ void eval_q_f32(int l, int N, cf c, cf &P, cf &dP) { eval_q_t<float>(l, N, c, P, dP); }

// ---------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Per-wave work queue over the items [0, n): the wave owns the index range
// [next, end), taken `chunk` items at a time (one atomic per chunk instead
// of one per item).  Requests to one address serialise -- about 16 ns each
// across the XCDs of the chip, so the 8192 waves of a persistent grid asking
// at once would wait up to 130 us -- hence wave w of the grid (W waves)
// starts with the chunk [w chunk, (w + 1) chunk) without an atomic, and the
// counter hands out the chunks from W chunk on.  A plain read of the counter
// first spares the atomic once the items are exhausted (the counter only
// grows, so a stale value never ends a queue early).  The two fields are
// wave-uniform: every lane holds the same copy and applies the same updates.
// Lanes with need get distinct indices (>= n: no work left).  chunk >= 64.
struct wave_queue { uint64_t next, end; };

__global__ void k_set_counter(unsigned long long *counter, unsigned long long v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = v;
}

__device__ __forceinline__ uint64_t grid_waves() { return ((uint64_t)gridDim.x * blockDim.x) >> 6; }

__device__ __forceinline__ wave_queue wave_queue_start(uint64_t chunk)
{
    // wave-uniform (scalar registers)
    const uint32_t wb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wb;
    return {w * chunk, (w + 1) * chunk};
}

// value of `x` in lane `lane` as a wave-uniform (scalar) value
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t x, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// The plain form: every chunk from the counter as it stands.  The FP64
// descent uses it with the static first chunk (wave_queue_start) and a
// counter the host sets to W chunk beforehand (k_set_counter): computing
// that base in the kernel costs it two VGPRs, past its 64 (one wave per SIMD
// less).
__device__ __forceinline__ uint64_t wave_take_plain(wave_queue &q, unsigned long long *counter, uint64_t chunk,
                                                    bool need)
{
    const unsigned long long mask = __ballot(need);
    uint64_t idx = ~0ull;
    if (!mask) return idx;
    const uint32_t cnt = (uint32_t)__popcll(mask);
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    const uint64_t avail = q.end - q.next;
    if (avail < cnt) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        unsigned long long b = 0;
        if (lane_id() == leader) b = atomicAdd(counter, (unsigned long long)chunk);
        const uint64_t base = read_lane_u64(b, leader);
        if (need) idx = rank < avail ? q.next + rank : base + (rank - avail);
        q.next = base + (cnt - avail);
        q.end = base + chunk;
    } else {
        if (need) idx = q.next + rank;
        q.next += cnt;
    }
    return idx;
}

__device__ __forceinline__ uint64_t wave_take(wave_queue &q, unsigned long long *counter, uint64_t chunk, uint64_t n,
                                              bool need)
{
    const unsigned long long mask = __ballot(need);
    uint64_t idx = ~0ull;
    if (!mask) return idx;
    const uint32_t cnt = (uint32_t)__popcll(mask);
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    const uint64_t avail = q.end - q.next;
    if (avail < cnt) {
        const uint64_t first = grid_waves() * chunk; // counter value 0
        const int leader = __ffsll((unsigned long long)mask) - 1;
        unsigned long long b = 0;
        if (lane_id() == leader) {
            const unsigned long long seen = __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            b = first + seen >= n ? ~0ull : first + atomicAdd(counter, (unsigned long long)chunk);
        }
        const uint64_t base = read_lane_u64(b, leader);
        if (base == ~0ull) { // no chunk left: the lanes past this range get n
            if (need) idx = rank < avail ? q.next + rank : n;
            q.next = q.end;
        } else {
            if (need) idx = rank < avail ? q.next + rank : base + (rank - avail);
            q.next = base + (cnt - avail);
            q.end = base + chunk;
        }
    } else {
        if (need) idx = q.next + rank;
        q.next += cnt;
    }
    return idx;
}

// Segmented wave reduction: every lane holds (key, value); for each distinct
// key >= 0 present in the wave one lane applies op to the slot of that key
// with the reduction of the values of the lanes holding it.  A wave holds one
// or two keys in practice, so this costs one or two butterfly reductions and
// one atomic per key -- never one atomic per lane on a shared address (those
// serialise in the L2 atomic unit).  All lanes of the wave must call it.
enum red_op { RED_ADD, RED_MAX, RED_MIN };

template <red_op OP>
__device__ __forceinline__ unsigned long long red_combine(unsigned long long a, unsigned long long b)
{
    if (OP == RED_ADD) return a + b;
    if (OP == RED_MAX) return a > b ? a : b;
    return a < b ? a : b;
}

template <red_op OP>
__device__ __forceinline__ void wave_reduce_by_key(unsigned long long *base, int stride, int slot, int key,
                                                   unsigned long long value)
{
    const unsigned long long ident = (OP == RED_MIN) ? ~0ull : 0ull;
    bool pending = key >= 0;
    while (true) {
        const unsigned long long pend = __ballot(pending);
        if (!pend) break;
        const int leader = __ffsll(pend) - 1;
        const int k = __shfl(key, leader);
        const bool mine = pending && key == k;
        unsigned long long v = mine ? value : ident;
        for (int off = 32; off > 0; off >>= 1) v = red_combine<OP>(v, __shfl_xor(v, off));
        if (lane_id() == leader && v != ident) {
            unsigned long long *dst = base + (int64_t)k * stride + slot;
            if (OP == RED_ADD) atomicAdd(dst, v);
            else if (OP == RED_MAX) atomicMax(dst, v);
            else atomicMin(dst, v);
        }
        if (mine) pending = false;
    }
}

// Four sums under one key per lane (same contract as wave_reduce_by_key):
// one butterfly pass per distinct key, four atomics by its first lane into
// base[key * stride + slot_i].
__device__ __forceinline__ void wave_add4_by_key(unsigned long long *base, int stride, int key, const int slot[4],
                                                 const uint32_t v[4])
{
    bool pending = key >= 0;
    while (true) {
        const unsigned long long pend = __ballot(pending);
        if (!pend) break;
        const int leader = __ffsll(pend) - 1;
        const int k = __builtin_amdgcn_readlane(key, leader);
        const bool mine = pending && key == k;
        unsigned long long a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            unsigned long long x = mine ? (unsigned long long)v[i] : 0ull;
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            a[i] = x;
        }
        if (lane_id() == leader) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (a[i]) atomicAdd(base + (int64_t)k * stride + slot[i], a[i]);
        }
        if (mine) pending = false;
    }
}

// Append value to list for every lane with take: one atomic per wave on the
// length counter, lanes in lane order.  All lanes of the wave must call it.
__device__ __forceinline__ void wave_append(uint32_t *list, unsigned long long *count, bool take, uint32_t value)
{
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int leader = __ffsll(mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
    base = read_lane_u64(base, leader);
    if (take) {
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        list[base + rank] = value;
    }
}

// Order-preserving map of a double onto uint64 (sort key).
__device__ __forceinline__ uint64_t orderable(double x)
{
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

} // namespace msplit

namespace msplit {
__device__ __forceinline__ void eval_q_f32_wave(int l, int N, cf c, cf &P, cf &dP)
{
    const int l0 = __builtin_amdgcn_readfirstlane(l), N0 = __builtin_amdgcn_readfirstlane(N);
    if (__ballot(l != l0 || N != N0) == 0) eval_q_f32(l0, N0, c, P, dP);
    else eval_q_f32(l, N, c, P, dP);
}
} // namespace msplit
