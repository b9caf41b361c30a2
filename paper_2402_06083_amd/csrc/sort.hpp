// sort.hpp -- exclusive scan and segmented LSD radix sort whose sizes live in
// device memory, so that a whole split runs without a host round trip (and
// can be captured in a graph).  Reduce-then-scan throughout: no kernel waits
// on another block's progress.
#pragma once
#include "common.hpp"

namespace msplit {

constexpr int SC_BLOCK = 256;           // threads per block (4 waves)
constexpr int SC_ROWS = 16;             // rows of SC_BLOCK items per tile
constexpr int SC_TILE = SC_BLOCK * SC_ROWS;
constexpr int MAX_SEGS = 256;           // segments of one sort (one per type)

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive prefix sum over a block of SC_BLOCK threads, and the block total.
// Every thread of the block must call it (two barriers).
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *wsum, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_sum(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int i = 0; i < SC_BLOCK / 64; ++i) before += i < w ? wsum[i] : 0u;
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return before + inc - v;
}

// ------------------------------------------------------------------ scan
// out[i] = in[0] + ... + in[i-1] for i < *n (in == out allowed).  Two
// launches of the same grid; block b owns the tiles [b k, (b + 1) k) of
// SC_TILE values, k = ceil(tiles / grid): the first launch writes the sum of
// each block's values to part[b], the second adds up part[0..b) (at most one
// value per block of the grid) and rescans its tiles in order, carrying the
// running sum.  part holds gridDim.x entries.
__device__ __forceinline__ void scan_range(int64_t tiles, int64_t &t0, int64_t &t1)
{
    const int64_t k = (tiles + gridDim.x - 1) / gridDim.x;
    t0 = min((int64_t)blockIdx.x * k, tiles);
    t1 = min(t0 + k, tiles);
}

__global__ void __launch_bounds__(SC_BLOCK) k_scan_reduce(const uint32_t *in, const int64_t *n_dev, uint32_t *part)
{
    __shared__ uint32_t wsum[4];
    const int64_t n = *n_dev;
    int64_t t0, t1;
    scan_range((n + SC_TILE - 1) / SC_TILE, t0, t1);
    uint32_t s = 0;
    for (int64_t i = t0; i < t1; ++i) {
        const int64_t base = i * SC_TILE;
#pragma unroll
        for (int k = 0; k < SC_ROWS; ++k) {
            const int64_t g = base + (int64_t)k * SC_BLOCK + threadIdx.x;
            s += g < n ? in[g] : 0u;
        }
    }
    uint32_t tot;
    (void)block_excl_sum(s, wsum, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SC_BLOCK) k_scan_down(const uint32_t *in, uint32_t *out, const int64_t *n_dev,
                                                        const uint32_t *part)
{
    __shared__ uint32_t wsum[4];
    const int64_t n = *n_dev;
    int64_t t0, t1;
    scan_range((n + SC_TILE - 1) / SC_TILE, t0, t1);
    if (t0 >= t1) return; // (block-uniform)
    uint32_t pre = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += SC_BLOCK) pre += part[k];
    uint32_t carry;
    (void)block_excl_sum(pre, wsum, carry);
    for (int64_t i = t0; i < t1; ++i) {
        const int64_t base = i * SC_TILE;
        uint32_t v[SC_ROWS];
#pragma unroll
        for (int k = 0; k < SC_ROWS; ++k) {
            const int64_t g = base + (int64_t)k * SC_BLOCK + threadIdx.x;
            v[k] = g < n ? in[g] : 0u;
        }
#pragma unroll
        for (int k = 0; k < SC_ROWS; ++k) {
            uint32_t tot;
            const uint32_t ex = block_excl_sum(v[k], wsum, tot);
            const int64_t g = base + (int64_t)k * SC_BLOCK + threadIdx.x;
            if (g < n) out[g] = carry + ex;
            carry += tot;
        }
    }
}

// --------------------------------------------------------- radix sort
// Stable LSD radix sort of (key, value) pairs on key bits [0, bits), 8 bits
// per pass, within each of T segments (segment t = items [seg[t], seg[t+1])).
// Tiles of RS_TILE items never straddle two segments; the per-tile digit
// counts are laid out segment-major, digit-major, tile-minor, so that one
// exclusive scan over all of them gives every (segment, digit, tile) its
// first output position.  Segment order is kept, so bits above the sorted
// range need no pass when the input is ordered by segment.
constexpr int RS_BINS = 256;
constexpr int RS_ROWS = 16;
constexpr int RS_TILE = SC_BLOCK * RS_ROWS;
static_assert(SC_BLOCK == RS_BINS, "one thread per digit");
static_assert(RS_TILE < 65536, "ranks packed in 16 bits");

struct rs_segs {
    const int64_t *seg;   // T + 1 item offsets
    const int64_t *tile;  // T + 1 tile offsets (k_rs_tiles)
    int T;
};

__device__ __forceinline__ int rs_find(const int64_t *tile, int T, int64_t i)
{
    int lo = 0, hi = T;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// One thread: tile offsets of the segments and the number of digit counts
// (RS_BINS per tile), the size of the scan between the two sweeps.
__global__ void k_rs_tiles(const int64_t *seg, int T, int64_t *tile, int64_t *n_counts)
{
    if (blockIdx.x || threadIdx.x) return;
    int64_t a = 0;
    tile[0] = 0;
    for (int t = 0; t < T; ++t) {
        const int64_t n = seg[t + 1] - seg[t];
        a += n > 0 ? (n + RS_TILE - 1) / RS_TILE : 0;
        tile[t + 1] = a;
    }
    *n_counts = a * RS_BINS;
}

__device__ __forceinline__ void rs_load_tables(int64_t *sseg, int64_t *stile, const rs_segs &s)
{
    for (int i = threadIdx.x; i <= s.T; i += blockDim.x) {
        sseg[i] = s.seg[i];
        stile[i] = s.tile[i];
    }
}

// Digit counts of every tile.
__global__ void __launch_bounds__(SC_BLOCK) k_rs_upsweep(const uint64_t *keys, rs_segs s, int shift, uint32_t *counts)
{
    __shared__ int64_t sseg[MAX_SEGS + 1], stile[MAX_SEGS + 1];
    __shared__ uint32_t hist[RS_BINS];
    rs_load_tables(sseg, stile, s);
    __syncthreads();
    const int64_t total = stile[s.T];
    for (int64_t i = blockIdx.x; i < total; i += gridDim.x) {
        const int t = rs_find(stile, s.T, i);
        const int64_t j = i - stile[t], nt = stile[t + 1] - stile[t];
        const int64_t lo = sseg[t] + j * RS_TILE, hi = min(lo + RS_TILE, sseg[t + 1]);
        hist[threadIdx.x] = 0u;
        __syncthreads();
        uint32_t d[RS_ROWS];
#pragma unroll
        for (int k = 0; k < RS_ROWS; ++k) {
            const int64_t g = lo + (int64_t)k * SC_BLOCK + threadIdx.x;
            d[k] = g < hi ? (uint32_t)(keys[g] >> shift) & 255u : RS_BINS;
        }
#pragma unroll
        for (int k = 0; k < RS_ROWS; ++k)
            if (d[k] < RS_BINS) atomicAdd(&hist[d[k]], 1u);
        __syncthreads();
        counts[RS_BINS * stile[t] + (int64_t)threadIdx.x * nt + j] = hist[threadIdx.x];
        __syncthreads();
    }
}

// Stable scatter of every tile.  Wave w ranks its own RS_WAVE_ITEMS
// consecutive items of the tile (rows of 64, 8 ballots per row) against
// wave-private digit counts in LDS -- the lanes of one wave need no barrier
// between rows, LDS operations of a wave complete in order -- then the waves'
// counts are combined (exclusive over the waves per digit, exclusive over
// the digits for the tile), and the tile is reordered by digit in LDS so that
// consecutive threads write consecutive addresses.  Six barriers per tile.
constexpr int RS_WAVE_ITEMS = RS_TILE / (SC_BLOCK / 64);
constexpr int RS_WAVE_ROWS = RS_WAVE_ITEMS / 64;
static_assert(RS_WAVE_ROWS * 64 * (SC_BLOCK / 64) == RS_TILE, "whole rows per wave");

__global__ void __launch_bounds__(SC_BLOCK) k_rs_downsweep(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                           uint32_t *vout, rs_segs s, int shift,
                                                           const uint32_t *offs)
{
    __shared__ int64_t sseg[MAX_SEGS + 1], stile[MAX_SEGS + 1];
    __shared__ uint32_t loc[RS_BINS], gbase[RS_BINS];
    __shared__ uint32_t wh[SC_BLOCK / 64][RS_BINS]; // per-wave digit counts, then the bases of each wave
    __shared__ uint32_t wsum[4];
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[RS_TILE];
    rs_load_tables(sseg, stile, s);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int u = 0; u < SC_BLOCK / 64; ++u) wh[u][threadIdx.x] = 0u;
    __syncthreads();
    const int64_t total = stile[s.T], m = sseg[s.T];
    for (int64_t i = blockIdx.x; i < total; i += gridDim.x) {
        const int t = rs_find(stile, s.T, i);
        const int64_t j = i - stile[t], nt = stile[t + 1] - stile[t];
        const int64_t lo = sseg[t] + j * RS_TILE, hi = min(lo + RS_TILE, sseg[t + 1]);
        const int n_tile = (int)(hi - lo);
        uint64_t kk[RS_WAVE_ROWS];
        uint32_t vv[RS_WAVE_ROWS], rk[RS_WAVE_ROWS];
#pragma unroll
        for (int r = 0; r < RS_WAVE_ROWS; ++r) {
            const int idx = w * RS_WAVE_ITEMS + r * 64 + lane;
            kk[r] = idx < n_tile ? kin[lo + idx] : 0ull;
            vv[r] = idx < n_tile ? vin[lo + idx] : 0u;
        }
#pragma unroll
        for (int r = 0; r < RS_WAVE_ROWS; ++r) {
            const bool valid = w * RS_WAVE_ITEMS + r * 64 + lane < n_tile;
            const uint32_t d = (uint32_t)(kk[r] >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t below = lanes_below(peers);
            // every lane reads its digit's count before the digit's first
            // lane writes the count after this row
            const uint32_t base = wh[w][d];
            rk[r] = (d << 16) | (base + below);
            if (valid && below == 0u) wh[w][d] = base + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // thread = digit: bases of the waves, the tile's count
        uint32_t acc = 0u;
#pragma unroll
        for (int u = 0; u < SC_BLOCK / 64; ++u) {
            const uint32_t c = wh[u][threadIdx.x];
            wh[u][threadIdx.x] = acc;
            acc += c;
        }
        uint32_t tot;
        loc[threadIdx.x] = block_excl_sum(acc, wsum, tot);
        gbase[threadIdx.x] = offs[RS_BINS * stile[t] + (int64_t)threadIdx.x * nt + j];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_WAVE_ROWS; ++r) {
            if (w * RS_WAVE_ITEMS + r * 64 + lane < n_tile) {
                const uint32_t d = rk[r] >> 16;
                const uint32_t p = loc[d] + wh[w][d] + (rk[r] & 0xffffu);
                if (p < (uint32_t)RS_TILE) {
                    sk[p] = kk[r];
                    sv[p] = vv[r];
                }
            }
        }
        __syncthreads();
        // the counts start from zero for the next tile (read above, before
        // the barrier)
#pragma unroll
        for (int u = 0; u < SC_BLOCK / 64; ++u) wh[u][threadIdx.x] = 0u;
#pragma unroll
        for (int k = 0; k < RS_ROWS; ++k) {
            const int p = k * SC_BLOCK + (int)threadIdx.x;
            if (p < n_tile) {
                const uint64_t key = sk[p];
                const uint32_t d = (uint32_t)(key >> shift) & 255u;
                const int64_t dst = (int64_t)gbase[d] + (p - (int64_t)loc[d]);
                if (dst >= 0 && dst < m) {
                    kout[dst] = key;
                    vout[dst] = sv[p];
                }
            }
        }
        __syncthreads();
    }
}

} // namespace msplit
