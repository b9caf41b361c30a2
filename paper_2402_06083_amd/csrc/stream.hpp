// Streamed split of one type whose level line does not fit the device in one
// pass (p_31 .. p_33: 2^31 .. 2^33 starts).  The level line is cut into
// chunks of consecutive segments (the paper's independent jobs of Section
// 6.4.1: seed ranges of one level line); each chunk is walked, descended
// and identified on its own, and its identified roots -- sorted by real part
// within the chunk -- are appended to an accumulation.  The roots reached
// from two chunks repeat there (the paper's overlap between jobs), so a
// global identification follows, partitioned by real part: partition k
// takes the accumulated roots with keys in [lo_k - w, hi_k), w the key
// window of the identification radius, identifies them like one call (the
// window below lo_k only looks back: its roots belong to partition k - 1),
// classifies them and appends the ones with keys >= lo_k to the output.
// The partitions follow each other in key order, so the output is the one
// sorted nset a single pass would give; the certificate and the separation
// then run over the whole output.
#pragma once

#include "kernels.hpp"

namespace msplit {

constexpr int STREAM_HIST_SHIFT = 35;                              // key >> 35: bins of 2^-11 in Re c
constexpr int STREAM_HIST_BINS = 1 << (KEY_BITS - STREAM_HIST_SHIFT); // 8192 (32 KiB of LDS)
constexpr int STREAM_MAX_CHUNKS = 1024;

__global__ void k_fill_u64(unsigned long long *a, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// A collected root whose key is below key_lo is not emitted.
__global__ void k_drop_below(batch_args b, const cd *uz, uint32_t *keep, uint64_t key_lo)
{
    const int64_t n = b.coll_offs[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        if (root_key(0, uz[u].re) < key_lo) keep[u] = 0u;
}

// The identified roots of a chunk (collected index space, coll_offs[T] of
// them) to the accumulation at [off, off + n); slots from cap on are not
// written (the host sees the overflow in the chunk's C_UNIQUE count).
__global__ void k_append(batch_args b, const cd *uz, const cd *uz_lo, const uint8_t *uz_dd, cd *acc, cd *acc_lo,
                         uint8_t *acc_dd, int64_t off, int64_t cap)
{
    const int64_t n = b.coll_offs[b.T];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t d = off + i;
        if (d >= cap) break;
        const bool dd = uz_dd[i] != 0;
        acc[d] = uz[i];
        acc_lo[d] = dd ? uz_lo[i] : cd{0.0, 0.0};
        acc_dd[d] = dd;
    }
}

// Histogram of the accumulated keys, STREAM_HIST_BINS bins (LDS counts per
// block, then one global add per non-empty bin).
__global__ void __launch_bounds__(256) k_key_hist(const cd *acc, int64_t n, unsigned long long *hist)
{
    __shared__ uint32_t h[STREAM_HIST_BINS];
    for (int i = threadIdx.x; i < STREAM_HIST_BINS; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = root_key(0, acc[i].re) >> STREAM_HIST_SHIFT;
        atomicAdd(&h[k < (uint64_t)STREAM_HIST_BINS ? k : STREAM_HIST_BINS - 1], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < STREAM_HIST_BINS; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// Per chunk c, the accumulated indices [sl[2c], sl[2c+1]) whose keys lie in
// [k_lo, k_hi): each chunk's roots are sorted by key, so two binary
// searches.  One thread per (chunk, bound).
__global__ void k_slices(const cd *acc, const int64_t *chunk_offs, int nchunks, uint64_t k_lo, uint64_t k_hi,
                         int64_t *sl)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * nchunks) return;
    const int c = i >> 1;
    const uint64_t K = (i & 1) ? k_hi : k_lo;
    int64_t lo = chunk_offs[c], hi = chunk_offs[c + 1]; // first index with key >= K
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (root_key(0, acc[mid].re) < K) lo = mid + 1; else hi = mid;
    }
    sl[i] = lo;
}

// Prefix of the slice sizes: pre[c] = first selected position of chunk c,
// pre[nchunks] = the partition's size.  One thread.
__global__ void k_slice_prefix(const int64_t *sl, int nchunks, int64_t *pre)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t a = 0;
    for (int c = 0; c < nchunks; ++c) {
        pre[c] = a;
        a += sl[2 * c + 1] - sl[2 * c];
    }
    pre[nchunks] = a;
}

// The partition's candidates, chunk by chunk, as converged descents of one
// call (roots, roots_lo, status ST_CONVERGED or ST_DD); m bounds the count.
__global__ void __launch_bounds__(256) k_select(const cd *acc, const cd *acc_lo, const uint8_t *acc_dd,
                                                const int64_t *sl, const int64_t *pre, int nchunks, int64_t m,
                                                cd *roots, cd *roots_lo, uint8_t *status)
{
    __shared__ int64_t p[STREAM_MAX_CHUNKS + 1];
    for (int i = threadIdx.x; i <= nchunks; i += blockDim.x) p[i] = pre[i];
    __syncthreads();
    const int64_t n = p[nchunks] < m ? p[nchunks] : m;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int lo = 0, hi = nchunks; // chunk c with p[c] <= i < p[c + 1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (p[mid] <= i) lo = mid; else hi = mid;
        }
        const int64_t src = sl[2 * lo] + (i - p[lo]);
        const bool dd = acc_dd[src] != 0;
        roots[i] = acc[src];
        roots_lo[i] = acc_lo[src];
        status[i] = dd ? ST_DD : ST_CONVERGED;
    }
}

} // namespace msplit
