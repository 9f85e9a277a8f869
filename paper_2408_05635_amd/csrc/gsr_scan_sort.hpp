// Exclusive scan and stable LSD radix sort for the binning step, written for
// wave64.  Element counts may live in device memory, so a whole call can be
// enqueued (or captured in a graph) without a host synchronisation: grids are
// sized for a host-side capacity and blocks past the device count exit.
#pragma once

#include "gsr_common.hpp"

namespace gsr {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kChunk = kScanThreads * kScanItems;   // 4096 items per block

__device__ __forceinline__ int64_t dev_count(const int64_t *n_dev, int64_t n_host) {
    return n_dev ? *n_dev : n_host;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    const uint32_t lane = lane_id();
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= (uint32_t)off) x += y;
    }
    return x;
}

// Exclusive scan over the block; also returns the block total.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x, uint32_t &total) {
    __shared__ uint32_t s_w[NT / 64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan_u32(x);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
        const uint32_t c = s_w[w];
        if ((uint32_t)w < wave) before += c;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return before + incl - x;
}

// Pass 1: per-block sums of src(i) over a chunk of kChunk items.
template <class Src>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Src src, const int64_t *n_dev, int64_t n_host,
                                                              uint32_t *part) {
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= n) {
        if (threadIdx.x == 0) part[blockIdx.x] = 0;
        return;
    }
    uint32_t s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        if (i < n) s += src(i);
    }
    uint32_t tot;
    block_excl_scan_u32<kScanThreads>(s, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Pass 2: exclusive scan of the nb block sums in place (one block), total to *total.
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *part, int64_t nb, int64_t *total) {
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int64_t k = lo; k < hi; ++k) s += part[k];
    uint32_t tot;
    uint32_t run = block_excl_scan_u32<1024>(s, tot);
    for (int64_t k = lo; k < hi; ++k) {
        const uint32_t c = part[k];
        part[k] = run;
        run += c;
    }
    if (threadIdx.x == 0 && total) *total = (int64_t)tot;
}

// Pass 3: per-block scan with the block's offset; sink(i, exclusive_prefix, value).
template <class Src, class Sink>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Src src, Sink sink, const int64_t *n_dev, int64_t n_host,
                                                            const uint32_t *part) {
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= n) return;
    const int64_t first = base + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (first + j < n) ? src(first + j) : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t run = part[blockIdx.x] + block_excl_scan_u32<kScanThreads>(s, tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (first + j < n) sink(first + j, run, v[j]);
        run += v[j];
    }
}

template <class Src, class Sink>
inline void scan_exclusive(Src src, Sink sink, const int64_t *n_dev, int64_t n_cap, uint32_t *part, int64_t *total,
                           hipStream_t st) {
    const int64_t nb = (n_cap + kChunk - 1) / kChunk;
    if (nb == 0) {
        // still publish a zero total
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, part, (int64_t)0, total);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce<Src>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, src, n_dev, n_cap, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, part, nb, total);
    hipLaunchKernelGGL((k_scan_down<Src, Sink>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, src, sink, n_dev,
                       n_cap, part);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (uint32 key, uint32 value) pairs, <= 8 bits a pass
// ---------------------------------------------------------------------------

// Lanes of the wave holding the same digit as this lane (among `valid` lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int dbits, uint64_t valid) {
    uint64_t peers = valid;
    for (int b = 0; b < dbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = ballot(bit);
        peers &= bit ? bb : ~bb;
    }
    return peers;
}

// Per-block digit counts, stored digit-major: hist[d * nb + block].
__global__ __launch_bounds__(kScanThreads) void k_radix_hist(const uint32_t *__restrict__ keys, const int64_t *n_dev,
                                                             int64_t n_host, int shift, int dbits,
                                                             uint32_t *__restrict__ hist, int64_t nb) {
    __shared__ uint32_t h[256];
    const int64_t n = dev_count(n_dev, n_host);
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
        if (base + (int64_t)j * kScanThreads >= n) break;   // block-uniform
        const bool valid = i < n;
        const uint32_t d = valid ? (keys[i] >> shift) & mask : 0u;
        const uint64_t peers = match_digit(d, dbits, ballot(valid));
        if (valid && rank_below(peers) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    if ((int)threadIdx.x < nd) hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items keep their input order within a digit.
__global__ __launch_bounds__(kScanThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                const uint32_t *__restrict__ vin,
                                                                uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                                const int64_t *n_dev, int64_t n_host, int shift,
                                                                int dbits, const uint32_t *__restrict__ hist, int64_t nb) {
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_w[kScanThreads / 64][256];
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= n) return;
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    const uint32_t t = threadIdx.x, wave = t >> 6;
    if ((int)t < nd) s_off[t] = hist[(int64_t)t * nb + blockIdx.x];
    for (int j = 0; j < kScanItems; ++j) {
        if (base + (int64_t)j * kScanThreads >= n) break;   // block-uniform
        const int64_t i = base + (int64_t)j * kScanThreads + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & mask;
        for (int k = t; k < (kScanThreads / 64) * 256; k += kScanThreads) (&s_w[0][0])[k] = 0u;
        __syncthreads();
        const uint64_t peers = match_digit(d, dbits, ballot(valid));
        const uint32_t rank = rank_below(peers);
        if (valid && rank == 0) s_w[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if ((int)t < nd) {
            uint32_t run = s_off[t];
            for (int w = 0; w < kScanThreads / 64; ++w) {
                const uint32_t c = s_w[w][t];
                s_w[w][t] = run;
                run += c;
            }
            s_off[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = s_w[wave][d] + rank;
            if ((int64_t)pos < n) {   // always true for a correct histogram; keeps writes in bounds
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
    }
}

struct HistSrc {
    const uint32_t *h;
    __device__ uint32_t operator()(int64_t i) const { return h[i]; }
};
struct HistSink {
    uint32_t *h;
    __device__ void operator()(int64_t i, uint32_t pre, uint32_t) const { h[i] = pre; }
};

// nb_dev[0] = number of blocks for the device count, nb_dev[1] = 256 * that
__global__ void k_sort_blocks(const int64_t *n_dev, int64_t *nb_dev) {
    const int64_t nb = (*n_dev + kChunk - 1) / kChunk;
    nb_dev[0] = nb;
    nb_dev[1] = 256 * nb;
}

// Sorts n (device count, <= cap) pairs by key bits [0, bits).  Returns true if
// the result is in (k1, v1), false if in (k0, v0).  The histogram stride is the
// host capacity's block count; only the device count's blocks are touched.
inline bool radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const int64_t *n_dev, int64_t cap,
                       int bits, uint32_t *hist, uint32_t *part, int64_t *scratch_counts, hipStream_t st) {
    const int64_t nb = (cap + kChunk - 1) / kChunk;
    if (nb == 0 || bits <= 0) return false;
    bool in1 = false;
    for (int shift = 0; shift < bits; shift += 8) {
        const int dbits = bits - shift < 8 ? bits - shift : 8;
        uint32_t *ki = in1 ? k1 : k0, *vi = in1 ? v1 : v0;
        uint32_t *ko = in1 ? k0 : k1, *vo = in1 ? v0 : v1;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kScanThreads), 0, st, ki, n_dev, cap, shift, dbits,
                           hist, nb);
        // digit-major counts of all nb blocks (blocks past n wrote zeros or nothing:
        // they are cleared by k_radix_hist only when launched, so the scan covers
        // the full capacity grid, which k_radix_hist always writes)
        scan_exclusive(HistSrc{hist}, HistSink{hist}, nullptr, (int64_t)(1 << dbits) * nb, part, scratch_counts, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kScanThreads), 0, st, ki, vi, ko, vo, n_dev, cap,
                           shift, dbits, hist, nb);
        in1 = !in1;
    }
    return in1;
}

}  // namespace gsr
