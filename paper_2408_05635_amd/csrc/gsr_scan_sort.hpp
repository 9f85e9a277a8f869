// Exclusive scan and stable LSD radix sort for the binning step, written for
// wave64 and for few launches.
//
// The scan is single-pass with decoupled look-back: each block takes a ticket
// (tickets follow the order in which blocks start, so a block only ever
// waits for blocks that are already running), publishes its aggregate, then
// walks back over its predecessors' published values until it meets an
// inclusive prefix, and publishes its own.  A status word is 64 bits: the
// high half holds (id << 2 | flag), the low half the value.  The status
// words and tickets are cleared at the start of every call and every scan
// of a call has its own id, so a word left by an earlier scan never passes
// for a current one.  A waiting loop gives up after kSpinLimit polls and
// raises an error counter: every wave terminates, whatever happens.  The
// three-launch radix sort passes need no waiting; the one-launch passes for
// small sorts wait the same bounded way (see below).
//
// Element counts may live in device memory: grids are sized for a host-side
// capacity and blocks past the device count exit at once, so a whole call can
// be enqueued (or captured in a graph) without a host synchronisation.
#pragma once

#include <type_traits>

#include "gsr_common.hpp"

namespace gsr {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kChunk = kScanThreads * kScanItems;   // 4096 items per block
constexpr uint32_t kFlagAgg = 1u, kFlagPrefix = 2u;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kMaxSyncIds = 32;

// Synchronisation state of one call (cleared by the call's first kernel).
struct SyncState {
    uint32_t *tickets;   // [kMaxSyncIds] block tickets, one per scan
    uint64_t *status;    // [blocks of the largest scan] look-back words
    int64_t *error;      // raised when a wait gives up
};

__device__ __forceinline__ int64_t dev_count(const int64_t *n_dev, int64_t n_host) {
    return n_dev ? *n_dev : n_host;
}

// Status words carry their value with them, so relaxed device-wide atomics
// suffice: no other data is published through them.
__device__ __forceinline__ void store_word(uint64_t *p, uint32_t tag, uint32_t value) {
    __hip_atomic_store(p, ((uint64_t)tag << 32) | (uint64_t)value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void publish(uint64_t *p, uint32_t id, uint32_t flag, uint32_t value) {
    store_word(p, (id << 2) | flag, value);
}

__device__ __forceinline__ uint64_t peek(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value of a word once it carries `tag` (bounded wait; raises *error and
// returns 0 if it never does).
__device__ __forceinline__ uint32_t await_word(const uint64_t *p, uint64_t first, uint32_t tag, int64_t *error) {
    uint64_t v = first;
    for (uint32_t spins = 0; (uint32_t)(v >> 32) != tag; v = peek(p)) {
        if (++spins > kSpinLimit) {   // never expected: report it and stop waiting
            atomicAdd((unsigned long long *)error, 1ull);
            return 0u;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return (uint32_t)v;
}

__device__ __forceinline__ uint32_t take_ticket(uint32_t *tickets, uint32_t id) {
    return __hip_atomic_fetch_add(&tickets[id], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of block b in a chain of consecutive status words, walked
// by a whole wave: lane l of window k inspects block p - 64 k - l, and the
// kLookWindows windows are loaded at once, so one round trip covers 256
// predecessors.  All 64 lanes must call it.
constexpr int kLookWindows = 4;

__device__ __forceinline__ uint32_t look_back_wave(const uint64_t *chain, int64_t b, uint32_t id, int64_t *error) {
    const uint32_t lane = lane_id();
    const uint32_t t_agg = (id << 2) | kFlagAgg, t_pre = (id << 2) | kFlagPrefix;
    uint32_t excl = 0, spins = 0;
    int64_t p = b - 1;
    while (p >= 0) {
        uint64_t v[kLookWindows];
#pragma unroll
        for (int k = 0; k < kLookWindows; ++k) {
            const int64_t q = p - 64 * k - (int64_t)lane;
            v[k] = q >= 0 ? peek(chain + q) : 0ull;
        }
        bool finished = false, moved = false;
#pragma unroll
        for (int k = 0; k < kLookWindows; ++k) {
            const int64_t q = p - (int64_t)lane;   // p has moved past the windows already summed
            const uint32_t tag = q >= 0 ? (uint32_t)(v[k] >> 32) : t_pre;   // a zero prefix before block 0
            const uint32_t val = q >= 0 ? (uint32_t)v[k] : 0u;
            const uint64_t pre = ballot(tag == t_pre);
            const uint64_t ready = ballot(tag == t_pre || tag == t_agg);
            const int fp = pre ? (int)__builtin_ctzll(pre) : 64;   // nearest predecessor with a prefix
            const uint64_t need = fp >= 63 ? ~0ull : ((2ull << fp) - 1ull);
            if ((ready & need) != need) break;   // poll this window again
            uint32_t mine = ((int)lane <= fp) ? val : 0u;
            for (int off = 32; off >= 1; off >>= 1) mine += __shfl_xor(mine, off, 64);
            excl += mine;
            if (fp < 64) {
                finished = true;
                break;
            }
            p -= 64;
            moved = true;
        }
        if (finished) break;
        if (!moved) {
            if (++spins > kSpinLimit) {   // never expected: report it and stop waiting
                if (lane == 0) atomicAdd((unsigned long long *)error, 1ull);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
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

// The total of a scan goes to one int64.
struct TotalTo {
    int64_t *p;
    __device__ void operator()(int64_t t) const {
        if (p) *p = t;
    }
};

__device__ __forceinline__ uint32_t scan_slot(uint32_t k) { return k + (k >> 4); }

// Single-pass exclusive scan: sink(i, exclusive_prefix, value) for every
// i < n, then fin(total) once.  The sink may overwrite the source in place.
template <class Src, class Sink, class Fin>
__global__ __launch_bounds__(kScanThreads) void k_scan(Src src, Sink sink, const int64_t *n_dev, int64_t n_host,
                                                       SyncState ss, uint32_t id, Fin fin) {
    __shared__ uint32_t s_b, s_excl;
    __shared__ uint32_t s_val[kChunk + kChunk / 16], s_pre[kChunk + kChunk / 16];
    if (threadIdx.x == 0) s_b = take_ticket(ss.tickets, id);
    __syncthreads();
    const int64_t b = s_b;
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t nb = (n + kChunk - 1) / kChunk;
    if (b >= nb) {   // block-uniform
        if (nb == 0 && b == 0 && threadIdx.x == 0) fin(0);
        return;
    }
    // The block's items are read and written coalesced (item j kScanThreads +
    // thread in round j) through LDS, where each thread scans kScanItems
    // consecutive items (one pad word after every 16, so that a thread's
    // items fall in different banks).
    const int64_t base = b * kChunk;
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j * kScanThreads + (int64_t)t;
        s_val[scan_slot(j * kScanThreads + t)] = i < n ? src(i) : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = s_val[scan_slot(t * kScanItems + j)];
        s += v[j];
    }
    uint32_t agg;
    uint32_t run = block_excl_scan_u32<kScanThreads>(s, agg);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {   // each item's prefix within the block
        s_pre[scan_slot(t * kScanItems + j)] = run;
        run += v[j];
    }
    uint64_t *mine = ss.status + b;
    if (threadIdx.x == 0) publish(mine, id, b == 0 ? kFlagPrefix : kFlagAgg, agg);
    if (threadIdx.x < 64) {   // wave 0 looks back
        const uint32_t excl = b == 0 ? 0u : look_back_wave(ss.status, b, id, ss.error);
        if (threadIdx.x == 0) {
            if (b > 0) publish(mine, id, kFlagPrefix, excl + agg);
            s_excl = excl;
            if (b == nb - 1) fin((int64_t)excl + (int64_t)agg);
        }
    }
    __syncthreads();
    const uint32_t excl = s_excl;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t i = base + j * kScanThreads + (int64_t)t;
        const uint32_t k = scan_slot(j * kScanThreads + t);
        if (i < n) sink(i, excl + s_pre[k], s_val[k]);
    }
}

template <class Src, class Sink, class Fin>
inline void scan_exclusive(Src src, Sink sink, const int64_t *n_dev, int64_t n_cap, const SyncState &ss, uint32_t id,
                           Fin fin, hipStream_t st) {
    int64_t nb = (n_cap + kChunk - 1) / kChunk;
    if (nb < 1) nb = 1;   // one block still publishes a zero total
    hipLaunchKernelGGL((k_scan<Src, Sink, Fin>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, src, sink, n_dev,
                       n_cap, ss, id, fin);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (uint32 key, uint32 value) pairs, <= 8 bits a pass
//
// Three launches a pass, none of which waits for another block:
// k_radix_count stores every block's digit counts (plain stores, laid out
// digit-major); k_digit_scan, one block per digit, turns a digit's counts
// into exclusive offsets over the blocks and its total; k_radix_scatter adds
// the digit bases (an exclusive scan of the 256 totals, done by every block)
// and places its items stably.  The kernel boundaries order the passes, so
// nothing needs clearing between calls.
// ---------------------------------------------------------------------------

// Items per thread of a sort pass: 1024-item blocks up to 2M items, 4096
// above (fewer blocks, so fewer count rows to scan).
constexpr int64_t kSmallSortCap = 2ll << 20;
inline int sort_items(int64_t cap) { return cap <= kSmallSortCap ? 4 : 16; }
inline int64_t sort_blocks(int64_t cap) {
    const int64_t chunk = (int64_t)kScanThreads * sort_items(cap);
    return (cap + chunk - 1) / chunk;
}

// Per-call state of the sort passes (no clearing needed).
struct SortState {
    uint32_t *counts;   // [256][blocks of the largest sort] digit counts, then exclusive offsets over the blocks
    uint32_t *totals;   // [256] digit totals of the current pass
};

// Inputs of a sort pass.  PairIn: items [0, n) of (key, value) arrays.
// VisIn (the first pass of the depth sort): item i of [0, n) takes part only
// if cnt[i] != 0 (a visible record), with key zkey[i] and value i, so the pass
// also compacts the visible records, in index order within a digit.
struct PairIn {
    const uint32_t *k, *v;
    __device__ __forceinline__ bool load(int64_t i, int64_t n, uint32_t &key, uint32_t &val) const {
        if (i >= n) return false;
        key = k[i];
        val = v[i];
        return true;
    }
};
struct VisIn {
    const uint32_t *cnt, *zkey;
    __device__ __forceinline__ bool load(int64_t i, int64_t n, uint32_t &key, uint32_t &val) const {
        if (i >= n || cnt[i] == 0u) return false;
        key = zkey[i];
        val = (uint32_t)i;
        return true;
    }
};

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

template <int ITEMS, class In>
__global__ __launch_bounds__(kScanThreads) void k_radix_count(In in, const int64_t *n_dev, int64_t n_host, int shift,
                                                              int dbits, SortState so, int64_t nb_cap) {
    __shared__ uint32_t s_cnt[256];
    const uint32_t t = threadIdx.x;
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t nb = (n + (kScanThreads * ITEMS) - 1) / (kScanThreads * ITEMS);
    const int64_t b = blockIdx.x;
    if (b >= nb || b >= nb_cap) return;   // block-uniform
    const uint32_t mask = (1u << dbits) - 1u;
    s_cnt[t] = 0u;
    __syncthreads();
    const int64_t base = b * (kScanThreads * ITEMS);
    uint32_t key[ITEMS];   // all loads in flight at once
    bool ok[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        uint32_t val;
        key[j] = 0u;
        ok[j] = in.load(base + (int64_t)j * kScanThreads + t, n, key[j], val);
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = ok[j];
        const uint32_t d = (key[j] >> shift) & mask;
        const uint64_t peers = match_digit(d, dbits, ballot(valid));
        if (valid && rank_below(peers) == 0) atomicAdd(&s_cnt[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    so.counts[(size_t)t * nb_cap + b] = s_cnt[t];
}

// One block per digit: exclusive offsets of the digit over the blocks (in
// block order) and the digit's total; with total_out (zero beforehand), the
// sum of the totals, i.e. the number of items that took part.
template <int ITEMS>
__global__ __launch_bounds__(kScanThreads) void k_digit_scan(const int64_t *n_dev, int64_t n_host, int dbits,
                                                             SortState so, int64_t nb_cap, int64_t *total_out) {
    const int d = blockIdx.x;
    const int64_t n = dev_count(n_dev, n_host);
    int64_t nb = (n + (kScanThreads * ITEMS) - 1) / (kScanThreads * ITEMS);
    nb = nb < nb_cap ? nb : nb_cap;
    if (d >= (1 << dbits)) {   // block-uniform
        if (threadIdx.x == 0) so.totals[d] = 0u;
        return;
    }
    uint32_t *row = so.counts + (size_t)d * nb_cap;
    const int64_t per = (nb + kScanThreads - 1) / kScanThreads;   // consecutive blocks per thread
    const int64_t q0 = (int64_t)threadIdx.x * per;
    const int64_t q1 = q0 + per < nb ? q0 + per : nb;
    uint32_t s = 0;
    for (int64_t q = q0; q < q1; ++q) s += row[q];
    uint32_t all;
    uint32_t run = block_excl_scan_u32<kScanThreads>(s, all);
    for (int64_t q = q0; q < q1; ++q) {
        const uint32_t c = row[q];
        row[q] = run;
        run += c;
    }
    if (threadIdx.x == 0) {
        so.totals[d] = all;
        if (total_out) atomicAdd((unsigned long long *)total_out, (unsigned long long)all);   // integer: any order
    }
}

// Stable scatter: items keep their input order within a digit.  The block
// first ranks its items within their digits (each wave its own contiguous
// run, in input order), then places them in LDS in digit order and writes
// each digit's run to consecutive global positions, so that the stores are
// coalesced runs instead of one transaction per item.
// ranges (the last pass only, else null): every key's [first, last + 1)
// position in the output, for keys < n_keys.  Within a block's run of one
// digit the items are in final order, so a key's first and last positions are
// where its LDS neighbours differ, or at the ends of a run, where the adjacent
// block may hold the same key: atomicMin / atomicMax over the candidates
// (ranges start as (0xffffffff, 0)) give the exact bounds in any order.
template <int ITEMS, class In>
__global__ __launch_bounds__(kScanThreads) void k_radix_scatter(In in, uint32_t *__restrict__ kout,
                                                                uint32_t *__restrict__ vout, const int64_t *n_dev,
                                                                int64_t n_host, int shift, int dbits, SortState so,
                                                                int64_t nb_cap, uint2 *__restrict__ ranges,
                                                                int64_t n_keys) {
    constexpr int kItems = kScanThreads * ITEMS;
    constexpr int kWaves = kScanThreads / 64;
    __shared__ uint32_t s_goff[256];   // global position of the block's first item of each digit
    __shared__ uint32_t s_cnt[256];    // the block's count of each digit, then the digit's first slot in s_k
    __shared__ uint32_t s_h[kWaves][256];   // per wave: running count of each digit, then the wave's offset in it
    __shared__ uint32_t s_k[kItems], s_v[kItems];
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t b = blockIdx.x;
    const int64_t base = b * kItems;
    if (base >= n) return;   // block-uniform
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63u;
    {   // global position of the block's first item of each digit: the digit's
        // base (totals of the smaller digits) plus the counts of earlier blocks
        uint32_t all;
        const uint32_t dbase = block_excl_scan_u32<kScanThreads>((int)t < nd ? so.totals[t] : 0u, all);
        s_goff[t] = ((int)t < nd ? so.counts[(size_t)t * nb_cap + b] : 0u) + dbase;
    }
    for (uint32_t k = lane; k < 256u; k += 64u) s_h[wave][k] = 0u;
    // Each wave holds a contiguous run of 64 * ITEMS items of the block, so the
    // block's stable order is (wave, round, lane): every wave ranks its own
    // items in order without block barriers, and one scan over the waves per
    // digit joins them.
    const int64_t wbase = base + (int64_t)wave * (64 * ITEMS);
    uint32_t keys[ITEMS], vals[ITEMS], lrank[ITEMS];   // all loads in flight at once
    bool ok[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        keys[j] = vals[j] = lrank[j] = 0u;
        ok[j] = in.load(wbase + (int64_t)j * 64 + lane, n, keys[j], vals[j]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const bool valid = ok[j];
        const uint64_t vmask = ballot(valid);
        if (vmask == 0) continue;   // wave-uniform
        const uint32_t d = (keys[j] >> shift) & mask;
        const uint64_t peers = match_digit(d, dbits, vmask);
        const uint32_t rank = rank_below(peers);
        // every lane reads the digit's count before its first lane updates it
        // (the LDS completes one wave's operations in order)
        const uint32_t before = s_h[wave][d];
        lrank[j] = before + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) s_h[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    uint32_t run = 0;
    if ((int)t < nd) {
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = s_h[w][t];
            s_h[w][t] = run;
            run += c;
        }
    }
    s_cnt[t] = run;
    __syncthreads();
    // digits' first slots in the block's digit-ordered staging
    uint32_t tot;
    const uint32_t lbase = block_excl_scan_u32<kScanThreads>(s_cnt[t], tot);
    s_cnt[t] = lbase;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (ok[j]) {
            const uint32_t d = (keys[j] >> shift) & mask;
            const uint32_t lp = s_cnt[d] + s_h[wave][d] + lrank[j];
            if (lp < (uint32_t)kItems) {   // always true for consistent counts
                s_k[lp] = keys[j];
                s_v[lp] = vals[j];
            }
        }
    }
    __syncthreads();
    const int nblk = (int)(tot < (uint32_t)kItems ? tot : (uint32_t)kItems);   // the block's items that take part
    for (int i = t; i < nblk; i += kScanThreads) {
        const uint32_t key = s_k[i];
        const uint32_t d = (key >> shift) & mask;
        const uint32_t pos = s_goff[d] + ((uint32_t)i - s_cnt[d]);
        if ((int64_t)pos < n) {   // always true for consistent counts; keeps writes in bounds
            kout[pos] = key;
            vout[pos] = s_v[i];
            if (ranges && (int64_t)key < n_keys) {   // block-uniform choice
                const uint32_t run0 = s_cnt[d], run1 = d + 1u < 256u ? s_cnt[d + 1] : tot;
                if ((uint32_t)i == run0 || s_k[i - 1] != key) atomicMin(&ranges[key].x, pos);
                if ((uint32_t)i + 1u == run1 || s_k[i + 1] != key) atomicMax(&ranges[key].y, pos + 1u);
            }
        }
    }
}

// One pass: items of `in` -> (ko, vo) by key bits [shift, shift + dbits).
template <class In>
inline void radix_pass(In in, uint32_t *ko, uint32_t *vo, const int64_t *n_dev, int64_t n_host, int64_t cap,
                       int shift, int dbits, const SortState &so, int64_t *total_out, hipStream_t st,
                       uint2 *ranges = nullptr, int64_t n_keys = 0) {
    const int64_t nb = sort_blocks(cap);
    const bool small = sort_items(cap) == 4;
    hipLaunchKernelGGL((small ? k_radix_count<4, In> : k_radix_count<16, In>), dim3((unsigned)nb), dim3(kScanThreads), 0,
                       st, in, n_dev, n_host, shift, dbits, so, nb);
    hipLaunchKernelGGL(small ? k_digit_scan<4> : k_digit_scan<16>, dim3(256), dim3(kScanThreads), 0, st, n_dev, n_host,
                       dbits, so, nb, total_out);
    hipLaunchKernelGGL((small ? k_radix_scatter<4, In> : k_radix_scatter<16, In>), dim3((unsigned)nb),
                       dim3(kScanThreads), 0, st, in, ko, vo, n_dev, n_host, shift, dbits, so, nb, ranges, n_keys);
}

// Sorts n (device count, <= cap) pairs by key bits [0, bits).  Returns true
// if the result is in (k1, v1), false if in (k0, v0).  With ranges, the last
// pass also records every key's [start, end) (see k_radix_scatter).
inline bool radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const int64_t *n_dev, int64_t cap,
                       int bits, const SortState &so, hipStream_t st, uint2 *ranges = nullptr, int64_t n_keys = 0) {
    if (sort_blocks(cap) == 0 || bits <= 0) return false;
    bool in1 = false;
    for (int shift = 0; shift < bits; shift += 8) {
        const int dbits = bits - shift < 8 ? bits - shift : 8;
        const bool last = shift + 8 >= bits;
        radix_pass(PairIn{in1 ? k1 : k0, in1 ? v1 : v0}, in1 ? k0 : k1, in1 ? v0 : v1, n_dev, cap, cap, shift, dbits,
                   so, nullptr, st, last ? ranges : nullptr, n_keys);
        in1 = !in1;
    }
    return in1;
}

// The depth sort: the visible records among the n (view, Gaussian) items
// (cnt[i] != 0), compacted and stably sorted by the 32-bit depth key; the
// first pass reads the projection's arrays and writes the number of visible
// records to *n_out (zero beforehand), which bounds the later passes.  Four
// passes, (k1, v1), (k0, v0), (k1, v1), (k0, v0): the result is in (k0, v0).
inline void radix_sort_visible(const uint32_t *cnt, const uint32_t *zkey, int64_t n, uint32_t *k0, uint32_t *v0,
                               uint32_t *k1, uint32_t *v1, int64_t *n_out, const SortState &so, hipStream_t st) {
    if (sort_blocks(n) == 0) return;
    radix_pass(VisIn{cnt, zkey}, k1, v1, nullptr, n, n, 0, 8, so, n_out, st);
    radix_pass(PairIn{k1, v1}, k0, v0, n_out, n, n, 8, 8, so, nullptr, st);
    radix_pass(PairIn{k0, v0}, k1, v1, n_out, n, n, 16, 8, so, nullptr, st);
    radix_pass(PairIn{k1, v1}, k0, v0, n_out, n, n, 24, 8, so, nullptr, st);
}

// ---------------------------------------------------------------------------
// One launch per pass (the "onesweep" scheme of Adinets and Merrill, 2022)
//
// The digit totals of every pass are known before the first one: the keys are
// the same multiset in every pass, so one histogram of all their digits,
// taken where the keys are produced, serves them all.  A pass is then a single
// kernel: each block takes a ticket, ranks its chunk of 4096 items, publishes
// its count of every digit, and finds the counts of the blocks before it by a
// decoupled look-back per digit (thread d walks digit d's words back, 32
// blocks per poll, until it meets an inclusive prefix), so no block ever waits
// for a block that started after it.  Look-back words are 32 bits: a 5-bit tag
// (pass id << 1 | inclusive) over a 27-bit count; they are cleared with the
// rest of the synchronisation region at the start of every call, and every
// pass of a call has its own id.  Sorts of more than kSweepMaxBlocks chunks
// take the three-launch passes above instead: with hundreds of blocks polling
// at once the look-back chains resolve more slowly than the two extra
// launches cost, and this scheme pays off where launches dominate (small
// sorts, such as one view's records and pairs in a tracking iteration).
// ---------------------------------------------------------------------------
constexpr int kSweepThreads = 1024;
constexpr int kSweepItems = 4;
constexpr int kSweepChunk = kSweepThreads * kSweepItems;   // 4096 items per block
constexpr int kSweepWaves = kSweepThreads / 64;
constexpr int kSweepLook = 32;                             // predecessors per thread and poll
constexpr int64_t kSweepMaxBlocks = 256;   // 1M items
constexpr uint32_t kSweepValBits = 27;
constexpr uint32_t kSweepValMask = (1u << kSweepValBits) - 1u;

inline int64_t sweep_blocks(int64_t cap) { return (cap + kSweepChunk - 1) / kSweepChunk; }
inline bool sweep_fits(int64_t cap) { return sweep_blocks(cap) <= kSweepMaxBlocks; }

struct SweepState {
    uint32_t *status;    // [blocks][256] look-back words
    uint32_t *tickets;   // block tickets, indexed by pass id
    int64_t *error;      // raised when a wait gives up
};

__device__ __forceinline__ uint32_t sweep_word(uint32_t pass_id, bool inclusive, uint32_t v) {
    return (((pass_id << 1) | (inclusive ? 1u : 0u)) << kSweepValBits) | (v & kSweepValMask);
}

__device__ __forceinline__ void sweep_store(uint32_t *p, uint32_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t sweep_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Count of digit d in the blocks before block b (b > 0), from their words in
// `status` (row q = block q).  Bounded wait: raises *error and returns what it
// has summed if a predecessor never publishes.
__device__ __forceinline__ uint32_t sweep_look_back(const uint32_t *status, int64_t b, uint32_t d, uint32_t pass_id,
                                                    int64_t *error) {
    const uint32_t tag_agg = pass_id << 1, tag_pre = (pass_id << 1) | 1u;
    uint32_t excl = 0, spins = 0;
    int64_t p = b - 1;   // next predecessor to read
    while (p >= 0) {
        uint32_t w[kSweepLook];
#pragma unroll
        for (int k = 0; k < kSweepLook; ++k)
            w[k] = p - k >= 0 ? sweep_load(status + (size_t)(p - k) * 256 + d) : (tag_pre << kSweepValBits);
        int k = 0;
        bool done = false;
#pragma unroll
        for (int j = 0; j < kSweepLook; ++j) {   // in order of decreasing block
            if (done || k != j) continue;
            const uint32_t tag = w[j] >> kSweepValBits;
            if (tag == tag_pre) {
                excl += w[j] & kSweepValMask;
                done = true;
            } else if (tag == tag_agg) {
                excl += w[j] & kSweepValMask;
                ++k;
            }
        }
        if (done) break;
        p -= k;
        if (k == 0) {
            if (++spins > kSpinLimit) {   // never expected: report it and stop waiting
                atomicAdd((unsigned long long *)error, 1ull);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// One pass: items of `in` -> (kout, vout) stably by key bits [shift, shift +
// dbits); totals[d] = number of items with digit d.  ranges as in
// k_radix_scatter (last pass of the tile sort only).
template <class In>
__global__ __launch_bounds__(kSweepThreads) void k_sweep(In in, uint32_t *__restrict__ kout,
                                                         uint32_t *__restrict__ vout, const int64_t *n_dev,
                                                         int64_t n_host, int shift, int dbits,
                                                         const uint32_t *__restrict__ totals, SweepState sw,
                                                         uint32_t pass_id, uint2 *__restrict__ ranges,
                                                         int64_t n_keys) {
    __shared__ uint32_t s_b;
    __shared__ uint32_t s_goff[256];   // digit base, then the global position of the block's first item of the digit
    __shared__ uint32_t s_cnt[256];    // the block's count of each digit, then the digit's first slot in s_k
    __shared__ uint32_t s_h[kSweepWaves][256];
    __shared__ uint32_t s_k[kSweepChunk], s_v[kSweepChunk];
    const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63u;
    const int64_t n = dev_count(n_dev, n_host);
    const int64_t nb = (n + kSweepChunk - 1) / kSweepChunk;
    // grids are sized for the capacity: the blocks past the device count leave
    // without a ticket, so the tickets of the others are exactly [0, nb)
    if ((int64_t)blockIdx.x >= nb) return;   // block-uniform
    if (t == 0) s_b = take_ticket(sw.tickets, pass_id);
    for (uint32_t k = lane; k < 256u; k += 64u) s_h[wave][k] = 0u;
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    {   // digit bases: exclusive scan of the totals
        uint32_t all;
        const uint32_t dbase = block_excl_scan_u32<kSweepThreads>((int)t < nd ? totals[t] : 0u, all);
        if (t < 256u) s_goff[t] = dbase;
    }
    __syncthreads();   // s_b, s_h and s_goff are set
    const int64_t b = s_b;
    const int64_t wbase = b * kSweepChunk + (int64_t)wave * (64 * kSweepItems);
    uint32_t keys[kSweepItems], vals[kSweepItems], lrank[kSweepItems];
    bool ok[kSweepItems];
#pragma unroll
    for (int j = 0; j < kSweepItems; ++j) {
        keys[j] = vals[j] = lrank[j] = 0u;
        ok[j] = in.load(wbase + (int64_t)j * 64 + lane, n, keys[j], vals[j]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < kSweepItems; ++j) {   // per-wave stable ranks, as in k_radix_scatter
        const bool valid = ok[j];
        const uint64_t vmask = ballot(valid);
        if (vmask == 0) continue;   // wave-uniform
        const uint32_t d = (keys[j] >> shift) & mask;
        const uint64_t peers = match_digit(d, dbits, vmask);
        const uint32_t rank = rank_below(peers);
        const uint32_t before = s_h[wave][d];
        lrank[j] = before + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) s_h[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if ((int)t < nd) {
        uint32_t run = 0;
        for (int w = 0; w < kSweepWaves; ++w) {
            const uint32_t c = s_h[w][t];
            s_h[w][t] = run;
            run += c;
        }
        s_cnt[t] = run;
        uint32_t *mine = sw.status + (size_t)b * 256 + t;
        if (b == 0) {
            sweep_store(mine, sweep_word(pass_id, true, run));
        } else {
            sweep_store(mine, sweep_word(pass_id, false, run));
            const uint32_t excl = sweep_look_back(sw.status, b, t, pass_id, sw.error);
            sweep_store(mine, sweep_word(pass_id, true, excl + run));
            s_goff[t] += excl;
        }
    } else if (t < 256u) {
        s_cnt[t] = 0u;
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t lbase = block_excl_scan_u32<kSweepThreads>(t < 256u ? s_cnt[t] : 0u, tot);
    if (t < 256u) s_cnt[t] = lbase;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSweepItems; ++j) {
        if (ok[j]) {
            const uint32_t d = (keys[j] >> shift) & mask;
            const uint32_t lp = s_cnt[d] + s_h[wave][d] + lrank[j];
            if (lp < (uint32_t)kSweepChunk) {   // always true for consistent counts
                s_k[lp] = keys[j];
                s_v[lp] = vals[j];
            }
        }
    }
    __syncthreads();
    const int nblk = (int)(tot < (uint32_t)kSweepChunk ? tot : (uint32_t)kSweepChunk);
    for (int i = t; i < nblk; i += kSweepThreads) {
        const uint32_t key = s_k[i];
        const uint32_t d = (key >> shift) & mask;
        const uint32_t pos = s_goff[d] + ((uint32_t)i - s_cnt[d]);
        if ((int64_t)pos < n) {   // always true for consistent counts; keeps writes in bounds
            kout[pos] = key;
            vout[pos] = s_v[i];
            if (ranges && (int64_t)key < n_keys) {   // block-uniform choice
                const uint32_t run0 = s_cnt[d], run1 = d + 1u < 256u ? s_cnt[d + 1] : tot;
                if ((uint32_t)i == run0 || s_k[i - 1] != key) atomicMin(&ranges[key].x, pos);
                if ((uint32_t)i + 1u == run1 || s_k[i + 1] != key) atomicMax(&ranges[key].y, pos + 1u);
            }
        }
    }
}

// Adds a valid key's 8-bit digits of bits [0, bits) into hist[pass][256] in
// LDS.  Plain LDS atomics: lanes that share a digit are serialised by the
// LDS, which costs less than finding them with ballots.
__device__ __forceinline__ void add_digit_hist(uint32_t key, bool valid, int bits, uint32_t *s_hist) {
    if (!valid) return;
    for (int shift = 0, p = 0; shift < bits; shift += 8, ++p)
        atomicAdd(&s_hist[p * 256 + ((key >> shift) & 255u)], 1u);
}

// Adds a block's LDS histogram (passes x 256) into the global one (zero
// before the call's first block), skipping empty bins.
__device__ __forceinline__ void flush_digit_hist(const uint32_t *s_hist, int passes, uint32_t *hist) {
    for (int k = threadIdx.x; k < passes * 256; k += blockDim.x) {
        const uint32_t c = s_hist[k];
        if (c) atomicAdd(&hist[k], c);
    }
}

// The visible items (cnt[i] != 0) among the n (view, Gaussian) items,
// compacted in index order into (kout = depth key, vout = index) by a
// single-pass scan (decoupled look-back over blocks of kCompactThreads x ITEMS
// items: 4 per thread, or 8 for a million items or more, where half as many
// blocks make a shorter look-back),
// and their number (written to *n_out by the last block).  With hist (the
// first step of the one-launch depth sort), also the histograms of the four
// byte digits of their keys (added into hist[4][256], zero beforehand).  With
// first (items in groups of `group`, here the views' N Gaussians), also the
// output place of every group's first visible item: the number of visible
// items before the group.
constexpr int kCompactThreads = 1024;
constexpr int64_t kCompactWideMin = 1 << 20;   // items from which a thread takes 8

template <int ITEMS>
__global__ __launch_bounds__(kCompactThreads) void k_compact_hist(const uint32_t *__restrict__ cnt,
                                                                  const uint32_t *__restrict__ zkey, int64_t n,
                                                                  uint32_t *__restrict__ kout,
                                                                  uint32_t *__restrict__ vout, SyncState ss,
                                                                  uint32_t id, uint32_t *__restrict__ hist,
                                                                  int64_t *__restrict__ n_out,
                                                                  uint32_t *__restrict__ first_of, int64_t group) {
    __shared__ uint32_t s_b, s_excl;
    __shared__ uint32_t s_hist[4 * 256];
    const uint32_t t = threadIdx.x;
    const int64_t nb = (n + (kCompactThreads * ITEMS) - 1) / (kCompactThreads * ITEMS);
    if ((int64_t)blockIdx.x >= nb) return;   // block-uniform
    if (t == 0) s_b = take_ticket(ss.tickets, id);
    s_hist[t] = 0u;
    __syncthreads();
    const int64_t b = s_b;
    const int64_t first = b * (kCompactThreads * ITEMS) + (int64_t)t * ITEMS;
    uint32_t c[ITEMS], k[ITEMS];
    if (first + ITEMS <= n) {   // 16-byte aligned runs of 4
        const uint4 *c4 = reinterpret_cast<const uint4 *>(cnt + first);
        const uint4 *k4 = reinterpret_cast<const uint4 *>(zkey + first);
#pragma unroll
        for (int q = 0; q < ITEMS / 4; ++q) {
            const uint4 a = c4[q], z = k4[q];
            c[4 * q] = a.x, c[4 * q + 1] = a.y, c[4 * q + 2] = a.z, c[4 * q + 3] = a.w;
            k[4 * q] = z.x, k[4 * q + 1] = z.y, k[4 * q + 2] = z.z, k[4 * q + 3] = z.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool in = first + j < n;
            c[j] = in ? cnt[first + j] : 0u;
            k[j] = in ? zkey[first + j] : 0u;
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) s += c[j] != 0u ? 1u : 0u;
    if (hist) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) add_digit_hist(k[j], c[j] != 0u, 32, s_hist);
    }
    uint32_t agg;
    uint32_t run = block_excl_scan_u32<kCompactThreads>(s, agg);
    uint64_t *mine = ss.status + b;
    if (t == 0) publish(mine, id, b == 0 ? kFlagPrefix : kFlagAgg, agg);
    if (t < 64) {   // wave 0 looks back
        const uint32_t excl = b == 0 ? 0u : look_back_wave(ss.status, b, id, ss.error);
        if (t == 0) {
            if (b > 0) publish(mine, id, kFlagPrefix, excl + agg);
            s_excl = excl;
            if (b == nb - 1) *n_out = (int64_t)excl + (int64_t)agg;
        }
    }
    __syncthreads();   // also orders the LDS histogram's atomics before the flush
    run += s_excl;
    // the first group start at or after this thread's first item
    int64_t gs = -1;
    if (first_of && first < n) gs = (first + group - 1) / group * group;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (gs == first + j && gs < n) {   // a group starts at item first + j
            first_of[gs / group] = run;
            gs += group;
        }
        if (c[j] != 0u) {
            kout[run] = k[j];
            vout[run] = (uint32_t)(first + j);
            ++run;
        }
    }
    if (hist) flush_digit_hist(s_hist, 4, hist);
}

// ---------------------------------------------------------------------------
// per-tile sort (tile-local binning)
//
// The emission places every (tile, record) pair in its tile's range in no
// particular order; k_tile_sort then orders each list by the 64-bit key
// (float32 depth bits, record), the order that a stable sort by depth followed
// by a stable sort by tile gives.  Keys are distinct (records are).
//
// Lists of up to kTileSortCap keys are merge-sorted in LDS: each thread sorts
// E = 1, 2, 4 or 8 keys in registers (Batcher's odd-even merge networks), then
// rounds merge pairs of sorted runs of L keys into runs of 2L, each thread
// producing E consecutive outputs: a binary search along its diagonal of the
// merge (the "merge path" of Odeh et al., 2012) finds how many of them precede
// it in the first run, and a sequential merge of E steps follows.  Lists under
// 512 keys take one wave each (E chosen so that most lanes hold keys); longer
// ones a workgroup.  A list longer than kTileSortCap sorts its
// kTileSortCap-blocks that way and merges them with Batcher's bitonic network
// in global memory (rare: the tile-local binning is chosen for short lists).
// ---------------------------------------------------------------------------
constexpr int kTileSortThreads = 256;
constexpr uint32_t kTileSortCap = 8 * kTileSortThreads;   // 2048 keys (16 KB of LDS)
constexpr uint32_t kTileSortWaveCap = 8 * 64;              // lists below this take one wave
constexpr uint64_t kKeyInf = ~0ull;                        // above every key

__device__ __forceinline__ void cmp_swap(uint64_t &a, uint64_t &b) {
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

template <int E>
__device__ __forceinline__ void sort_regs(uint64_t (&k)[E]) {   // Batcher's networks for 1, 2, 4, 8 keys
    if constexpr (E == 2) {
        cmp_swap(k[0], k[1]);
    } else if constexpr (E == 4) {
        cmp_swap(k[0], k[1]), cmp_swap(k[2], k[3]);
        cmp_swap(k[0], k[2]), cmp_swap(k[1], k[3]);
        cmp_swap(k[1], k[2]);
    } else if constexpr (E == 8) {
        cmp_swap(k[0], k[1]), cmp_swap(k[2], k[3]), cmp_swap(k[4], k[5]), cmp_swap(k[6], k[7]);
        cmp_swap(k[0], k[2]), cmp_swap(k[1], k[3]), cmp_swap(k[4], k[6]), cmp_swap(k[5], k[7]);
        cmp_swap(k[1], k[2]), cmp_swap(k[5], k[6]);
        cmp_swap(k[0], k[4]), cmp_swap(k[1], k[5]), cmp_swap(k[2], k[6]), cmp_swap(k[3], k[7]);
        cmp_swap(k[2], k[4]), cmp_swap(k[3], k[5]);
        cmp_swap(k[1], k[2]), cmp_swap(k[3], k[4]), cmp_swap(k[5], k[6]);
    }
}

// Sorts n keys (n <= E nt, all nt threads calling with their t; thread t
// holds keys E t .. E t + E - 1 in k, kKeyInf past n) using s[0, n) in LDS,
// and writes their low words (the records) in order to dst[0, n).  sync()
// orders the LDS accesses of the nt threads.  E (keys per thread) is 1, 2, 4
// or 8: the smallest that keeps the threads busy.
template <int E, class Sync>
__device__ __forceinline__ void lds_merge_sort(uint64_t *s, uint32_t n, uint32_t t, uint64_t (&k)[E], uint32_t *dst,
                                               Sync sync) {
    const uint32_t d0 = E * t;
    sort_regs<E>(k);
    if (n <= (uint32_t)E) {   // uniform: one thread holds all
#pragma unroll
        for (int q = 0; q < E; ++q)
            if (d0 + q < n) dst[d0 + q] = (uint32_t)k[q];
        return;
    }
#pragma unroll
    for (int q = 0; q < E; ++q)
        if (d0 + q < n) s[d0 + q] = k[q];
    sync();
    for (uint32_t L = E; L < n; L <<= 1) {
        uint64_t o[E];
        uint32_t cnt = 0;
        if (d0 < n) {
            const uint32_t base = d0 & ~(2 * L - 1u), d = d0 - base;
            const uint32_t na = n - base < L ? n - base : L;
            const uint32_t nb = n - base > L ? (n - base - L < L ? n - base - L : L) : 0u;
            const uint64_t *A = s + base, *B = A + L;
            uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
            while (lo < hi) {   // outputs [0, d) hold A[0, lo) and B[0, d - lo)
                const uint32_t mid = (lo + hi) >> 1;
                if (A[mid] < B[d - 1u - mid])
                    lo = mid + 1u;
                else
                    hi = mid;
            }
            uint32_t i = lo, j = d - lo;
            uint64_t ai = i < na ? A[i] : kKeyInf, bj = j < nb ? B[j] : kKeyInf;
            cnt = na + nb - d < (uint32_t)E ? na + nb - d : (uint32_t)E;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                // branch-free: the side taken advances and its next key is read
                // at an address in bounds (the run's first key when past it)
                const bool take = ai < bj;
                o[q] = take ? ai : bj;
                if (q < E - 1) {
                    i += take ? 1u : 0u;
                    j += take ? 0u : 1u;
                    const bool in = take ? i < na : j < nb;
                    const uint64_t nxt = (in && !take ? B : A)[in ? (take ? i : j) : 0u];   // A[0] exists
                    const uint64_t v = in ? nxt : kKeyInf;
                    ai = take ? v : ai;
                    bj = take ? bj : v;
                }
            }
        }
        if (2 * L >= n) {   // the last round writes the records (uniform)
#pragma unroll
            for (int q = 0; q < E; ++q)
                if ((uint32_t)q < cnt) dst[d0 + q] = (uint32_t)o[q];
            return;
        }
        sync();
#pragma unroll
        for (int q = 0; q < E; ++q)
            if ((uint32_t)q < cnt) s[d0 + q] = o[q];
        sync();
    }
}

// Positions (i, l), i < l, of comparator c of a bitonic step with distance j
// (written with ascending comparators only: the first step of the merge of
// two sorted k/2-blocks, j = k / 2, flip, compares i with its mirror image in
// the k-block; the later steps i with i + j).  Over a power of two P >= n,
// positions >= n behave as +inf: no comparator moves a key into them, so the
// comparators that reach past n are skipped.
__device__ __forceinline__ void bitonic_pair(uint32_t c, uint32_t j, bool flip, uint32_t &i, uint32_t &l) {
    const uint32_t off = c & (j - 1u);
    i = ((c - off) << 1) + off;
    l = flip ? i + ((j - off) << 1) - 1u : i + j;
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t n) {
    uint32_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Sorts one tile's list: in = the emission's list, out = the sorted one, both
// over the pair range [ranges[tile].x, ranges[tile].y); zrec = the records'
// depth keys.  big: the whole workgroup calls (a list of kTileSortWaveCap keys
// or more), else one wave with its own kTileSortWaveCap keys of s.  hi / lo:
// scratch over the pair range for the keys of a list longer than kTileSortCap.
// The list [r.x, r.y) of placed (depth key, record) pairs kv[].
__device__ __forceinline__ void sort_tile_list(uint64_t *s, bool big, uint2 r, int64_t K, uint32_t n_rec,
                                               const uint32_t *__restrict__ zrec, const uint2 *__restrict__ kv,
                                               uint32_t *__restrict__ out, uint32_t *__restrict__ hi,
                                               uint32_t *__restrict__ lo, int64_t *__restrict__ error) {
    const uint32_t t = threadIdx.x, wave = t >> 6, lane = t & 63u;
    if (!(r.x < r.y) || (int64_t)r.y > K) return;   // empty (or never expected: out of range); uniform
    const uint32_t n = r.y - r.x;
    const uint2 *src = kv + r.x;
    uint32_t *dst = out + r.x;
    auto block_sync = [] { __syncthreads(); };
    // thread u's E keys (depth key, record) from list[0, m) (all loads in
    // flight together), then the sort of m keys over s
    auto sort_with = [&](auto e, uint64_t *sm, const uint2 *list, uint32_t m, uint32_t u, uint32_t *to, auto sync) {
        constexpr int E = decltype(e)::value;
        uint2 p[E];
        uint64_t k[E];
#pragma unroll
        for (int q = 0; q < E; ++q) p[q] = E * u + q < m ? list[E * u + q] : make_uint2(0u, 0u);
#pragma unroll
        for (int q = 0; q < E; ++q) k[q] = E * u + q < m ? ((uint64_t)p[q].x << 32) | (uint64_t)p[q].y : kKeyInf;
        lds_merge_sort<E>(sm, m, u, k, to, sync);
    };
    if (!big) {   // one wave, its own kTileSortWaveCap keys of LDS
        if (n > kTileSortWaveCap) {   // never expected (nbig counts every such list); noted, not sorted
            if (lane == 0) atomicAdd((unsigned long long *)error, 1ull);
            return;
        }
        uint64_t *w = s + wave * kTileSortWaveCap;
        auto wave_sync = [] {   // LDS operations of a wave complete in order
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        };
        if (n <= 64)
            sort_with(std::integral_constant<int, 1>{}, w, src, n, lane, dst, wave_sync);
        else if (n <= 128)
            sort_with(std::integral_constant<int, 2>{}, w, src, n, lane, dst, wave_sync);
        else if (n <= 256)
            sort_with(std::integral_constant<int, 4>{}, w, src, n, lane, dst, wave_sync);
        else
            sort_with(std::integral_constant<int, 8>{}, w, src, n, lane, dst, wave_sync);
        return;
    }
    constexpr uint32_t NT = kTileSortThreads, C = kTileSortCap;
    if (n <= C) {
        if (n <= 4 * NT)
            sort_with(std::integral_constant<int, 4>{}, s, src, n, t, dst, block_sync);
        else
            sort_with(std::integral_constant<int, 8>{}, s, src, n, t, dst, block_sync);
        return;
    }
    // a long list: its C-blocks merge-sorted into (hi, lo), then Batcher's
    // merges of 2C-blocks and wider, the steps of distance >= C in global
    // memory and the rest within each C-block in LDS
    uint32_t *kh = hi + r.x, *kl = lo + r.x;
    const uint32_t P = pow2_at_least(n), nblk = (n + C - 1) / C;
    for (uint32_t b = 0; b < nblk; ++b) {
        const uint32_t base = b * C, nb = n - base < C ? n - base : C;
        __syncthreads();   // the previous block's use of s
        sort_with(std::integral_constant<int, 8>{}, s, src + base, nb, t, kl + base, block_sync);   // records into lo
        __syncthreads();
        for (uint32_t c = t; c < nb; c += NT) kh[base + c] = zrec[kl[base + c] < n_rec ? kl[base + c] : 0u];
        __syncthreads();
    }
    for (uint32_t k = 2 * C; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j >= C; j >>= 1) {
            const bool flip = j == (k >> 1);
            for (uint32_t c = t; c < (P >> 1); c += NT) {
                uint32_t i, l;
                bitonic_pair(c, j, flip, i, l);
                if (l < n) {
                    const uint64_t a = ((uint64_t)kh[i] << 32) | kl[i], b = ((uint64_t)kh[l] << 32) | kl[l];
                    if (b < a) {
                        kh[i] = (uint32_t)(b >> 32), kl[i] = (uint32_t)b;
                        kh[l] = (uint32_t)(a >> 32), kl[l] = (uint32_t)a;
                    }
                }
            }
            __syncthreads();   // the workgroup's global stores before its next loads
        }
        for (uint32_t b = 0; b < nblk; ++b) {
            const uint32_t base = b * C, nb = n - base < C ? n - base : C, half = pow2_at_least(nb) >> 1;
            for (uint32_t c = t; c < nb; c += NT) s[c] = ((uint64_t)kh[base + c] << 32) | kl[base + c];
            __syncthreads();
            for (uint32_t j = C >> 1; j >= 1; j >>= 1) {   // the half-cleaners of this merge within the block
                for (uint32_t c = t; c < half; c += NT) {
                    uint32_t i, l;
                    bitonic_pair(c, j, false, i, l);
                    if (l < nb) {
                        const uint64_t a = s[i], b2 = s[l];
                        if (b2 < a) {
                            s[i] = b2;
                            s[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
            for (uint32_t c = t; c < nb; c += NT) {
                if (k == P) {
                    dst[base + c] = (uint32_t)s[c];
                } else {
                    kh[base + c] = (uint32_t)(s[c] >> 32);
                    kl[base + c] = (uint32_t)s[c];
                }
            }
            __syncthreads();
        }
    }
}

// Every tile's list sorted.  torder = the tiles by decreasing list length, of
// which the first nbig = counters[kCntSortBig] have kTileSortWaveCap keys or
// more: work item w < nbig is tile torder[w] for a whole workgroup, the later
// items are four short lists each, one per wave; the workgroups loop over the
// items (grid-stride), so none is launched only to find no work.  kv: the
// placed (depth key, record) pairs (zrec: the records' keys, for the long
// lists' merges).
// (register-bound to 6 waves per SIMD, one more than the compiler's own choice
// allows: more lists in flight; 37.0 against 38.4 us on the 8-view step)
__global__ __launch_bounds__(kTileSortThreads) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_tile_sort(const uint2 *__restrict__ ranges,
                                                                const uint32_t *__restrict__ torder, int64_t n_tiles,
                                                                int64_t *__restrict__ counters,
                                                                const uint32_t *__restrict__ zrec,
                                                                const uint2 *__restrict__ kv,
                                                                uint32_t *__restrict__ out, uint32_t *__restrict__ hi,
                                                                uint32_t *__restrict__ lo) {
    __shared__ uint64_t s[kTileSortCap];
    const uint32_t wave = threadIdx.x >> 6;
    const int64_t nbig = counters[kCntSortBig];
    const int64_t K = counters[kCntPairsUsed];
    const uint32_t n_rec = (uint32_t)counters[kCntVisible];
    const int64_t items = nbig + (n_tiles - nbig + 3) / 4;
    for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {   // uniform over the workgroup
        const bool big = w < nbig;
        const int64_t slot = big ? w : nbig + 4 * (w - nbig) + wave;
        if (slot < n_tiles) {   // wave-uniform; always true for a big item
            const uint32_t tile = torder[slot];
            if ((int64_t)tile < n_tiles)   // always true: torder is a permutation
                sort_tile_list(s, big, ranges[tile], K, n_rec, zrec, kv, out, hi, lo, counters + kCntSyncError);
        }
        __syncthreads();   // every wave done with s before the next item
    }
}

}  // namespace gsr
