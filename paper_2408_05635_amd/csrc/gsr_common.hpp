// Internal definitions shared by the gfx950 kernels of the rasteriser:
// the per-view table, the workspace counters and wave64 primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsr.h"

namespace gsr {

// Alpha rules of the compositing (eqs. 2-4 with the usual cut-offs).
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
// Blend blocks: one wave64 composites an 8x8 pixel block, one pixel per lane.
constexpr int kBlk = 8;
constexpr float kLn2f = 0.693147180559945309f;

// Per-view constants, uploaded once per call into the workspace.
struct ViewInfo {
    int32_t W, H;
    float fx, fy, cx, cy;
    int64_t pix_off;    // first pixel of the view in the concatenated images
    int32_t tiles_x, tiles_y, tile_off;   // binning tiles of the view, first global tile id
    int32_t blk_off;                      // first blend block (8x8) of the view
    int32_t pad[2];
};

struct ViewTable {
    int32_t n_views;
    int32_t tile_w, tile_h;
    int32_t total_tiles;
    int32_t total_blocks;
    int32_t pose_centre;   // GSR_POSE_CENTRE: the pose translation input is the camera centre C
    int32_t deterministic; // GSR_DETERMINISTIC: per-pair gradient rows summed in a fixed order
    int32_t pad;
    ViewInfo v[GSR_MAX_VIEWS];
};

// Device counters in the workspace (int64 each).
enum Counter {
    kCntVisible = 0,     // M: visible (view, Gaussian) records
    kCntPairs = 1,       // K needed
    kCntPairsUsed = 2,   // K if it fits the capacity, else 0
    kCntOverflow = 3,    // 1 if K exceeded the capacity
    kCntOverflowAny = 4, // 1 if K exceeded it in any call of a tracking loop (kept across its iterations)
    kCntSyncError = 6,   // waits between blocks that gave up (never expected)
    kCntLossTicket = 7,  // per-view loss blocks that have finished (the last one forms the total)
    // work counters (GSR_COUNT_WORK): (pixel, entry) evaluations and
    // contributions in the forward and backward blends, and (wave, entry)
    // gradient reductions in the backward
    kCntEvalFwd = 8,
    kCntContribFwd = 9,
    kCntEvalBwd = 10,
    kCntContribBwd = 11,
    kCntReduceBwd = 12,
    kCntWorkItems = 13,  // the backward's work items (tiles, or chunks of split lists)
    kCntSortBig = 14,    // tile-local binning: lists that the per-tile sort gives a whole workgroup
    kNumCounters = 16
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` below the calling lane
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the 64 lanes; the total lands in lane 63 (other lanes hold
// partial sums).  Must be called with all 64 lanes active.
__device__ __forceinline__ float wave_sum_to63(float x) {
    x += dpp_f<0xb1>(x);          // quad_perm [1,0,3,2]
    x += dpp_f<0x4e>(x);          // quad_perm [2,3,0,1]
    x += dpp_f<0x114>(x);         // row_shr:4
    x += dpp_f<0x118>(x);         // row_shr:8
    x += dpp_f<0x142, 0xa>(x);    // row_bcast:15 into rows 1 and 3
    x += dpp_f<0x143, 0xc>(x);    // row_bcast:31 into rows 2 and 3
    return x;
}

__device__ __forceinline__ float wave_sum(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to63(x)), 63));
}

__device__ __forceinline__ double wave_sum_f64(double x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    for (int off = 32; off >= 1; off >>= 1) {
        uint32_t y = __shfl_xor(x, off, 64);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ float ld_nc(const float *p) { return __builtin_nontemporal_load(p); }

}  // namespace gsr
