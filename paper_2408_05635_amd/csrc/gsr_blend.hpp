// Front-to-back alpha compositing of RGB (eq. 2), depth (eq. 3) and
// silhouette (eq. 4), and its reverse-order backward.
//
// Work decomposition: one wave64 workgroup per 8x8 pixel block in the
// forward, one wave per 8x8 block of a tile in the backward, one pixel per
// lane.  A block reads the depth-sorted list of the binning tile it lies in,
// 64 entries at a time: each lane fetches one record and tests exactly whether
// the record's alpha >= 1/255 ellipse can reach the 8x8 block (with a safety
// margin, so no contributing entry is ever dropped); survivors are compacted in
// order into LDS and the wave composites them.  Culling never changes a
// result, because an entry with alpha < 1/255 at a pixel leaves that pixel's
// state untouched; it only removes work.
//
// Record layout (3 x float4 per visible (view, Gaussian), depth-sorted):
//   A = (mx_hi, my_hi, mx_lo, my_lo)   mean as an FP32 pair (mx = hi + lo)
//   B = (l11, l21, l22, o)             scaled conic factor and opacity
//   C = (r, g, b, z)                   colour and camera depth
#pragma once

#include <type_traits>

#include "gsr_common.hpp"

namespace gsr {

struct BlockPos {
    int v;            // view
    int tile;         // tile index within the view
    int tg;           // tile index over all views
    int sub;          // the block's place in its tile (row-major 8x8 blocks)
    int bx0, by0;     // top-left pixel of the 8x8 block
    bool valid;
};

// List chunks of the backward.  The reverse walk of a long list is the
// serial path of a whole backward launch, so a tile whose list is longer than
// kSplitMin entries may be walked by several workgroups, one per chunk of
// kChunkEntries entries.  The forward leaves, at every chunk boundary b and
// for every pixel of such a tile, the transmittance in front of entry b and
// the five channel sums over the entries before b; a chunk starts its walk
// from there (T = T_b, and the colour behind = final image - sums, per unit
// of T_b), which is the state the full walk would reach at b.
constexpr uint32_t kChunkEntries = 128;   // a multiple of 64: the forward's staging rounds meet every boundary
constexpr uint32_t kSplitMin = 192;
constexpr uint32_t kMaxChunks = 256;      // chunk index in the top 8 bits of a work item
constexpr uint32_t kNoSplit = 0xffffffffu;
constexpr int kCpValues = 6;              // T, r, g, b, depth, silhouette

__device__ __forceinline__ uint32_t chunks_of(uint32_t len) { return (len + kChunkEntries - 1) / kChunkEntries; }

// checkpoint value q of lane `lane` of block `sub` in slot `slot`
__device__ __forceinline__ size_t cp_index(uint32_t slot, int nsub, int sub, int q, uint32_t lane) {
    return (((size_t)slot * (size_t)nsub + (size_t)sub) * kCpValues + (size_t)q) * 64 + lane;
}

// The block of workgroup i: tiles go heaviest first (torder, a permutation of
// the tiles), tile rank r to XCD r mod 8 (the hardware deals workgroups to the
// XCDs in turn), and the sub-blocks of a tile run one after the other on the
// same XCD, whose L2 then holds the tile's records for all of them:
// i = 8 (nsub floor(r / 8) + sub) + r mod 8.
__device__ __forceinline__ BlockPos locate_block(const ViewTable *vt, const uint32_t *__restrict__ torder) {
    BlockPos bp;
    const int sx = vt->tile_w / kBlk, sy = vt->tile_h / kBlk, nsub = sx * sy;
    const int32_t T = vt->total_tiles;
    const uint32_t i = blockIdx.x, k = i >> 3;
    const int32_t r = (int32_t)(8u * (k / (uint32_t)nsub) + (i & 7u));
    const int sub = (int)(k % (uint32_t)nsub);
    bp.valid = r < T;
    if (!bp.valid) return bp;
    const int32_t tg = (int32_t)torder[r];
    bp.valid = tg < T;   // always true for a permutation; keeps reads in bounds
    if (!bp.valid) return bp;
    int v = 0;
    while (v + 1 < vt->n_views && vt->v[v + 1].tile_off <= tg) ++v;
    bp.v = v;
    const ViewInfo &V = vt->v[v];
    const int tile = tg - V.tile_off;
    const int ty = tile / V.tiles_x, tx = tile - ty * V.tiles_x;
    bp.tile = tile;
    bp.tg = tg;
    bp.sub = sub;
    bp.bx0 = tx * vt->tile_w + (sub % sx) * kBlk;
    bp.by0 = ty * vt->tile_h + (sub / sx) * kBlk;
    bp.valid = bp.bx0 < V.W && bp.by0 < V.H;
    return bp;
}

// Can the record reach alpha >= 1/255 anywhere in the 8x8 block?  The
// quadratic form Q = (l11 dx + l21 dy)^2 + (l22 dy)^2 is minimised over the
// block's box: zero if the mean is inside, else the least value along the four
// edges (each edge's minimiser is the clamped 1-D minimiser, located with a
// hardware reciprocal: its error moves Q only to second order).  Kept when
// Q_min <= log2(255 o) with a relative margin of 2^-8, far above FP32 rounding.
__device__ __forceinline__ bool block_may_contribute(const float4 A, const float4 B, float bx0, float by0) {
    const float o = B.w;
    if (!(255.0f * o > 1.0f)) return false;
    const float qcut = __builtin_amdgcn_logf(255.0f * o);   // log2
    const float mx = A.x + A.z, my = A.y + A.w;
    const float dx0 = bx0 - mx, dx1 = bx0 + (float)(kBlk - 1) - mx;
    const float dy0 = by0 - my, dy1 = by0 + (float)(kBlk - 1) - my;
    if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return true;
    const float l11 = B.x, l21 = B.y, l22 = B.z;
    const float qa = l11 * l11, qb = l11 * l21, qc = l21 * l21 + l22 * l22;
    auto Q = [&](float dx, float dy) {
        const float u = l11 * dx + l21 * dy, w = l22 * dy;
        return u * u + w * w;
    };
    auto clampf = [](float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); };
    const float rqc = __builtin_amdgcn_rcpf(qc), rqa = __builtin_amdgcn_rcpf(qa);
    float q = Q(dx0, clampf(-qb * dx0 * rqc, dy0, dy1));
    q = fminf(q, Q(dx1, clampf(-qb * dx1 * rqc, dy0, dy1)));
    q = fminf(q, Q(clampf(-qb * dy0 * rqa, dx0, dx1), dy0));
    q = fminf(q, Q(clampf(-qb * dy1 * rqa, dx0, dx1), dy1));
    return q <= qcut * (1.0f + 0x1p-8f) + 0x1p-10f;
}

// alpha of one record at one pixel; identical instruction sequence in the
// forward and the backward kernels (explicit fma, no contraction), so both
// take the same decisions.  The record enters through its offset from the
// 8x8 block's origin, d0 = (bx0 - mx, by0 - my), formed once per (block,
// entry) by block_offset; the pixel adds its place (jx, jy) in the block.
struct AlphaEval {
    float dx, dy, u, w, G, alpha;
    bool clamped;
};

__device__ __forceinline__ float2 block_offset(const float4 A, float bx0, float by0) {
    return make_float2(__fsub_rn(__fsub_rn(bx0, A.x), A.z), __fsub_rn(__fsub_rn(by0, A.y), A.w));
}

__device__ __forceinline__ AlphaEval eval_alpha(const float2 d0, const float4 B, float jx, float jy) {
#pragma clang fp contract(off)
    AlphaEval e;
    e.dx = __fadd_rn(d0.x, jx);
    e.dy = __fadd_rn(d0.y, jy);
    e.u = __builtin_fmaf(B.y, e.dy, __fmul_rn(B.x, e.dx));
    e.w = __fmul_rn(B.z, e.dy);
    const float p2 = -__builtin_fmaf(e.u, e.u, __fmul_rn(e.w, e.w));
    e.G = __builtin_amdgcn_exp2f(p2);
    const float og = __fmul_rn(B.w, e.G);
    e.clamped = og > kAlphaMax;
    e.alpha = fminf(og, kAlphaMax);   // og for og <= kAlphaMax (a min, one instruction where clamped is unused)
    return e;
}

struct BlendOut {
    float *rgb, *depth, *sil;   // images
    float *t_final;             // per pixel
    uint32_t *n_last;           // per pixel: list position + 1 of the last contributor (0: none)
    uint32_t *hash;             // per pixel: hash of the contributing records, clamp flags and the stop
    uint64_t *cmask;            // the forward's culling decisions, for the backward (cmask_index)
};

// The forward's culling ballot of list entries [start + 64 c, start + 64 c +
// 64) of tile tg (list range [start, end)) for 8x8 block `sub` of the tile:
// word (start / 64 + tg + c) nsub + sub.  The words of successive tiles do not
// overlap (a tile's ceil((end - start) / 64) words end by end / 64 + tg + 1),
// so the array needs K / 64 + T + 2 words per block of a tile.  The backward
// takes these bits instead of repeating block_may_contribute: the same test
// for the same block, so the same decisions.
__device__ __forceinline__ size_t cmask_index(uint32_t start, int32_t tg, uint32_t rel, int nsub, int sub) {
    return ((size_t)(start >> 6) + (size_t)tg + (size_t)(rel >> 6)) * (size_t)nsub + (size_t)sub;
}

// HASH: also fold the pixel's decisions into out.hash (a test hook; 0 otherwise).
template <bool COUNT, bool HASH>
__global__ __launch_bounds__(64) void k_blend_fwd(const ViewTable *__restrict__ vt, const float4 *__restrict__ rec,
                                                  const uint32_t *__restrict__ pair_rec,
                                                  const uint2 *__restrict__ ranges,
                                                  const uint32_t *__restrict__ torder,
                                                  const uint32_t *__restrict__ cpoff, float *__restrict__ cp,
                                                  int64_t *__restrict__ counters, BlendOut out) {
    // staged entries: offset from the block origin (x, y; float4-strided like
    // the others, so that one base address serves all three), B and C
    __shared__ float4 s_d[64], s_b[64], s_c[64];
    __shared__ uint32_t s_pos[64], s_rec_id[64];
    const BlockPos bp = locate_block(vt, torder);
    if (!bp.valid) return;
    const ViewInfo &V = vt->v[bp.v];
    const uint32_t lane = threadIdx.x;
    const int px = bp.bx0 + (int)(lane & 7u), py = bp.by0 + (int)(lane >> 3);
    const bool inside = px < V.W && py < V.H;
    const float fjx = (float)(lane & 7u), fjy = (float)(lane >> 3);   // the pixel's place in its block
    uint2 rg = ranges[V.tile_off + bp.tile];
    const uint32_t n_rec = (uint32_t)counters[kCntVisible];
    const uint32_t n_pair = (uint32_t)counters[kCntPairsUsed];
    if (rg.y > n_pair || rg.x > rg.y) rg = make_uint2(0u, 0u);   // never expected; keeps reads in bounds

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, cd = 0.0f, cs = 0.0f;
    uint32_t last = 0, n_eval = 0, n_contrib = 0, hsh = 0x811c9dc5u;
    bool done = !inside;
    // chunk boundaries of a split list: the state in front of entry rg.x + j C
    const uint32_t cpo = cpoff[bp.tg];
    const uint32_t n_ch = rg.y > rg.x ? chunks_of(rg.y - rg.x) : 1u;
    const uint32_t n_cp = (cpo != kNoSplit && n_ch <= kMaxChunks) ? n_ch - 1u : 0u;
    const int nsub = (vt->tile_w / kBlk) * (vt->tile_h / kBlk);
    uint32_t next_cp = 1;
    auto write_cp = [&](uint32_t j) {
        float *d = cp + cp_index(cpo + (j - 1u), nsub, bp.sub, 0, lane);
        d[0] = T;
        d[64] = c0;
        d[128] = c1;
        d[192] = c2;
        d[256] = cd;
        d[320] = cs;
    };
    // The list is read one round ahead of its use, so that a round's loads
    // wait behind the compositing of the round before: the list entries of
    // round c + 128 and the records of round c + 64 are requested during round
    // c (a sentinel >= n_rec past the list's end).
    auto list_entry = [&](uint32_t c) { return c + lane < rg.y ? pair_rec[c + lane] : 0xffffffffu; };
    float4 A, B, C;
    auto load_rec = [&](uint32_t s, float4 &a, float4 &b, float4 &cc) {
        if (s < n_rec) {
            a = rec[3 * (size_t)s];
            b = rec[3 * (size_t)s + 1];
            cc = rec[3 * (size_t)s + 2];
        }
    };
    uint32_t s = list_entry(rg.x);
    load_rec(s, A, B, C);
    uint32_t s_next = list_entry(rg.x + 64u);
    for (uint32_t c = rg.x; c < rg.y; c += 64) {
        if (ballot(!done) == 0) break;
        if (next_cp <= n_cp && c == rg.x + next_cp * kChunkEntries) write_cp(next_cp++);   // wave-uniform
        const uint32_t e = c + lane;
        float4 A2, B2, C2;
        load_rec(s_next, A2, B2, C2);
        const uint32_t s_after = list_entry(c + 128u);
        const bool keep = s < n_rec && block_may_contribute(A, B, (float)bp.bx0, (float)bp.by0);
        const uint64_t m = ballot(keep);
        if (lane == 0) out.cmask[cmask_index(rg.x, bp.tg, c - rg.x, nsub, bp.sub)] = m;
        if (keep) {
            const uint32_t slot = rank_below(m);
            const float2 d0 = block_offset(A, (float)bp.bx0, (float)bp.by0);
            s_d[slot] = make_float4(d0.x, d0.y, 0.0f, 0.0f);
            s_b[slot] = B;
            s_c[slot] = C;
            s_pos[slot] = e;
            if (HASH) s_rec_id[slot] = s;
        }
        __syncthreads();
        const int n = __popcll(m);
        // staging slot of this lane's last contributor within the chunk (-1:
        // none yet); turned into the list position once the chunk is done
        int lastk = -1;
        // Every lane evaluates; a lane that is done, or that the entry does
        // not reach, takes weight 0, which leaves its sums exactly as they
        // were (fma(0, c, x) = x), so the updates need no branches.
        auto entry = [&](int k) {
            const float4 d4 = s_d[k];
            const AlphaEval ev = eval_alpha(make_float2(d4.x, d4.y), s_b[k], fjx, fjy);
            if (COUNT) n_eval += done ? 0u : 1u;
            const bool hit = !done && ev.alpha >= kAlphaMin;
            const float Tn = __builtin_fmaf(-ev.alpha, T, T);   // T (1 - alpha), rounded once
            const bool stop = hit && Tn < kTMin;
            const bool take = hit != stop;   // hit and not stopped
            if (COUNT) n_contrib += take ? 1u : 0u;
            const float4 cc = s_c[k];
            const float wgt = take ? ev.alpha * T : 0.0f;
            c0 = __builtin_fmaf(wgt, cc.x, c0);
            c1 = __builtin_fmaf(wgt, cc.y, c1);
            c2 = __builtin_fmaf(wgt, cc.z, c2);
            cd = __builtin_fmaf(wgt, cc.w, cd);
            cs += wgt;
            T = take ? Tn : T;
            lastk = take ? k : lastk;
            if (HASH) {
                uint32_t rid2 = 2u * s_rec_id[k] + (ev.clamped ? 1u : 0u);
                asm volatile("" : "+v"(rid2));
                const uint32_t hin = take ? rid2 : 0xffffffffu;
                hsh = (take || stop) ? (hsh ^ hin) * 0x01000193u : hsh;
            }
            done = done || stop;
        };
        // groups of 8 entries (LDS addresses as immediate offsets), then the
        // wave checks whether any of its pixels is still open
        for (int k0 = 0; k0 < n; k0 += 8) {
            // the group's first slot held in a vector register, so the
            // entries' staging reads take one base and immediate offsets
            int vk = k0;
            asm volatile("" : "+v"(vk));
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (k0 + j < n) entry(vk + j);
            if (ballot(!done) == 0) break;
        }
        if (lastk >= 0) last = s_pos[lastk] + 1u;
        __syncthreads();
        s = s_next;
        s_next = s_after;
        A = A2;
        B = B2;
        C = C2;
    }
    for (; next_cp <= n_cp; ++next_cp) write_cp(next_cp);   // boundaries past the end: the final state
    if (COUNT) {
        const uint32_t e = wave_sum_u32(n_eval), c = wave_sum_u32(n_contrib);
        if (lane == 0) {
            atomicAdd((unsigned long long *)&counters[kCntEvalFwd], (unsigned long long)e);
            atomicAdd((unsigned long long *)&counters[kCntContribFwd], (unsigned long long)c);
        }
    }
    if (inside) {
        const int64_t P = (int64_t)V.W * V.H;
        const int64_t pix = (int64_t)py * V.W + px;
        out.rgb[3 * V.pix_off + pix] = c0;
        out.rgb[3 * V.pix_off + P + pix] = c1;
        out.rgb[3 * V.pix_off + 2 * P + pix] = c2;
        out.depth[V.pix_off + pix] = cd;
        out.sil[V.pix_off + pix] = cs;
        out.t_final[V.pix_off + pix] = T;
        out.n_last[V.pix_off + pix] = last;
        out.hash[V.pix_off + pix] = HASH ? hsh : 0u;
    }
}

// Loss weights and targets for the fused loss, or upstream image gradients.
struct LossIn {
    const float *t_rgb, *t_depth, *t_sil, *t_prior, *t_weight;
    float w_rgb, w_depth, w_sil, w_prior, sil_thresh;
    const float *g_rgb, *g_depth, *g_sil;   // upstream dL/dimage (split backward)
    double *loss;                           // [V] per-view loss (fused; written by loss_final_view)
    double *loss_tile;                      // [tiles] per-tile loss partials (fused, workspace)
};

__device__ __forceinline__ float sgnf(float x) { return (float)((x > 0.0f) - (x < 0.0f)); }

// Backward blend.  One workgroup per work item, a binning tile or one chunk
// of a split list, one wave per 8x8 block of the tile (tiles are at most
// 32x32, so at most sixteen waves).  The item's entries are walked in reverse,
// from the last contributor of any pixel of the tile, in segments of kSeg
// entries; within a segment every wave reads the forward's culling decisions
// for its own block (one lane per entry, one bit each), then takes the
// survivors one by one, reading
// each one's record at a wave-uniform address (scalar loads, no LDS staging),
// and sums each entry's partial derivatives over its 64 pixels (DPP quad
// sums, then a batched column sum in LDS) into its own LDS slots.
// At the end of the segment the waves' slots are added in a fixed order and
// written, without atomics, to the pair's own row of `grad_pairs`: record s
// owns the rows [poff[s], poff[s] + tiles of s), one per tile of its
// rectangle in row-major order, so that a record's rows are contiguous.
// Every pair of the list gets exactly one row per call.
//
// Partial derivatives per (pixel, entry), for alpha = o exp2(p2),
// p2 = -(u^2 + w^2), u = l11 dx + l21 dy, w = l22 dy, dx = px - mx:
//   dL/dalpha = T_k sum_ch g_ch (f_ch - B_ch)    (B: colour behind, per unit of
//                                                 the transmittance after k)
//             = T_k (S_k - W)   with S_k = sum_ch g_ch f_ch (f_sil = 1) and
//                               W = sum_ch g_ch B_ch, which obeys the same
//                               recursion as each B_ch: W <- alpha S_k + (1 - alpha) W
//   dL/df_ch  = g_ch alpha T_k                   (rgb and depth)
//   dL/do = dL/dalpha G,  dL/dp2 = dL/dalpha alpha ln2   (unless clamped)
//   dL/dmx = dL/dp2 2u l11,  dL/dmy = dL/dp2 2(u l21 + w l22)
//   dL/dl11 = -dL/dp2 2u dx, dL/dl21 = -dL/dp2 2u dy, dL/dl22 = -dL/dp2 2w dy
// With 2 dL/dp2 = k dL/do, k = 2 o ln2, and (k, l11, l21, l22) fixed per entry,
// a pair's row holds R = (sum u dL/do, sum w dL/do, -sum u dx dL/do,
// -sum u dy dL/do, -sum w dy dL/do, sum dL/do, sum dL/df_ch) over the tile's
// pixels, and the record's backward applies the factors to the summed rows:
// dL/dmx = k l11 R0, dL/dmy = k (l21 R0 + l22 R1), dL/dl.. = k R2..R4.
// Pose-only rows (NV = 6) hold R0..R4 and the depth partial.
// Sums of each value over every quad of lanes (4 neighbouring pixels of a
// row), the NV chains interleaved; afterwards every lane of a quad holds the
// quad's sums.  Contraction is off so that each stage stays one DPP add (fused
// with the product that made the value, the add would become an FMA, whose
// addend cannot take the DPP operand).  The empty asm keeps the last stage in
// front of the caller's store branch: sunk into it, each add would split into
// a DPP move for all lanes and a masked add.
template <int NV>
__device__ __forceinline__ void quad_sums(float (&d)[NV]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int c = 0; c < NV; ++c) d[c] += dpp_f<0xb1>(d[c]);    // quad_perm [1,0,3,2]
#pragma unroll
    for (int c = 0; c < NV; ++c) d[c] += dpp_f<0x4e>(d[c]);    // quad_perm [2,3,0,1]
#pragma unroll
    for (int c = 0; c < NV; ++c) asm volatile("" : "+v"(d[c]));
}

// Waves of a backward workgroup, one per 8x8 block of the tile: tiles up to
// 16x16 (or 32x8) take the 4-wave build, larger ones (32x16, 32x32) the
// 16-wave build, whose LDS arrays are sized for 16 waves.
constexpr int kBwdWavesSmall = 4;
constexpr int kBwdWavesLarge = 16;
// List entries per segment: 48 with all gradients (NV = 10), whose LDS then
// leaves room for 8 workgroups per CU; 64 with pose gradients only, whose
// smaller slots keep that occupancy at the longer segment.
template <int NV>
constexpr int seg_entries() { return NV == 10 ? 48 : 64; }
constexpr int kRowStride = 10;   // floats per record row of the atomic backward (NV of them used)

// NV = 10: all partials per entry (dL/d of the conic factors and mean, opacity,
// colour, depth).  NV = 6 (pose only): the opacity and colour partials do not
// reach the pose, so only (0..4, depth) are formed, reduced and written.
// ATOMIC: instead of a row per (tile, entry), each entry's sum over the tile
// is added with global float atomics (skipping exact zeros) to its record's
// row, grad_pairs[kRowStride * record], zeroed by the gather; entries no pixel
// reaches cost nothing.  The sums then arrive in a varying order.
template <bool FUSED, bool COUNT, int NV, bool ATOMIC, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_blend_bwd(const ViewTable *__restrict__ vt, const float4 *__restrict__ rec,
                                                   const uint32_t *__restrict__ pair_rec,
                                                   const uint32_t *__restrict__ poff, const uint2 *__restrict__ trect,
                                                   const uint2 *__restrict__ ranges,
                                                   const uint32_t *__restrict__ work, const int64_t *__restrict__ n_work,
                                                   const uint32_t *__restrict__ cpoff, const float *__restrict__ cp,
                                                   int64_t *__restrict__ counters, BlendOut st, LossIn L,
                                                   float *__restrict__ grad_pairs) {
    // The NV partials of an entry are summed over the wave in two steps: DPP
    // sums over each quad of lanes, stored by the quad's first lane into
    // s_q[wave][batch slot][quad][NV]; once kBatch entries are stored, lane
    // (k, c) adds the 16 quad sums of value c of entry k, in quad order, into
    // s_acc[wave][entry of the segment][c].
    constexpr int kBatch = 40 / NV;   // entries per batch: 4 (NV = 10) or 6 (NV = 6), LDS sized for occupancy
    // batch slots kQStride floats apart: 16 quads x NV values, padded by 8
    // floats so that the column sums of a batch's entries (lanes (k, c) reading
    // slot k, value c) fall in different LDS banks, where a stride of 160
    // (a multiple of the bank count) put the four slots' value c in one bank
    constexpr int kQStride = 16 * NV + 8;
    __shared__ float s_q[WAVES][kBatch * kQStride];
    constexpr int kSeg = seg_entries<NV>();
    __shared__ float s_acc[WAVES][kSeg * NV];
    __shared__ uint32_t s_wmax[WAVES];
    __shared__ uint32_t s_j[kSeg];   // gradient-row slot of each entry of the segment
    __shared__ float2 s_d[WAVES][kSeg];   // per wave: the segment's entries' offsets from the block origin
    __shared__ double s_loss[WAVES];

    // work item of this workgroup: the i-th (tile, chunk) of the order, longest
    // first (the hardware deals workgroups to the XCDs in turn, so the long
    // ones spread over all of them)
    const int32_t T_all = vt->total_tiles;
    if ((int64_t)blockIdx.x >= *n_work) return;
    const uint32_t item = work[blockIdx.x];
    const int32_t tid_g = (int32_t)(item & 0xffffffu);
    const uint32_t chunk = item >> 24;
    if (tid_g >= T_all) return;   // never expected; keeps reads in bounds
    int v = 0;
    while (v + 1 < vt->n_views && vt->v[v + 1].tile_off <= tid_g) ++v;
    const ViewInfo &V = vt->v[v];
    const int tile = tid_g - V.tile_off;
    const int ty = tile / V.tiles_x, tx = tile - ty * V.tiles_x;
    const int sx = vt->tile_w / kBlk;
    const int nw = (vt->tile_w / kBlk) * (vt->tile_h / kBlk);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const int bx0 = tx * vt->tile_w + (int)(wave % sx) * kBlk;
    const int by0 = ty * vt->tile_h + (int)(wave / sx) * kBlk;
    const int px = bx0 + (int)(lane & 7u), py = by0 + (int)(lane >> 3);
    const bool inside = px < V.W && py < V.H;
    const float fjx = (float)(lane & 7u), fjy = (float)(lane >> 3);   // the pixel's place in its block
    const int64_t P = (int64_t)V.W * V.H;
    const int64_t pix = (int64_t)py * V.W + px;
    const int64_t gp = V.pix_off + pix;

    // dL/d(r, g, b, depth, silhouette) at this pixel
    float g[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    float T = 1.0f;
    uint32_t last = 0;
    double lp = 0.0;   // this pixel's loss term (fused)
    if (inside) {
        T = st.t_final[gp];
        last = st.n_last[gp];
        if (FUSED) {
            const float wgt = L.t_weight ? L.t_weight[gp] : 1.0f;
            if (wgt != 0.0f) {
                const float C0 = st.rgb[3 * V.pix_off + pix], C1 = st.rgb[3 * V.pix_off + P + pix],
                            C2 = st.rgb[3 * V.pix_off + 2 * P + pix];
                const float D = st.depth[gp], S = st.sil[gp];
                const float r0 = C0 - L.t_rgb[3 * V.pix_off + pix];
                const float r1 = C1 - L.t_rgb[3 * V.pix_off + P + pix];
                const float r2 = C2 - L.t_rgb[3 * V.pix_off + 2 * P + pix];
                const float td = L.t_depth[gp];
                const float rd = D - td;
                const float rs = S - (L.t_sil ? L.t_sil[gp] : 0.0f);
                const float tp = L.t_prior ? L.t_prior[gp] : 0.0f;
                const float rp = D - tp;
                const float trk = (L.sil_thresh >= 0.0f) ? (S > L.sil_thresh ? 1.0f : 0.0f) : 1.0f;
                const float dm = td > 0.0f ? 1.0f : 0.0f;
                const float dpr = tp > 0.0f ? 1.0f : 0.0f;
                const float sc = wgt / (float)P;
                const double scd = (double)wgt / (double)P;
                lp = scd * ((double)(trk * dm) * ((double)L.w_rgb * (fabs((double)r0) + fabs((double)r1) + fabs((double)r2)) +
                                                   (double)L.w_depth * fabs((double)rd)) +
                            (double)L.w_sil * fabs((double)rs) + (double)(trk * dpr) * (double)L.w_prior * fabs((double)rp));
                g[0] = sc * trk * dm * L.w_rgb * sgnf(r0);
                g[1] = sc * trk * dm * L.w_rgb * sgnf(r1);
                g[2] = sc * trk * dm * L.w_rgb * sgnf(r2);
                g[3] = sc * (trk * dm * L.w_depth * sgnf(rd) + trk * dpr * L.w_prior * sgnf(rp));
                g[4] = sc * L.w_sil * sgnf(rs);
            }
        } else {
            if (L.g_rgb) {
                g[0] = L.g_rgb[3 * V.pix_off + pix];
                g[1] = L.g_rgb[3 * V.pix_off + P + pix];
                g[2] = L.g_rgb[3 * V.pix_off + 2 * P + pix];
            }
            if (L.g_depth) g[3] = L.g_depth[gp];
            if (L.g_sil) g[4] = L.g_sil[gp];
        }
    }
    if (FUSED) {   // all 64 lanes take part in the reduction
        const double tot = wave_sum_f64(lp);
        if (lane == 0) s_loss[wave] = tot;
    }
    if (!(g[0] != 0.f || g[1] != 0.f || g[2] != 0.f || g[3] != 0.f || g[4] != 0.f)) last = 0;

    uint2 rg = ranges[tid_g];
    const uint32_t n_rec = (uint32_t)counters[kCntVisible];
    const uint32_t n_pair = (uint32_t)counters[kCntPairsUsed];
    if (rg.y > n_pair || rg.x > rg.y) rg = make_uint2(0u, 0u);   // never expected; keeps reads in bounds
    // this workgroup's entries [lo, hi): the whole list, or one chunk of a split one
    const uint32_t cpo = cpoff[tid_g];
    const uint32_t n_ch = rg.y > rg.x ? chunks_of(rg.y - rg.x) : 1u;
    const bool split = cpo != kNoSplit && n_ch <= kMaxChunks;
    uint32_t lo = rg.x, hi = rg.y;
    if (split) {
        lo = rg.x + chunk * kChunkEntries < rg.y ? rg.x + chunk * kChunkEntries : rg.y;
        hi = lo + kChunkEntries < rg.y ? lo + kChunkEntries : rg.y;
    } else if (chunk != 0u) {
        lo = hi = rg.y;   // never expected: only split lists have chunks past the first
    }
    // a chunk before the last starts from the forward's state at hi (W: the
    // colour behind, weighted by dL/d(channel), per unit of T)
    float W = 0.f;
    if (split && hi < rg.y && inside) {
        const int nsub = (vt->tile_w / kBlk) * (vt->tile_h / kBlk);
        const float *c = cp + cp_index(cpo + chunk, nsub, (int)wave, 0, lane);
        const float Tb = c[0];
        const float b0 = st.rgb[3 * V.pix_off + pix] - c[64];
        const float b1 = st.rgb[3 * V.pix_off + P + pix] - c[128];
        const float b2 = st.rgb[3 * V.pix_off + 2 * P + pix] - c[192];
        const float bd = st.depth[gp] - c[256];
        const float bs = st.sil[gp] - c[320];
        W = (g[0] * b0 + g[1] * b1 + g[2] * b2 + g[3] * bd + g[4] * bs) / Tb;
        T = Tb;
    }
    const uint32_t wmax = wave_max_u32(last);
    if (lane == 0) s_wmax[wave] = wmax;
    __syncthreads();
    if (FUSED && threadIdx.x == 0 && chunk == 0u) {   // the tile's loss: its waves in a fixed order
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += s_loss[w];
        L.loss_tile[tid_g] = t;
    }
    uint32_t bmax = rg.x;
    for (int w = 0; w < nw; ++w) bmax = s_wmax[w] > bmax ? s_wmax[w] : bmax;
    const uint32_t top = bmax < lo ? lo : (bmax > hi ? hi : bmax);   // the walk starts here
    // The gradient row of entry e: records own the rows [poff, poff + tiles)
    // of their tile rectangles, row-major, so the slot follows from the
    // record and this tile's place in its rectangle (~0u: not a valid entry).
    auto row_of = [&](uint32_t e) -> uint32_t {
        const uint32_t s = pair_rec[e];
        if (s >= n_rec) return ~0u;   // never expected; keeps writes in bounds
        if constexpr (ATOMIC) return s;   // the record's own row
        const uint2 tr = trect[s];
        const uint32_t tx0 = tr.x & 0xffffu, nx = (tr.x >> 16) - tx0 + 1u, ty0 = tr.y & 0xffffu;
        const uint32_t j = poff[s] + ((uint32_t)ty - ty0) * nx + ((uint32_t)tx - tx0);
        return j < n_pair ? j : ~0u;
    };
    // entries behind every pixel's last contributor get zero rows
    for (uint32_t e = top + threadIdx.x; !ATOMIC && e < hi; e += blockDim.x) {
        const uint32_t j = row_of(e);
        if (j == ~0u) continue;
        float *dst = grad_pairs + NV * (size_t)j;
#pragma unroll
        for (int c = 0; c < NV; ++c) dst[c] = 0.0f;
    }

    // W: sum over the channels of dL/d(channel) x (channel behind the current entry)
    uint32_t n_eval = 0, n_contrib = 0, n_red = 0;
    float *qs = &s_q[wave][0];
    const uint32_t fk = lane / NV, fc = lane - fk * NV;   // the batch entry and the value this lane adds up
    // Adds the quad sums of the batch's nb entries (lanes of one wave; LDS
    // operations of a wave complete in order, so no barrier beyond the wave's).
    // bpack: the batch entries' places in the segment, 6 bits each (a
    // wave-uniform value, held in scalar registers).
    using Pack = std::conditional_t<6 * kBatch <= 32, uint32_t, uint64_t>;
    static_assert(6 * kBatch <= 64, "batch places fit one 64-bit word");
    auto flush = [&](uint32_t nb, Pack bpack) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (fk < nb) {
            const float *src = qs + fk * kQStride + fc;
            float sum = src[0];
#pragma unroll
            for (int q = 1; q < 16; ++q) sum += src[q * NV];
            const uint32_t slot = (uint32_t)(bpack >> (6u * fk)) & 63u;
            s_acc[wave][slot * NV + fc] = sum;   // 32-bit LDS index
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    // A segment's list entries and the forward's culling words for them are
    // read one segment ahead (the lane's entry seg_lo + lane, ~0u where the
    // wave has none), so that only the kept entries' records are read when a
    // segment starts.
    auto seg_lo_of = [&](uint32_t hi_) { return hi_ - lo > (uint32_t)kSeg ? hi_ - kSeg : lo; };
    uint32_t pf_s = ~0u;
    uint64_t pf_cm = 0;
    auto prefetch = [&](uint32_t slo, uint32_t shi) {
        const uint32_t whi = wmax < shi ? wmax : shi;   // this wave's last entry + 1 in the segment
        const uint32_t e = slo + lane;
        pf_s = ~0u;
        pf_cm = 0;
        if (wmax > slo && lane < (uint32_t)kSeg && e < whi) {
            pf_s = pair_rec[e];
            pf_cm = st.cmask[cmask_index(rg.x, tid_g, e - rg.x, nw, (int)wave)];
        }
    };
    if (top > lo) prefetch(seg_lo_of(top), top);
    for (uint32_t seg_hi = top; seg_hi > lo;) {
        const uint32_t seg_lo = seg_lo_of(seg_hi);
        const uint32_t s_cur = pf_s;
        const uint64_t cm_cur = pf_cm;
        if (seg_lo > lo) prefetch(seg_lo_of(seg_lo), seg_lo);
        for (int c = lane; c < kSeg * NV; c += 64) s_acc[wave][c] = 0.0f;
        if (threadIdx.x < seg_hi - seg_lo) s_j[threadIdx.x] = row_of(seg_lo + threadIdx.x);   // read after the barrier
        if (wmax > seg_lo) {   // wave-uniform: this wave has pixels with entries in the segment
            const uint32_t e = seg_lo + lane;
            bool keep = false;
            uint32_t s = 0;
            if (s_cur < n_rec) {   // an entry of this wave in the segment
                // the forward's decision for this entry and block
                keep = (cm_cur >> ((e - rg.x) & 63u)) & 1ull;
                if (keep) {
                    s = s_cur;
                    s_d[wave][lane] = block_offset(rec[3 * (size_t)s], (float)bx0, (float)by0);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the offsets before the entries read them
            __builtin_amdgcn_wave_barrier();
            // survivors in reverse list order: the lanes of the set bits of mm, highest first;
            // an entry's record is read at a wave-uniform address (scalar loads)
            uint64_t mm = ballot(keep);
            uint32_t nb = 0;   // entries stored in the batch (wave-uniform)
            Pack bpack = 0;   // their places in the segment (wave-uniform)
            auto entry = [&](int src) {
                const uint32_t pos = seg_lo + (uint32_t)src;
                const uint32_t rs = __builtin_amdgcn_readlane(s, src);
                const bool act = pos < last;
                const uint64_t m_act = ballot(act);
                if (m_act == 0) return;   // wave-uniform
                const float4 b = rec[3 * (size_t)rs + 1];
                // every lane evaluates (the wave pays for it either way); the
                // decisions and the state updates are selects, not branches
                const AlphaEval ev = eval_alpha(s_d[wave][src], b, fjx, fjy);
                const bool reach = ev.alpha >= kAlphaMin;
                const bool contrib = act && reach;
                if (COUNT) n_eval += act ? 1u : 0u;
                if ((ballot(reach) & m_act) == 0) return;   // wave-uniform: nothing to add for this entry
                if (COUNT) {
                    n_contrib += contrib ? 1u : 0u;
                    ++n_red;
                }
                const float4 cc = rec[3 * (size_t)rs + 2];
                // A lane that does not take this entry continues with alpha = 0:
                // every update below then leaves its state exactly as it was
                // (fma(0, S - W, W) = W, T rcp(1) = T) and every partial is
                // zero, so no branch and no select is needed for the state.
                const float ae = contrib ? ev.alpha : 0.0f;
                const float oma = 1.0f - ae;
                const float Tk = T * __builtin_amdgcn_rcpf(oma);   // transmittance in front of this entry
                const float S = __builtin_fmaf(g[0], cc.x, __builtin_fmaf(g[1], cc.y, __builtin_fmaf(g[2], cc.z, __builtin_fmaf(g[3], cc.w, g[4]))));
                const float sw = S - W;
                const float dal = Tk * sw;
                // unclamped: alpha = o G, so dL/do = dL/dalpha G and
                // 2 dL/dp2 = dL/dalpha alpha 2 ln2 = dL/do (2 o ln2); the
                // entry's constant factors (2 o ln2, l11, l21, l22) are applied
                // to the row sums, once per record
                const float dop = dal * ((contrib && !ev.clamped) ? ev.G : 0.0f);
                const float tu = ev.u * dop, tw = ev.w * dop;
                const float wc = ae * Tk;
                // quad sums of (u, w, -u dx) dL/do, dL/do and the colour
                // partials; the four lanes of a quad share their row, hence dy,
                // so -u dy dL/do and -w dy dL/do follow from the sums
                constexpr int NQ = NV - 2;
                float q[NQ];
                q[0] = tu;
                q[1] = tw;
                q[2] = -tu * ev.dx;
                if constexpr (NV == 10) {
                    q[3] = dop;
                    q[4] = g[0] * wc;
                    q[5] = g[1] * wc;
                    q[6] = g[2] * wc;
                    q[7] = g[3] * wc;
                } else {
                    q[3] = g[3] * wc;
                }
                W = __builtin_fmaf(ae, sw, W);   // alpha S + (1 - alpha) W
                T = Tk;
                quad_sums<NQ>(q);
                float d[NV];
                d[0] = q[0];
                d[1] = q[1];
                d[2] = q[2];
                d[3] = -ev.dy * q[0];
                d[4] = -ev.dy * q[1];
#pragma unroll
                for (int c = 5; c < NV; ++c) d[c] = q[c - 2];
                if ((lane & 3u) == 0u) {
                    float2 *dst = reinterpret_cast<float2 *>(&s_q[wave][nb * kQStride + (lane >> 2) * NV]);
#pragma unroll
                    for (int c = 0; c < NV / 2; ++c) dst[c] = make_float2(d[2 * c], d[2 * c + 1]);
                }
                bpack |= (Pack)(pos - seg_lo) << (6u * nb);
                if (++nb == (uint32_t)kBatch) {
                    flush(nb, bpack);
                    nb = 0;
                    bpack = 0;
                }
            };
            while (mm != 0) {   // wave-uniform
                const int src = 63 - __builtin_clzll(mm);
                mm &= ~(1ull << src);
                entry(src);
            }
            if (nb != 0) flush(nb, bpack);
        }
        __syncthreads();
        // add the waves' sums in a fixed order and write each entry's row
        const uint32_t n_e = seg_hi - seg_lo;
        for (uint32_t idx = threadIdx.x; idx < n_e * NV; idx += blockDim.x) {
            const uint32_t e = idx / NV, c = idx - e * NV;
            float sum = 0.0f;
            for (int w = 0; w < nw; ++w) sum += s_acc[w][idx];
            const uint32_t j = s_j[e];
            if constexpr (ATOMIC) {
                if (j != ~0u && sum != 0.0f) atomicAdd(&grad_pairs[kRowStride * (size_t)j + c], sum);
            } else {
                if (j != ~0u) grad_pairs[NV * (size_t)j + c] = sum;
            }
        }
        __syncthreads();
        seg_hi = seg_lo;
    }
    if (COUNT) {
        const uint32_t e = wave_sum_u32(n_eval), c = wave_sum_u32(n_contrib);
        if (lane == 0) {
            atomicAdd((unsigned long long *)&counters[kCntEvalBwd], (unsigned long long)e);
            atomicAdd((unsigned long long *)&counters[kCntContribBwd], (unsigned long long)c);
            atomicAdd((unsigned long long *)&counters[kCntReduceBwd], (unsigned long long)n_red);
        }
    }
}

// Per-view loss: the view's tile partials added in a fixed order (one
// 256-thread block per view); also copied to hist if that is set.  The block
// that finishes last (a ticket taken with acquire-release ordering at device
// scope, so it sees every other block's view loss) adds the V view losses in
// view order into loss[V], the total.
__device__ __forceinline__ void loss_final_view(const ViewTable *__restrict__ vt, const double *__restrict__ loss_tile,
                                                double *__restrict__ loss, double *__restrict__ hist,
                                                int64_t *__restrict__ ticket, int view) {
    __shared__ double s[4];
    const ViewInfo &V = vt->v[view];
    const int n = V.tiles_x * V.tiles_y;
    double t = 0.0;
#pragma unroll 8   // loads in flight together; the additions keep their order
    for (int k = threadIdx.x; k < n; k += 256) t += loss_tile[V.tile_off + k];
    t = wave_sum_f64(t);   // each wave's butterfly, then the four waves in order
    if ((threadIdx.x & 63u) == 0u) s[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double lv = ((s[0] + s[1]) + s[2]) + s[3];
        loss[view] = lv;
        if (hist) hist[view] = lv;   // a tracking loop's per-iteration record
        const int nv = vt->n_views;
        if (nv == 1) {   // the only view: its loss is the total, no other block to wait for
            loss[1] = lv;
            return;
        }
        const int64_t k = __hip_atomic_fetch_add(ticket, (int64_t)1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (k == (int64_t)nv - 1) {
            double tot = 0.0;
            for (int v = 0; v < nv; ++v) tot += v == view ? lv : __hip_atomic_load(&loss[v], __ATOMIC_RELAXED,
                                                                                    __HIP_MEMORY_SCOPE_AGENT);
            loss[nv] = tot;
        }
    }
}

}  // namespace gsr
