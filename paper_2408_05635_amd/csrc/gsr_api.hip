// C ABI of the rasteriser (include/gsr.h): workspace layout, launch sequence
// and the per-Gaussian kernels (projection, binning, chain rule to the
// parameters and the pose).  The per-pixel kernels are in gsr_blend.hpp, the
// scan and radix sort in gsr_scan_sort.hpp.
//
// Launch sequence of one call (all views at once, no host synchronisation):
//   setup+project view table, FP64 poses, cleared counters; per Gaussian, per
//                 view: visibility, depth key, tiles touched
//   depth sort    stable radix sort of the visible records on the float32
//                 depth bits; its first pass also compacts them
//   gather        per visible record in depth order: full projection -> record
//   offsets       scan of tiles touched; emit -> (global tile id, record) pairs
//   tile sort     stable radix sort on the tile id: per-tile lists in depth
//                 order; its last pass also records every tile's [start, end)
//   work order    tiles heaviest first; with few tiles, long lists in chunks
//   blend_fwd     compositing (eqs. 2-4)
//   blend_bwd     loss + reverse compositing -> per-pair 2D gradient rows
//   record_bwd    chain rule to the raw parameters; pose partials per block
//   finalize      per view (q, t) and decoupled (q | C fixed, C) pose gradients
//                 and the loss; per Gaussian the sum over views
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gsr_blend.hpp"
#include "gsr_common.hpp"
#include "gsr_project.hpp"
#include "gsr_scan_sort.hpp"
#include "gsr_optim.hpp"

using namespace gsr;

// Per-stage HIP event timing (gsr_set_timing / gsr_read_timing).
enum Stage { kStageBinning = 0, kStageBlendFwd = 1, kStageBlendBwd = 2, kStageProjectBwd = 3, kNumStages = 4 };

struct gsr_ctx {
    int device;
    int num_cus;
    std::string err;
    void *scratch = nullptr;                           // this device's static scratch (device address)
    bool timing = false;
    bool capturing = false;                            // no event timing inside a graph capture
    bool no_alloc = false;                             // a call that must not create events either
    std::map<std::string, std::pair<int, int>> tuned;  // autotuned tile per input shape
    std::map<int32_t, hipGraphExec_t> graphs;          // captured call sequences
    int32_t next_graph = 1;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t take_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

// Brackets the launches of one stage with events when timing is on.
struct StageTimer {
    gsr_ctx *ctx;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(gsr_ctx *c, int s, hipStream_t stream) : ctx(c), stage(s), st(stream) {
        if (ctx->timing && !ctx->capturing && !ctx->no_alloc && ctx->recs.size() < 65536) {
            a = ctx->take_event();
            b = ctx->take_event();
            if (a && b) (void)hipEventRecord(a, st);
        }
    }
    ~StageTimer() {
        if (a && b) {
            (void)hipEventRecord(b, st);
            ctx->recs.push_back({stage, a, b});
        }
    }
};

static std::string g_create_err;

// The workspace of gsr_render_loss_grad_noalloc, for callers that cannot
// allocate: one array per device, held by the loaded module until the
// process ends.  Its name is not a device address in host code; the device
// address of each device's copy is looked up once (gsr_create, with that
// device current) and kept in g_scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices] = {};

namespace {

constexpr size_t kAlign = 256;
constexpr int kRecGrad = 14;   // per-record parameter gradient: mu 3, q 4, log_s 3, logit 1, rgb 3
constexpr size_t kCpBudgetBytes = 96u << 20;   // checkpoints of split lists (the longest lists get them first)
constexpr int64_t kSplitMaxTiles = 2048;       // about the backward workgroups resident at once
constexpr int kRecBwdMaxBlocks = 1024;   // grid cap of the record backward (one pose row per block)
constexpr int64_t kRecBwdItemsPerBlock = 1024;   // (view, Gaussian) items per record-backward block below the cap
constexpr int kEmitChunk = 4096;         // pairs per emission block
constexpr int kTuneCandidates = 7;       // tile shapes the autotuner tries
// synchronisation region, cleared by every call: block tickets (256 B), the
// single-pass scans' look-back words, the one-launch sort passes' look-back
// words and their digit histograms
constexpr size_t kSyncTickets = 256;
// ids of the binning's scans and sort passes (tickets and look-back tags)
enum SyncId : uint32_t { kIdOffsets = 1, kIdCompact = 2, kIdSweepDepth = 8, kIdSweepTile = 12 };
constexpr int kDepthPasses = 4, kMaxTilePasses = 3;
// tile-local binning: at most this many tiles, and a pair capacity of at most
// this many pairs per tile
constexpr int64_t kTileLocalMaxTiles = 16384;   // a block's tile counts fit LDS (64 KB)
constexpr int64_t kTileLocalMaxAvg = 4096;
constexpr int64_t kTileSortGrid = 2048;          // workgroups of the per-tile sort (8 per CU), looping over the lists

struct Layout {
    int64_t vn;           // V * N
    int64_t kcap;         // pair capacity
    int64_t P;            // total pixels
    int64_t T;            // total tiles
    int32_t G;            // total blend blocks
    int tile_bits;        // key bits of the tile sort
    size_t views, poses, counters, cnt, zkey, dk0, dv0, dk1, dv1, inv, rec, trect, cnt_s, poff, pk0, pv0, pk1, pv1,
        chunk, ranges, torder, cpoff, work, nwork, cp, tfinal, nlast, phash, cmask, gpairs, rrows, rgrad, losst, poseblk, scounts,
        stotals, sync;
    int64_t cp_slots;     // checkpoint slots of split lists (each: the tile's pixels x 6 floats)
    int64_t work_cap;     // backward work items at most: one per tile plus one per slot
    int64_t sort_nb;      // blocks of the larger three-launch sort (row length of scounts)
    bool depth_sweep, tile_sweep;   // sorts done with one launch per pass
    // tile-local binning (short lists): records in index order, pairs placed
    // per tile and each list sorted on its own; else the two global sorts
    bool tile_local;
    int64_t tv_max;       // tiles of the largest view (row length of the per-block tile counts)
    size_t tcnt, ttot, tstart, espan, pkv;
    // offsets in the sync region (cleared by every call): scan look-back words,
    // sort-pass look-back words, digit histograms (depth passes, then tile
    // passes), every view's first record (tile-local binning)
    size_t sync_status, sync_sweep, sync_hist, sync_vstart, sync_bytes;
    size_t total;
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int bits_for(int64_t n) {   // bits to hold ids 0..n-1
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

gsr_status fail(gsr_ctx *ctx, gsr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_create_err = buf;
    return st;
}

gsr_status check_hip(gsr_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return GSR_OK;
    return fail(ctx, GSR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Key of an input shape for the autotuner: views' resolutions, the size class
// of N (power of two) and the flags that change the work.
std::string shape_key(int64_t n, const gsr_views *views, uint32_t flags) {
    std::string k = std::to_string(views->n_views) + ":";
    for (int v = 0; v < views->n_views; ++v)
        k += std::to_string(views->cams[v].width) + "x" + std::to_string(views->cams[v].height) + ",";
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    k += "n2^" + std::to_string(b) + ":f" + std::to_string(flags & (GSR_ISOTROPIC | GSR_NO_GAUSS_GRADS | GSR_NO_POSE_GRADS));
    return k;
}

// opts with a zero tile replaced by the autotuned one (or 16x16).
gsr_options resolve_tile(const gsr_ctx *ctx, int64_t n, const gsr_views *views, const gsr_options *opts) {
    gsr_options o = *opts;
    if (o.tile_w == 0 && o.tile_h == 0 && views && views->cams && views->n_views >= 1 &&
        views->n_views <= GSR_MAX_VIEWS) {
        o.tile_w = o.tile_h = 16;
        if (ctx) {
            auto it = ctx->tuned.find(shape_key(n, views, opts->flags));
            if (it != ctx->tuned.end()) {
                o.tile_w = it->second.first;
                o.tile_h = it->second.second;
            }
        }
    }
    return o;
}

bool tile_side_ok(int s) { return s == 8 || s == 16 || s == 32; }

gsr_status validate_views(gsr_ctx *ctx, const gsr_views *views, const gsr_options *opts) {
    if (!views || !opts) return fail(ctx, GSR_EINVAL, "views and opts must not be NULL");
    if (views->n_views < 1) return fail(ctx, GSR_EINVAL, "n_views must be >= 1 (got %d)", views->n_views);
    if (views->n_views > GSR_MAX_VIEWS)
        return fail(ctx, GSR_EUNSUPPORTED, "at most %d views per call (got %d)", GSR_MAX_VIEWS, views->n_views);
    if (!views->cams) return fail(ctx, GSR_EINVAL, "views->cams must not be NULL");
    for (int v = 0; v < views->n_views; ++v) {
        const gsr_camera &c = views->cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
            return fail(ctx, GSR_EINVAL, "view %d: image size %dx%d out of range [1, 16384]", v, c.width, c.height);
        if (!std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy) ||
            c.fx <= 0.f || c.fy <= 0.f)
            return fail(ctx, GSR_EINVAL, "view %d: focal lengths must be finite and > 0", v);
    }
    const int tw = opts->tile_w, th = opts->tile_h;
    if (!tile_side_ok(tw) || !tile_side_ok(th))
        return fail(ctx, GSR_EINVAL, "tile size %dx%d: each side must be 8, 16 or 32", tw, th);
    if (!(opts->blur2d >= 0.f) || !std::isfinite(opts->blur2d))
        return fail(ctx, GSR_EINVAL, "blur2d must be finite and >= 0");
    if (!(opts->z_near >= 0.f) || !std::isfinite(opts->z_near))
        return fail(ctx, GSR_EINVAL, "z_near must be finite and >= 0");
    if (opts->blur2d == 0.f && opts->z_near == 0.f) {
        // allowed: degenerate covariances are culled
    }
    return GSR_OK;
}

void build_table(const gsr_views *views, const gsr_options *opts, ViewTable &vt) {
    memset(&vt, 0, sizeof(vt));
    vt.n_views = views->n_views;
    vt.tile_w = opts->tile_w;
    vt.tile_h = opts->tile_h;
    vt.pose_centre = (opts->flags & GSR_POSE_CENTRE) ? 1 : 0;
    vt.deterministic = (opts->flags & GSR_DETERMINISTIC) ? 1 : 0;
    int64_t pix = 0;
    int32_t tiles = 0, blocks = 0;
    const int spt = (opts->tile_w / kBlk) * (opts->tile_h / kBlk);
    for (int v = 0; v < views->n_views; ++v) {
        const gsr_camera &c = views->cams[v];
        ViewInfo &vi = vt.v[v];
        vi.W = c.width;
        vi.H = c.height;
        vi.fx = c.fx;
        vi.fy = c.fy;
        vi.cx = c.cx;
        vi.cy = c.cy;
        vi.pix_off = pix;
        vi.tiles_x = (c.width + opts->tile_w - 1) / opts->tile_w;
        vi.tiles_y = (c.height + opts->tile_h - 1) / opts->tile_h;
        vi.tile_off = tiles;
        vi.blk_off = blocks;
        pix += (int64_t)c.width * c.height;
        tiles += vi.tiles_x * vi.tiles_y;
        blocks += vi.tiles_x * vi.tiles_y * spt;
    }
    vt.total_tiles = tiles;
    vt.total_blocks = blocks;
}

Layout make_layout(int64_t n, const ViewTable &vt, int64_t kcap) {
    Layout L;
    const int V = vt.n_views;
    L.vn = (int64_t)V * n;
    L.kcap = kcap;
    L.P = 0;
    for (int v = 0; v < V; ++v) L.P += (int64_t)vt.v[v].W * vt.v[v].H;
    L.T = vt.total_tiles;
    L.G = vt.total_blocks;
    L.tile_bits = std::max(bits_for(L.T), 1);   // at least one pass: its scatter records the tile ranges
    // lists short enough on average for the per-tile sort, and few enough
    // tiles for a block's counts in LDS
    L.tile_local = L.T <= kTileLocalMaxTiles && kcap <= kTileLocalMaxAvg * L.T;
    L.tv_max = 1;
    for (int v = 0; v < V; ++v) L.tv_max = std::max<int64_t>(L.tv_max, (int64_t)vt.v[v].tiles_x * vt.v[v].tiles_y);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes ? bytes : 1);
        return o;
    };
    const size_t vn = (size_t)L.vn, kc = (size_t)kcap;
    L.counters = take(sizeof(int64_t) * kNumCounters);   // first: gsr_read_counters finds it at offset 0
    L.views = take(sizeof(ViewTable));
    L.poses = take(sizeof(PoseF64) * V);
    L.cnt = take(4 * vn);
    L.zkey = take(4 * vn);
    L.dk0 = take(4 * vn);
    L.dv0 = take(4 * vn);
    L.dk1 = take(4 * vn);
    L.dv1 = take(4 * vn);
    L.inv = take(4 * vn);
    L.rec = take(48 * vn);
    L.trect = take(8 * vn);
    L.cnt_s = take(4 * vn);
    L.poff = take(4 * vn);
    L.pk0 = take(4 * kc);
    L.pv0 = take(4 * kc);
    L.pk1 = take(4 * kc);
    L.pv1 = take(4 * kc);
    L.chunk = take(4 * (size_t)((kc + kEmitChunk - 1) / kEmitChunk + 1));
    L.ranges = take(8 * (size_t)L.T);
    // one row per (emission block, view it touches): row b + v (see k_emit_count)
    L.tcnt = take(L.tile_local ? 4 * (size_t)((kc + kEmitChunk - 1) / kEmitChunk + V) * (size_t)L.tv_max : 0);
    L.ttot = take(L.tile_local ? 4 * (size_t)L.T : 0);
    L.espan = take(L.tile_local ? 8 * (size_t)((kc + kEmitChunk - 1) / kEmitChunk) : 0);   // views of each block
    L.pkv = take(L.tile_local ? 8 * kc : 0);   // each placed pair's (depth key, record)
    L.tstart = take(L.tile_local ? 4 * (size_t)L.T : 0);
    L.torder = take(4 * (size_t)L.T);
    L.cpoff = take(4 * (size_t)L.T);
    {   // a split list needs chunks_of(len) - 1 slots; at most kcap / kChunkEntries in all, within a budget
        const size_t slot_bytes = (size_t)(vt.tile_w / kBlk) * (vt.tile_h / kBlk) * kCpValues * 64 * 4;
        // only when the tiles leave resident workgroups idle: with more, the
        // heaviest-first order already balances the backward
        L.cp_slots = L.T <= kSplitMaxTiles
                         ? std::min<int64_t>(std::min<int64_t>(kcap / kChunkEntries + 1, L.T),
                                             (int64_t)(kCpBudgetBytes / slot_bytes))
                         : 0;
        L.work_cap = L.T + L.cp_slots;
        L.work = take(4 * (size_t)L.work_cap);
        L.nwork = take(8);
        L.cp = take(slot_bytes * (size_t)L.cp_slots);
    }
    L.tfinal = take(4 * (size_t)L.P);
    L.nlast = take(4 * (size_t)L.P);
    L.phash = take(4 * (size_t)L.P);
    // the forward's culling ballots for the backward: K / 64 + T + 2 words per block of a tile
    L.cmask = take(8 * (size_t)((vt.tile_w / kBlk) * (vt.tile_h / kBlk)) * ((size_t)(kc / 64) + (size_t)L.T + 2));
    // the backward's 2D gradient rows: one per (tile, entry) pair with
    // GSR_DETERMINISTIC, else one per record (kRowStride floats each)
    L.gpairs = take(vt.deterministic ? 4 * kRowStride * kc : 0);
    L.rrows = take(vt.deterministic ? 0 : 4 * kRowStride * vn);
    L.rgrad = take(4 * kRecGrad * vn);
    L.losst = take(sizeof(double) * (size_t)L.T);
    L.poseblk = take(sizeof(double) * 12 * V * (size_t)std::max<int64_t>(
                                           std::min<int64_t>((L.vn + kRecBwdItemsPerBlock - 1) / kRecBwdItemsPerBlock, kRecBwdMaxBlocks), 1));
    // blocks of the record scan (256 records each) bound those of the compaction
    const int64_t nb_scan = std::max<int64_t>((L.vn + 255) / 256, 1);
    L.depth_sweep = sweep_fits(L.vn);
    L.tile_sweep = sweep_fits(kcap);
    L.sort_nb = std::max<int64_t>(std::max(L.depth_sweep ? 0 : sort_blocks(L.vn), L.tile_sweep ? 0 : sort_blocks(kcap)), 1);
    L.scounts = take(4 * 256 * (size_t)L.sort_nb);
    L.stotals = take(4 * 256);
    // the one-launch sort passes' look-back words (none with tile-local binning, which has no global sort)
    const int64_t nb_sweep = L.tile_local ? 0
                                          : std::max(L.depth_sweep ? sweep_blocks(L.vn) : 0,
                                                     L.tile_sweep ? sweep_blocks(kcap) : 0);
    L.sync_status = kSyncTickets;
    L.sync_sweep = align_up(L.sync_status + 8 * (size_t)nb_scan);
    L.sync_hist = align_up(L.sync_sweep + 4 * 256 * (size_t)nb_sweep);
    L.sync_vstart = align_up(L.sync_hist + 4 * 256 * (size_t)(kDepthPasses + kMaxTilePasses));
    L.sync_bytes = align_up(L.sync_vstart + 4 * (size_t)(V + 1));
    L.sync = take(L.sync_bytes);
    L.total = off;
    return L;
}

template <class T>
T *at(const gsr_workspace &ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws.ptr) + off);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

struct ProjParams {
    gsr_gaussians g;
    int64_t n;
    double z_near, blur;
    bool iso;
};

__device__ __forceinline__ uint32_t tiles_of(const Proj &r, const ViewTable *vt, const ViewInfo &V, uint32_t &tr0,
                                            uint32_t &tr1) {
    const int tx0 = r.px0 / vt->tile_w, tx1 = r.px1 / vt->tile_w;
    const int ty0 = r.py0 / vt->tile_h, ty1 = r.py1 / vt->tile_h;
    tr0 = (uint32_t)tx0 | ((uint32_t)tx1 << 16);
    tr1 = (uint32_t)ty0 | ((uint32_t)ty1 << 16);
    return (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
}

// The call's first kernel.  Set-up: the view table and the FP64 poses are
// written for the later kernels, the counters zeroed (block 0), the
// synchronisation region and every tile's range cleared (all blocks); each
// block also forms the poses in LDS for itself.  Then per Gaussian i, per view
// v: tiles touched (0 = not visible) and the depth key.
template <bool ISO>
__global__ __launch_bounds__(256) void k_setup_project(ViewTable tab, ViewTable *vt, const float *__restrict__ pq,
                                                       const float *__restrict__ pt, PoseF64 *poses,
                                                       int64_t *counters, uint4 *sync, int64_t sync16, uint2 *ranges,
                                                       int64_t n_tiles, bool keep_sticky, ProjParams pp,
                                                       uint32_t *__restrict__ cnt, uint32_t *__restrict__ zkey) {
    __shared__ PoseF64 s_pose[GSR_MAX_VIEWS];
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = gtid; k < sync16; k += gstride) sync[k] = make_uint4(0u, 0u, 0u, 0u);
    // every tile's range starts empty, (0xffffffff, 0); the tile sort's last
    // pass narrows those of the tiles with pairs
    for (int64_t k = gtid; k < n_tiles; k += gstride) ranges[k] = make_uint2(0xffffffffu, 0u);
    const int t = threadIdx.x;
    if (blockIdx.x == 0) {
        const int words = (int)(sizeof(ViewTable) / 4);
        const int32_t *src = reinterpret_cast<const int32_t *>(&tab);
        int32_t *dst = reinterpret_cast<int32_t *>(vt);
        for (int k = t; k < words; k += blockDim.x) dst[k] = src[k];
        if (t < kNumCounters && !(keep_sticky && t == kCntOverflowAny)) counters[t] = 0;
    }
    const int V = tab.n_views;
    if (t < V) {
        PoseF64 p;
        quat_to_rot_f64(pq[4 * t], pq[4 * t + 1], pq[4 * t + 2], pq[4 * t + 3], p.W);
        if (tab.pose_centre) {   // X_c = W (X - C) = W X + t with t = -W C
            const double C[3] = {(double)pt[3 * t], (double)pt[3 * t + 1], (double)pt[3 * t + 2]};
            for (int k = 0; k < 3; ++k) p.t[k] = -(p.W[3 * k] * C[0] + p.W[3 * k + 1] * C[1] + p.W[3 * k + 2] * C[2]);
        } else {
            for (int k = 0; k < 3; ++k) p.t[k] = (double)pt[3 * t + k];
        }
        s_pose[t] = p;
        if (blockIdx.x == 0) poses[t] = p;
    }
    __syncthreads();
    const int64_t i = gtid;
    if (i >= pp.n) return;
    const GaussIn p = load_gauss<ISO>(pp.g, i);
    GaussPre pre;   // once for all views
    prep_gauss<ISO>(p, pre);
    for (int v = 0; v < V; ++v) {
        Proj r;
        project_pre<false, ISO>(p, pre, s_pose[v], tab.v[v], pp.z_near, pp.blur, r);
        uint32_t c = 0;
        if (r.visible) {
            uint32_t a, b;
            c = tiles_of(r, &tab, tab.v[v], a, b);
        }
        cnt[(int64_t)v * pp.n + i] = c;
        zkey[(int64_t)v * pp.n + i] = __float_as_uint(r.z32);
    }
}

// Pair offsets of the records; also the first record of every kEmitChunk
// pairs (the record whose range holds pair m * kEmitChunk).
struct OffSink {
    uint32_t *off, *chunk_first;
    int64_t n_chunks;   // capacity of chunk_first
    __device__ void operator()(int64_t s, uint32_t pos, uint32_t cnt) const {
        off[s] = pos;
        if (cnt == 0) return;
        for (int64_t m = ((int64_t)pos + kEmitChunk - 1) / kEmitChunk;
             m * kEmitChunk < (int64_t)pos + cnt && m < n_chunks; ++m)
            chunk_first[m] = (uint32_t)s;
    }
};

// The pair total: the capacity check is made by the scan's last block.
struct PairTotal {
    int64_t *counters;
    int64_t cap;
    __device__ void operator()(int64_t K) const {
        counters[kCntPairs] = K;
        counters[kCntPairsUsed] = K <= cap ? K : 0;
        counters[kCntOverflow] = K <= cap ? 0 : 1;
        if (K > cap) counters[kCntOverflowAny] = 1;
    }
};

// Per visible record s (in depth order, or in (view, index) order with
// tile-local binning): full projection -> record, tile rect.  One record:
// written at s, its tile count returned (every thread of the record kernels
// below calls it for s < M).
template <bool ISO>
__device__ __forceinline__ uint32_t gather_record(const ProjParams &pp, const ViewTable *__restrict__ vt,
                                                  const PoseF64 *__restrict__ poses,
                                                  const uint32_t *__restrict__ sorted_gid, float4 *__restrict__ rec,
                                                  uint2 *__restrict__ trect, uint32_t *__restrict__ cnt_s,
                                                  uint32_t *__restrict__ inv, const float *__restrict__ rgb,
                                                  float *__restrict__ rrows, int64_t s) {
    const uint32_t gid = sorted_gid[s];
    int v = (int)(gid / (uint32_t)pp.n);
    if (v >= vt->n_views) v = 0;   // never expected; keeps reads in bounds
    const int64_t i = (int64_t)gid - (int64_t)v * pp.n;
    const GaussIn p = load_gauss<ISO>(pp.g, i);
    Proj r;
    project<true, ISO>(p, poses[v], vt->v[v], pp.z_near, pp.blur, r);
    uint32_t a = 0, b = 0;
    const uint32_t c = tiles_of(r, vt, vt->v[v], a, b);
    rec[3 * s] = make_float4(r.mxh, r.myh, r.mxl, r.myl);
    rec[3 * s + 1] = make_float4((float)r.l11, (float)r.l21, (float)r.l22, (float)r.o);
    rec[3 * s + 2] = make_float4(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], r.z32);
    trect[s] = make_uint2(a, b);
    cnt_s[s] = c;
    inv[gid] = (uint32_t)s;
    if (rrows) {   // the backward's atomics add into this record's row
        float2 *z = reinterpret_cast<float2 *>(rrows + kRowStride * (size_t)s);
#pragma unroll
        for (int k = 0; k < kRowStride / 2; ++k) z[k] = make_float2(0.0f, 0.0f);
    }
    return c;
}

template <bool ISO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_gather(ProjParams pp, const ViewTable *__restrict__ vt,
                                                const PoseF64 *__restrict__ poses, const int64_t *__restrict__ counters,
                                                const uint32_t *__restrict__ sorted_gid, float4 *__restrict__ rec,
                                                uint2 *__restrict__ trect, uint32_t *__restrict__ cnt_s,
                                                uint32_t *__restrict__ inv, const float *__restrict__ rgb,
                                                float *__restrict__ rrows) {
    // one record per thread (the grid covers every (view, Gaussian) item): no
    // loop, so that the registers fit more waves
    const int64_t M = counters[kCntVisible];
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < M) gather_record<ISO>(pp, vt, poses, sorted_gid, rec, trect, cnt_s, inv, rgb, rrows, s);
}

// The same, fused with the pair offsets: the exclusive scan of the records'
// tile counts, found in the same launch by decoupled look-back over blocks
// (blocks take tickets and block b holds records [256 b, 256 b + 256)); the
// block of the last record forms the pair total and checks it against the
// capacity.  Used where launches dominate (few records).
template <bool ISO>
__global__ __launch_bounds__(256) void k_gather_scan(ProjParams pp, const ViewTable *__restrict__ vt,
                                                     const PoseF64 *__restrict__ poses, int64_t *__restrict__ counters,
                                                     const uint32_t *__restrict__ sorted_gid, float4 *__restrict__ rec,
                                                     uint2 *__restrict__ trect, uint32_t *__restrict__ cnt_s,
                                                     uint32_t *__restrict__ inv, const float *__restrict__ rgb,
                                                     float *__restrict__ rrows, SyncState ss, uint32_t id,
                                                     OffSink sink, PairTotal fin) {
    __shared__ uint32_t s_b, s_excl;
    const uint32_t t = threadIdx.x;
    const int64_t M = counters[kCntVisible];
    const int64_t nb = (M + 255) / 256;
    // the grid is sized for V x N: the blocks past the records leave without a
    // ticket, so the tickets of the others are exactly [0, nb)
    if ((int64_t)blockIdx.x >= nb) {   // block-uniform
        if (nb == 0 && blockIdx.x == 0 && t == 0) fin(0);
        return;
    }
    if (t == 0) s_b = take_ticket(ss.tickets, id);
    __syncthreads();
    const int64_t b = s_b;
    const int64_t s = b * 256 + t;
    const uint32_t c =
        s < M ? gather_record<ISO>(pp, vt, poses, sorted_gid, rec, trect, cnt_s, inv, rgb, rrows, s) : 0u;
    uint32_t agg;
    const uint32_t run = block_excl_scan_u32<256>(c, agg);
    uint64_t *mine = ss.status + b;
    if (t == 0) publish(mine, id, b == 0 ? kFlagPrefix : kFlagAgg, agg);
    if (t < 64) {   // wave 0 looks back
        const uint32_t excl = b == 0 ? 0u : look_back_wave(ss.status, b, id, ss.error);
        if (t == 0) {
            if (b > 0) publish(mine, id, kFlagPrefix, excl + agg);
            s_excl = excl;
            if (b == nb - 1) fin((int64_t)excl + (int64_t)agg);
        }
    }
    __syncthreads();
    if (s < M) sink(s, s_excl + run, c);
}

struct CntSrc {
    const uint32_t *cnt;
    __device__ uint32_t operator()(int64_t i) const { return cnt[i]; }
};

// Pair j: key = global tile id, value = its record.  Records own contiguous
// ranges [poff[s], poff[s] + cnt_s[s]) in record order (every visible record
// touches at least one tile), so pair j's record is the last s with
// poff[s] <= j.  Chunk m holds pairs [m C, m C + C) (C = kEmitChunk): their
// records lie between the chunk's first record and the next chunk's, at most
// C + 1 of them; a block stages their offsets in LDS and each pair searches
// there.  j itself is recovered later from (record, tile).
constexpr int kEmitThreads = 1024;

struct EmitWindow {
    int64_t s0;   // first record of the chunk
    int nwin;     // records staged
};

// Stages chunk m's record offsets in s_off (the whole block calls it; the
// caller synchronises before the searches).
__device__ __forceinline__ EmitWindow emit_stage(int64_t m, int64_t K, int64_t M, const uint32_t *__restrict__ poff,
                                                 const uint32_t *__restrict__ chunk_first, uint32_t *s_off) {
    EmitWindow w;
    w.s0 = chunk_first[m];
    const int64_t s1 = (m + 1) * kEmitChunk < K ? (int64_t)chunk_first[m + 1] + 1 : M;   // window end
    w.nwin = (int)(s1 - w.s0 < kEmitChunk + 1 ? s1 - w.s0 : kEmitChunk + 1);
    for (int k = threadIdx.x; k < w.nwin; k += blockDim.x) s_off[k] = poff[w.s0 + k];
    return w;
}

// Pair j of the staged chunk -> its tile key, and its record in rec_s.
__device__ __forceinline__ uint32_t emit_pair(int64_t j, const EmitWindow &w, const uint32_t *s_off,
                                              const uint2 *__restrict__ trect, const uint32_t *__restrict__ gid,
                                              const ViewTable *__restrict__ vt, int64_t n, uint32_t &rec_s) {
    int lo = 0, hi = w.nwin;   // s_off[0] <= j; find the last entry <= j
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)s_off[mid] <= j)
            lo = mid;
        else
            hi = mid;
    }
    rec_s = (uint32_t)(w.s0 + lo);
    const uint32_t k = (uint32_t)j - s_off[lo];
    const uint2 tr = trect[rec_s];
    const uint32_t tx0 = tr.x & 0xffffu, nx = (tr.x >> 16) - tx0 + 1u, ty0 = tr.y & 0xffffu;
    int v = (int)(gid[rec_s] / (uint32_t)n);
    if (v >= vt->n_views) v = 0;
    const ViewInfo &V = vt->v[v];
    const uint32_t ty = ty0 + k / nx, tx = tx0 + k % nx;
    return (uint32_t)V.tile_off + ty * (uint32_t)V.tiles_x + tx;
}

// f(j, tile key, record, z) for the consecutive pairs j in [ja, jb) of the
// staged chunk: one search for the first pair, then the record's tiles in
// row-major order, moving to the next record after its last tile.  With
// zrec, z = zrec[record] (read with the record's rectangle), else 0.
template <class F>
__device__ __forceinline__ void emit_run(int64_t ja, int64_t jb, const EmitWindow &w, const uint32_t *s_off,
                                         const uint2 *__restrict__ trect, const uint32_t *__restrict__ gid,
                                         const ViewTable *__restrict__ vt, int64_t n, F f,
                                         const uint32_t *__restrict__ zrec = nullptr) {
    if (ja >= jb) return;
    int lo = 0, hi = w.nwin;   // s_off[0] <= ja; find the last entry <= ja
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)s_off[mid] <= ja)
            lo = mid;
        else
            hi = mid;
    }
    uint32_t rec = (uint32_t)(w.s0 + lo), k = (uint32_t)ja - s_off[lo];
    uint32_t tx0, tx1, tx, ty, np, base, tiles_x, z = 0;
    auto load_rec = [&]() {
        const uint2 tr = trect[rec];
        if (zrec) z = zrec[rec];
        tx0 = tr.x & 0xffffu;
        tx1 = tr.x >> 16;
        const uint32_t ty0 = tr.y & 0xffffu, nx = tx1 - tx0 + 1u;
        np = nx * ((tr.y >> 16) - ty0 + 1u);
        int v = (int)(gid[rec] / (uint32_t)n);
        if (v >= vt->n_views) v = 0;
        base = (uint32_t)vt->v[v].tile_off;
        tiles_x = (uint32_t)vt->v[v].tiles_x;
        ty = ty0 + k / nx;
        tx = tx0 + k % nx;
    };
    load_rec();
    for (int64_t j = ja; j < jb; ++j) {
        f(j, base + ty * tiles_x + tx, rec, z);
        if (j + 1 < jb) {
            if (++k == np) {   // the record's last pair: the next record starts at its first tile
                ++rec;
                k = 0;
                load_rec();
            } else if (++tx > tx1) {
                tx = tx0;
                ++ty;
            }
        }
    }
}

// One block per chunk: keys[j] = tile, vals[j] = record.  With hist (the
// one-launch tile sort), the histograms of the key bits [0, key_bits) in
// 8-bit digits are also added into hist[pass][256] (zero beforehand).
__global__ __launch_bounds__(kEmitThreads) void k_emit(const int64_t *__restrict__ counters, const uint32_t *__restrict__ poff,
                                              const uint32_t *__restrict__ chunk_first,
                                              const uint2 *__restrict__ trect, const uint32_t *__restrict__ gid,
                                              const ViewTable *__restrict__ vt, int64_t n,
                                              uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                              uint32_t *__restrict__ hist, int key_bits) {
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_hist[3 * 256];
    const int64_t K = counters[kCntPairsUsed];
    const int64_t M = counters[kCntVisible];
    const int64_t j0 = (int64_t)blockIdx.x * kEmitChunk;
    if (j0 >= K) return;   // block-uniform
    const int passes = hist ? (key_bits + 7) / 8 : 0;
    for (int k = threadIdx.x; k < passes * 256; k += blockDim.x) s_hist[k] = 0u;
    const EmitWindow w = emit_stage(blockIdx.x, K, M, poff, chunk_first, s_off);
    __syncthreads();
    for (int q0 = 0; q0 < kEmitChunk; q0 += blockDim.x) {
        const int64_t j = j0 + q0 + (int)threadIdx.x;
        const bool live = j < K;
        uint32_t key = 0;
        if (live) {
            uint32_t rs;
            key = emit_pair(j, w, s_off, trect, gid, vt, n, rs);
            keys[j] = key;
            vals[j] = rs;
        }
        if (passes) add_digit_hist(key, live, key_bits, s_hist);
    }
    if (passes) {
        __syncthreads();
        flush_digit_hist(s_hist, passes, hist);
    }
}

// Tile-local binning, the emission in two passes over the same pairs, one
// block per chunk.  Records are in view order, so the pairs of block b belong
// to a run of views [v0, v1] (usually one); k_emit_count counts them per tile
// in LDS and stores, for each of those views v, the row counts[b + v][0, T_v)
// (b + v grows with (b, v) over the rows written, so rows never collide), and
// the block's [v0, v1] for the placing pass.
// k_tile_offsets turns every tile's column, over the blocks holding pairs of
// its view, into exclusive offsets (and the tile's total); k_tile_ranges turns
// the totals into list starts; k_emit_place gives each pair the next free
// place of its tile within its block's share, cursor = start + offset in LDS.
// No global atomics: a tile's pairs come from every part of its view's records.
struct ViewSpan {
    int v0, v1;
};

// the views of the first and last pair of the staged chunk (thread 0 finds
// them; the caller synchronises before s_span is read)
__device__ __forceinline__ void chunk_views(int64_t m, int64_t K, const EmitWindow &w, const uint32_t *s_off,
                                            const uint2 *__restrict__ trect, const uint32_t *__restrict__ gid,
                                            const ViewTable *__restrict__ vt, int64_t n, ViewSpan *s_span) {
    if (threadIdx.x != 0) return;
    const int64_t j0 = m * kEmitChunk, j1 = (j0 + kEmitChunk < K ? j0 + kEmitChunk : K) - 1;
    uint32_t r0, r1;
    (void)emit_pair(j0, w, s_off, trect, gid, vt, n, r0);
    (void)emit_pair(j1, w, s_off, trect, gid, vt, n, r1);
    int v0 = (int)(gid[r0] / (uint64_t)n), v1 = (int)(gid[r1] / (uint64_t)n);
    const int nv = vt->n_views;
    v0 = v0 < nv ? v0 : nv - 1;   // never expected; keeps rows in bounds
    v1 = v1 < nv ? (v1 > v0 ? v1 : v0) : nv - 1;
    s_span->v0 = v0;
    s_span->v1 = v1;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit_count(const int64_t *__restrict__ counters,
                                                             const uint32_t *__restrict__ poff,
                                                             const uint32_t *__restrict__ chunk_first,
                                                             const uint2 *__restrict__ trect,
                                                             const uint32_t *__restrict__ gid,
                                                             const ViewTable *__restrict__ vt, int64_t n,
                                                             int64_t n_tiles, int64_t row_len,
                                                             uint32_t *__restrict__ counts,
                                                             uint2 *__restrict__ espan) {
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_h[kTileLocalMaxTiles];
    __shared__ ViewSpan s_span;
    const int64_t K = counters[kCntPairsUsed], M = counters[kCntVisible];
    const int64_t m = blockIdx.x, j0 = m * kEmitChunk;
    if (j0 >= K) return;   // block-uniform: rows past the pairs are never read
    for (int64_t k = threadIdx.x; k < n_tiles; k += blockDim.x) s_h[k] = 0u;
    const EmitWindow w = emit_stage(m, K, M, poff, chunk_first, s_off);
    __syncthreads();
    chunk_views(m, K, w, s_off, trect, gid, vt, n, &s_span);
    {   // each thread kEmitChunk / kEmitThreads consecutive pairs
        constexpr int kRun = kEmitChunk / kEmitThreads;
        const int64_t ja = j0 + (int64_t)threadIdx.x * kRun, je = j0 + kEmitChunk < K ? j0 + kEmitChunk : K;
        emit_run(ja, ja + kRun < je ? ja + kRun : je, w, s_off, trect, gid, vt, n,
                 [&](int64_t, uint32_t key, uint32_t, uint32_t) {
                     if ((int64_t)key < n_tiles) atomicAdd(&s_h[key], 1u);   // always true; keeps accesses in bounds
                 });
    }
    __syncthreads();
    if (threadIdx.x == 0) espan[m] = make_uint2((uint32_t)s_span.v0, (uint32_t)s_span.v1);   // for the placing pass
    for (int v = s_span.v0; v <= s_span.v1; ++v) {
        const ViewInfo &V = vt->v[v];
        const int tv = V.tiles_x * V.tiles_y;
        uint32_t *row = counts + (size_t)(m + v) * (size_t)row_len;
        for (int k = threadIdx.x; k < tv; k += blockDim.x) row[k] = s_h[V.tile_off + k];
    }
}

// Four threads per tile (adjacent lanes), each taking a quarter of its column
// over the blocks that hold pairs of its view (those whose chunks meet the
// view's pair range [start(v), start(v + 1)): start(v) is the first pair of the
// view's first record vrec[v], K past the last record): each sums its rows,
// the four sums are scanned by lane shuffles, and each writes its rows'
// exclusive offsets from its share of that scan; the first writes the tile's
// total.  A quarter of up to kOffsetsBatch rows stays in registers between
// the two steps, a longer one is read again.
constexpr int kOffsetsBatch = 32;   // rows of a column read together
constexpr int kOffsetsParts = 4;

__global__ __launch_bounds__(256) void k_tile_offsets(const ViewTable *__restrict__ vt,
                                                      const int64_t *__restrict__ counters,
                                                      const uint32_t *__restrict__ vrec,
                                                      const uint32_t *__restrict__ poff, int64_t n_tiles,
                                                      int64_t row_len, uint32_t *__restrict__ counts,
                                                      uint32_t *__restrict__ ttot) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t t = g / kOffsetsParts;
    const int part = (int)(g % kOffsetsParts);
    // every lane goes on to the shuffles; lanes past the tiles take no rows
    int64_t r0 = 0, r1 = 0;
    uint32_t *col = counts;
    if (t < n_tiles) {
        const int64_t K = counters[kCntPairsUsed], M = counters[kCntVisible];
        const int nv = vt->n_views;
        int v = 0;
        while (v + 1 < nv && vt->v[v + 1].tile_off <= t) ++v;
        const int64_t x = t - vt->v[v].tile_off;
        const int64_t ps = (int64_t)vrec[v] < M ? (int64_t)poff[vrec[v]] : K;
        const int64_t pe = v + 1 < nv && (int64_t)vrec[v + 1] < M ? (int64_t)poff[vrec[v + 1]] : K;
        if (pe > ps && pe <= K) {
            const int64_t b0 = ps / kEmitChunk, b1 = (pe - 1) / kEmitChunk;
            col = counts + (size_t)(b0 + v) * (size_t)row_len + (size_t)x;
            const int64_t nb = b1 - b0 + 1, per = (nb + kOffsetsParts - 1) / kOffsetsParts;
            r0 = per * part < nb ? per * part : nb;
            r1 = r0 + per < nb ? r0 + per : nb;
        }
    }
    auto at_row = [&](int64_t r) -> uint32_t & { return col[(size_t)r * (size_t)row_len]; };
    const bool one = r1 - r0 <= kOffsetsBatch;
    uint32_t c[kOffsetsBatch];
    uint32_t sum = 0;
    if (one) {
#pragma unroll
        for (int q = 0; q < kOffsetsBatch; ++q) {
            c[q] = r0 + q < r1 ? at_row(r0 + q) : 0u;
            sum += c[q];
        }
    } else {
        for (int64_t b = r0; b < r1; b += kOffsetsBatch) {   // the batch's loads in flight together
#pragma unroll
            for (int q = 0; q < kOffsetsBatch; ++q) sum += b + q < r1 ? at_row(b + q) : 0u;
        }
    }
    // the tile's four sums: inclusive scan over its lanes, then the total from the last
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kOffsetsParts; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, kOffsetsParts);
        if (part >= d) incl += y;
    }
    const uint32_t total = __shfl(incl, kOffsetsParts - 1, kOffsetsParts);
    uint32_t run = incl - sum;
    if (one) {
#pragma unroll
        for (int q = 0; q < kOffsetsBatch; ++q) {
            if (r0 + q < r1) at_row(r0 + q) = run;
            run += c[q];
        }
    } else {
        for (int64_t b = r0; b < r1; b += kOffsetsBatch) {
            uint32_t cb[kOffsetsBatch];
#pragma unroll
            for (int q = 0; q < kOffsetsBatch; ++q) cb[q] = b + q < r1 ? at_row(b + q) : 0u;
#pragma unroll
            for (int q = 0; q < kOffsetsBatch; ++q) {
                if (b + q < r1) at_row(b + q) = run;
                run += cb[q];
            }
        }
    }
    if (t < n_tiles && part == 0) ttot[t] = total;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit_place(const int64_t *__restrict__ counters,
                                                             const uint32_t *__restrict__ poff,
                                                             const uint32_t *__restrict__ chunk_first,
                                                             const uint2 *__restrict__ trect,
                                                             const uint32_t *__restrict__ gid,
                                                             const ViewTable *__restrict__ vt, int64_t n,
                                                             int64_t n_tiles, int64_t row_len,
                                                             const uint32_t *__restrict__ offsets,
                                                             const uint32_t *__restrict__ tstart,
                                                             const uint2 *__restrict__ espan,
                                                             const uint32_t *__restrict__ zrec,
                                                             uint2 *__restrict__ kv) {
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_cur[kTileLocalMaxTiles];
    const int64_t K = counters[kCntPairsUsed], M = counters[kCntVisible];
    const int64_t m = blockIdx.x, j0 = m * kEmitChunk;
    if (j0 >= K) return;   // block-uniform
    // the block's views, as the counting pass found them: the cursors' rows
    // are read while the chunk's record offsets are staged
    const uint2 sp = espan[m];
    const int nv = vt->n_views;
    const int v0 = (int)sp.x < nv ? (int)sp.x : nv - 1;   // never expected; keeps rows in bounds
    const int v1 = (int)sp.y < nv ? (int)sp.y : nv - 1;
    const EmitWindow w = emit_stage(m, K, M, poff, chunk_first, s_off);
    for (int v = v0; v <= v1; ++v) {
        const ViewInfo &V = vt->v[v];
        const int tv = V.tiles_x * V.tiles_y;
        const uint32_t *row = offsets + (size_t)(m + v) * (size_t)row_len;
        for (int k = threadIdx.x; k < tv; k += blockDim.x) s_cur[V.tile_off + k] = tstart[V.tile_off + k] + row[k];
    }
    __syncthreads();   // the offsets and the cursors
    {
        constexpr int kRun = kEmitChunk / kEmitThreads;
        const int64_t ja = j0 + (int64_t)threadIdx.x * kRun, je = j0 + kEmitChunk < K ? j0 + kEmitChunk : K;
        emit_run(ja, ja + kRun < je ? ja + kRun : je, w, s_off, trect, gid, vt, n,
                 [&](int64_t, uint32_t key, uint32_t rs, uint32_t z) {
                     if ((int64_t)key < n_tiles) {   // always true; keeps accesses in bounds
                         const uint32_t slot = atomicAdd(&s_cur[key], 1u);
                         if ((int64_t)slot < K) kv[slot] = make_uint2(z, rs);   // always true; keeps writes in bounds
                     }
                 },
                 zrec);
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__global__ void k_fill_f64(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Heaviest work first.  (1) torder: a permutation of the tiles by decreasing
// list length (256 buckets of 16 entries, the longest first, any order within
// a bucket), the order in which the forward takes its tiles.  (2) In that
// order, each list longer than kSplitMin gets chunks_of(len) - 1 checkpoint
// slots (cpoff: its first slot, or kNoSplit) while they fit in slots_cap.
// (3) work: the backward's items (tile | chunk << 24), again longest first,
// and their number.  Only the order and the split of the work change, never a
// result; one block does it all.
constexpr int kOrderThreads = 1024;
constexpr uint32_t kOrderBuckets = 256;

// len_of(i): the list length of tile i.  s_ord: null, or an LDS array of
// n_tiles words, through which, without splits, the tile order and the work
// items are written coalesced rather than scattered (with splits the tiles
// are few and the order stays in s_to).
template <class Len>
__device__ __forceinline__ void work_order_block(Len len_of, int64_t n_tiles, int64_t slots_cap,
                                                 uint32_t *__restrict__ torder, uint32_t *__restrict__ cpoff,
                                                 uint32_t *__restrict__ work, int64_t *__restrict__ n_work,
                                                 int64_t *__restrict__ counters, uint32_t *s_ord = nullptr) {
    __shared__ uint32_t s_h[kOrderBuckets];
    // with chunk splits (at most kSplitMaxTiles tiles) the tile order and the
    // checkpoint slots are also kept here, so the later phases read no global
    // memory that this block wrote
    __shared__ uint32_t s_to_own[kSplitMaxTiles], s_cp[kSplitMaxTiles];
    uint32_t *s_to = s_to_own;
    const int t = threadIdx.x;
    const bool split_mode = slots_cap > 0 && n_tiles <= kSplitMaxTiles;   // the layout gives slots only then
    if (split_mode) s_ord = nullptr;
    auto bucket_of = [](uint32_t len) {
        const uint32_t b = len >> 4;
        return (kOrderBuckets - 1u) - (b < kOrderBuckets - 1u ? b : kOrderBuckets - 1u);
    };
    // turns the bucket counts into first positions; returns the total
    auto bucket_starts = [&]() {
        uint32_t all;
        const uint32_t first = block_excl_scan_u32<kOrderThreads>(t < (int)kOrderBuckets ? s_h[t] : 0u, all);
        if (t < (int)kOrderBuckets) s_h[t] = first;
        __syncthreads();
        return all;
    };
    // (1) tiles by decreasing length
    if (t < (int)kOrderBuckets) s_h[t] = 0u;
    __syncthreads();
    for (int64_t i = t; i < n_tiles; i += kOrderThreads) atomicAdd(&s_h[bucket_of(len_of(i))], 1u);
    __syncthreads();
    bucket_starts();
    for (int64_t i = t; i < n_tiles; i += kOrderThreads) {
        const uint32_t pos = atomicAdd(&s_h[bucket_of(len_of(i))], 1u);
        if ((int64_t)pos < n_tiles) {   // always true; keeps writes in bounds
            if (s_ord) {
                s_ord[pos] = (uint32_t)i;
            } else {
                torder[pos] = (uint32_t)i;
                if (split_mode)
                    s_to[pos] = (uint32_t)i;
                else
                    work[pos] = (uint32_t)i;   // no splits: the items are the tiles, in that order
            }
        }
        if (!split_mode) cpoff[i] = kNoSplit;
    }
    if (s_ord) {   // the order copied out in rank order; no splits: the items are the tiles, in that order
        __syncthreads();
        for (int64_t r = t; r < n_tiles; r += kOrderThreads) torder[r] = work[r] = s_ord[r];
    }
    if (!split_mode) {
        if (t == 0) *n_work = counters[kCntWorkItems] = n_tiles;
        return;
    }
    __syncthreads();
    // (2) checkpoint slots in that order: two consecutive places per thread, one block scan
    static_assert(kSplitMaxTiles <= 2 * kOrderThreads, "the split tiles take one scan");
    {
        uint32_t need[2] = {0u, 0u}, tile[2] = {0u, 0u};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t r = 2 * (int64_t)t + h;
            if (r < n_tiles) {
                tile[h] = s_to[r];
                const uint32_t len = len_of(tile[h]), nch = chunks_of(len);
                need[h] = (len > kSplitMin && nch <= kMaxChunks) ? nch - 1u : 0u;
            }
        }
        uint32_t tot;
        int64_t p = block_excl_scan_u32<kOrderThreads>(need[0] + need[1], tot);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (2 * (int64_t)t + h < n_tiles) {
                const uint32_t slot = (need[h] > 0u && p + (int64_t)need[h] <= slots_cap) ? (uint32_t)p : kNoSplit;
                cpoff[tile[h]] = slot;
                s_cp[tile[h]] = slot;
            }
            p += need[h];
        }
    }
    // (3) the backward's items, longest first.  The chunks of a split list
    // before its last are all full (kChunkEntries entries, one bucket), so
    // they take their places by wave prefix sums and one LDS add per wave;
    // each tile's last (or only) item takes its own.
    auto item_len = [&](uint32_t len, bool split, uint32_t m) {
        return split ? (len - m * kChunkEntries < kChunkEntries ? len - m * kChunkEntries : kChunkEntries) : len;
    };
    const uint32_t full_bucket = bucket_of(kChunkEntries);
    const uint32_t lane = (uint32_t)t & 63u;
    if (t < (int)kOrderBuckets) s_h[t] = 0u;
    __syncthreads();
    // a tile's items: split ? chunks_of(len) : 1, the last at m = n_items - 1
    auto tile_items = [&](int64_t i, uint32_t &len) -> uint32_t {
        len = len_of(i);
        return s_cp[i] != kNoSplit ? chunks_of(len) : 1u;
    };
    uint32_t n_full = 0;
    for (int64_t i = t; i < n_tiles; i += kOrderThreads) {
        uint32_t len;
        const uint32_t ni = tile_items(i, len);
        n_full += ni - 1u;
        atomicAdd(&s_h[bucket_of(item_len(len, s_cp[i] != kNoSplit, ni - 1u))], 1u);
    }
    n_full = wave_sum_u32(n_full);
    if (lane == 0u && n_full) atomicAdd(&s_h[full_bucket], n_full);
    __syncthreads();
    const uint32_t total = bucket_starts();
    if (t == 0) *n_work = counters[kCntWorkItems] = total;
    for (int64_t base = 0; base < n_tiles; base += kOrderThreads) {   // whole rounds: the wave sums need every lane
        const int64_t i = base + t;
        uint32_t len = 0, ni = 0;
        if (i < n_tiles) ni = tile_items(i, len);
        const uint32_t nf = ni > 0u ? ni - 1u : 0u;
        const uint32_t incl = wave_incl_scan_u32(nf);
        uint32_t wbase = 0;
        if (lane == 63u && incl) wbase = atomicAdd(&s_h[full_bucket], incl);
        wbase = __builtin_amdgcn_readlane(wbase, 63);
        for (uint32_t m = 0; m < nf; ++m) {
            const uint32_t pos = wbase + incl - nf + m;
            if (pos < total) work[pos] = (uint32_t)i | (m << 24);   // always true; keeps writes in bounds
        }
        if (ni > 0u) {
            const uint32_t m = ni - 1u;
            const uint32_t pos = atomicAdd(&s_h[bucket_of(item_len(len, s_cp[i] != kNoSplit, m))], 1u);
            if (pos < total) work[pos] = (uint32_t)i | (m << 24);   // always true; keeps writes in bounds
        }
    }
}

__global__ __launch_bounds__(kOrderThreads) void k_work_order(const uint2 *__restrict__ ranges, int64_t n_tiles,
                                                              int64_t slots_cap, uint32_t *__restrict__ torder,
                                                              uint32_t *__restrict__ cpoff, uint32_t *__restrict__ work,
                                                              int64_t *__restrict__ n_work,
                                                              int64_t *__restrict__ counters) {
    work_order_block(
        [&](int64_t i) {
            const uint2 r = ranges[i];
            return r.y > r.x ? r.y - r.x : 0u;
        },
        n_tiles, slots_cap, torder, cpoff, work, n_work, counters);
}

// Tile-local binning: every tile's list [start, end) from the tiles' pair
// totals (an exclusive scan in tile order), the starts for the placement, the
// number of lists that the per-tile sort gives a whole workgroup, then the
// work order.  One block.  The totals are read and the results written
// coalesced (tile r 1024 + thread in round r, all loads in flight), through
// LDS, where each thread scans 16 consecutive tiles; the starts stay there,
// one pad word after every 16 so that those 16 fall in different banks.
constexpr int kRangePer = (int)(kTileLocalMaxTiles / kOrderThreads);   // tiles per thread
__device__ __forceinline__ int32_t range_slot(int64_t i) { return (int32_t)(i + (i >> 4)); }

__global__ __launch_bounds__(kOrderThreads) void k_tile_ranges(const uint32_t *__restrict__ ttot, int64_t n_tiles,
                                                               uint2 *__restrict__ ranges, uint32_t *__restrict__ tstart,
                                                               int64_t slots_cap, uint32_t *__restrict__ torder,
                                                               uint32_t *__restrict__ cpoff, uint32_t *__restrict__ work,
                                                               int64_t *__restrict__ n_work,
                                                               int64_t *__restrict__ counters) {
    __shared__ uint32_t s_big;
    // tile i's start at range_slot(i) (tiles past n_tiles have none, so their
    // starts are the total), the total at range_slot(kTileLocalMaxTiles)
    __shared__ uint32_t s_st[kTileLocalMaxTiles + kTileLocalMaxTiles / 16 + 1];
    const int t = threadIdx.x;
    if (t == 0) s_big = 0u;
    uint32_t x[kRangePer];
#pragma unroll
    for (int r = 0; r < kRangePer; ++r) {
        const int64_t i = (int64_t)r * kOrderThreads + t;
        x[r] = i < n_tiles ? ttot[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRangePer; ++r) s_st[range_slot((int64_t)r * kOrderThreads + t)] = x[r];
    __syncthreads();
    const int64_t d0 = (int64_t)t * kRangePer;
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kRangePer; ++q) {
        x[q] = s_st[range_slot(d0 + q)];
        sum += x[q];
    }
    uint32_t tot;
    uint32_t start = block_excl_scan_u32<kOrderThreads>(sum, tot);   // its barriers order s_big's clear
#pragma unroll
    for (int q = 0; q < kRangePer; ++q) {   // a thread rewrites only its own tiles' slots
        s_st[range_slot(d0 + q)] = start;
        start += x[q];
    }
    if (t == 0) s_st[range_slot(kTileLocalMaxTiles)] = tot;
    __syncthreads();
    auto len_of = [&](int64_t i) { return s_st[range_slot(i + 1)] - s_st[range_slot(i)]; };
    uint32_t big = 0;
#pragma unroll
    for (int r = 0; r < kRangePer; ++r) {
        const int64_t i = (int64_t)r * kOrderThreads + t;
        if (i < n_tiles) {
            const uint32_t st = s_st[range_slot(i)], en = s_st[range_slot(i + 1)];
            ranges[i] = make_uint2(st, en);
            tstart[i] = st;
            big += en - st >= kTileSortWaveCap ? 1u : 0u;
        }
    }
    big = wave_sum_u32(big);
    if ((t & 63) == 0 && big) atomicAdd(&s_big, big);
    __syncthreads();
    if (t == 0) counters[kCntSortBig] = s_big;
    __shared__ uint32_t s_ord[kTileLocalMaxTiles];
    work_order_block(len_of, n_tiles, slots_cap, torder, cpoff, work, n_work, counters, s_ord);
}

struct GradOut {
    gsr_gaussian_grads gg;
    bool want_gauss, want_pose;
};

// Per visible record s (one view, one Gaussian): the record's 2D gradient is
// the sum of its pairs' rows (contiguous); the chain rule takes it to the raw
// parameters (written per record, 14 floats) and to the view's pose partials
// (G_W and g_t, 12 values), which are summed per view in FP64: in LDS over
// the block, then written as one row per block (no global atomics) for
// the pose finalisation to add in a fixed order.
//
// Load balance: records are depth-sorted, so the nearest ones, which can
// cover every tile of the image, are neighbours.  With a row per pair, lane l
// of wave slot w takes record l * W + w (W = number of wave slots needed),
// which spreads neighbours over different waves; the grid's waves walk the
// slots with a stride.  A record with more than kLongRows rows is summed by
// the whole wave (rows lane, lane + 64, ...; then a fixed-order reduction),
// so no lane walks a long range alone.  Both row sums are deterministic.
// With one row per record (ATOMIC) every record costs the same, and wave slot
// w takes records 64 w + l: coalesced reads, and the wave's records mostly of
// one view, whose pose partials it then sums before adding them.
constexpr uint32_t kLongRows = 32;

// ATOMIC: the record's 2D gradient is its own row of gpairs (kRowStride
// floats, summed there by the blend's atomics), which is read and cleared
// again, so that a second backward on the same forward state starts from zero.
template <bool ISO, int NV, bool ATOMIC>
__global__ __launch_bounds__(256) void k_record_bwd(ProjParams pp, const ViewTable *__restrict__ vt,
                                                    const PoseF64 *__restrict__ poses,
                                                    const uint32_t *__restrict__ gid_sorted,
                                                    const uint32_t *__restrict__ poff,
                                                    const uint32_t *__restrict__ cnt_s,
                                                    float *__restrict__ gpairs, const int64_t *__restrict__ counters,
                                                    float *__restrict__ rgrad, double *__restrict__ pose_blocks,
                                                    bool want_gauss, bool want_pose) {
    __shared__ double s_pose[GSR_MAX_VIEWS * 12];
    const int V = vt->n_views;
    if (want_pose) {
        for (int k = threadIdx.x; k < V * 12; k += blockDim.x) s_pose[k] = 0.0;
        __syncthreads();
    }
    const int64_t M = counters[kCntVisible];
    const bool have_pairs = counters[kCntPairsUsed] > 0;
    const int64_t W = (M + 63) / 64;
    const uint32_t lane = threadIdx.x & 63u;
    const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < W; w += wstride) {   // wave-uniform
        const int64_t s = ATOMIC ? 64 * w + (int64_t)lane : (int64_t)lane * W + w;
        const bool valid = s < M;
        uint32_t j0 = 0, nrow = 0;
        if (valid && have_pairs) {
            j0 = poff[s];
            nrow = cnt_s[s];
        }
        float r2[NV];   // the record's row sum (NV partials; 6 = pose only: 0..4 and depth)
#pragma unroll
        for (int c = 0; c < NV; ++c) r2[c] = 0.0f;
        if constexpr (ATOMIC) {
            if (valid && have_pairs) {
                float *row = gpairs + kRowStride * (size_t)s;
#pragma unroll
                for (int c = 0; c < NV; ++c) r2[c] = row[c];
#pragma unroll
                for (int c = 0; c < NV; ++c) row[c] = 0.0f;
            }
        } else if (nrow <= kLongRows) {   // rows in order; four rows' loads in flight at once
            uint32_t jj = j0;
            const uint32_t end = j0 + nrow;
            for (; jj + 4 <= end; jj += 4) {
                float rows[4 * NV];
                const float *row = gpairs + NV * (size_t)jj;
#pragma unroll
                for (int c = 0; c < 4 * NV; ++c) rows[c] = row[c];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < NV; ++c) r2[c] += rows[NV * q + c];
            }
            for (; jj < end; ++jj) {
                const float *row = gpairs + NV * (size_t)jj;
#pragma unroll
                for (int c = 0; c < NV; ++c) r2[c] += row[c];
            }
        }
        uint64_t longm = ATOMIC ? 0ull : ballot(nrow > kLongRows);
        while (longm) {   // wave-uniform loop over this wave's long records
            const int src = __builtin_ctzll(longm);
            longm &= longm - 1;
            const uint32_t a = __shfl(j0, src, 64), cnt = __shfl(nrow, src, 64);
            float part[NV];
#pragma unroll
            for (int c = 0; c < NV; ++c) part[c] = 0.0f;
            for (uint32_t jj = a + lane; jj < a + cnt; jj += 64) {
                const float *row = gpairs + NV * (size_t)jj;
#pragma unroll
                for (int c = 0; c < NV; ++c) part[c] += row[c];
            }
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const float t = wave_sum(part[c]);
                if ((int)lane == src) r2[c] = t;
            }
        }
        // every lane goes on to the pose sums below (lanes without a record
        // with zero partials)
        double gX[3] = {0.0, 0.0, 0.0}, GW[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int v = -1;
        if (valid) {
            const uint32_t gid = gid_sorted[s];
            v = (int)(gid / (uint64_t)pp.n);
            if (v >= V) v = -1;   // never expected; keeps reads in bounds
        }
        if (v >= 0) {
            const int64_t i = (int64_t)gid_sorted[s] - (int64_t)v * pp.n;
            const GaussIn p = load_gauss<ISO>(pp.g, i);
            Proj r;
            project<true, ISO>(p, poses[v], vt->v[v], pp.z_near, pp.blur, r);
            // the rows carry the conic-factor and mean partials without their
            // per-record factors k = 2 o ln2 and (l11, l21, l22)
            const double k2 = 2.0 * kLn2 * r.o;
            float g2[10];
            g2[0] = (float)(k2 * r.l11 * (double)r2[0]);
            g2[1] = (float)(k2 * (r.l21 * (double)r2[0] + r.l22 * (double)r2[1]));
#pragma unroll
            for (int c = 2; c < 5; ++c) g2[c] = (float)(k2 * (double)r2[c]);
            if constexpr (NV == 10) {
#pragma unroll
                for (int c = 5; c < 10; ++c) g2[c] = r2[c];
            } else {
                g2[5] = g2[6] = g2[7] = g2[8] = 0.0f;
                g2[9] = r2[5];
            }
            ParamGrad pg;
            for (int k = 0; k < 3; ++k) pg.mu[k] = pg.ls[k] = pg.rgb[k] = 0.0;
            for (int k = 0; k < 4; ++k) pg.q[k] = 0.0;
            pg.logit = 0.0;
            project_backward<ISO, NV == 10>(p, poses[v], vt->v[v], r, g2, pg, gX, GW);
            if (want_gauss) {
                float *o = rgrad + kRecGrad * (size_t)s;
                for (int k = 0; k < 3; ++k) o[k] = (float)pg.mu[k];
                for (int k = 0; k < 4; ++k) o[3 + k] = (float)pg.q[k];
                for (int k = 0; k < 3; ++k) o[7 + k] = (float)pg.ls[k];
                o[10] = (float)pg.logit;
                for (int k = 0; k < 3; ++k) o[11 + k] = (float)pg.rgb[k];
            }
        }
        if (want_pose) {
            // A wave whose records all belong to one view (always so for a
            // single view) sums its partials first, by butterflies, and adds
            // them once: the LDS adds of 64 lanes to the same 12 words would
            // be serialised.  Otherwise each lane adds its own.
            const uint64_t has = ballot(v >= 0);
            if (has != 0) {   // wave-uniform
                const int vf = __builtin_amdgcn_readlane(v, __builtin_ctzll(has));
                if (ballot(v >= 0 && v != vf) == 0) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) GW[k] = wave_sum_f64(GW[k]);
#pragma unroll
                    for (int k = 0; k < 3; ++k) gX[k] = wave_sum_f64(gX[k]);
                    if (lane == 0) {
                        for (int k = 0; k < 9; ++k) atomicAdd(&s_pose[vf * 12 + k], GW[k]);
                        for (int k = 0; k < 3; ++k) atomicAdd(&s_pose[vf * 12 + 9 + k], gX[k]);
                    }
                } else if (v >= 0) {
                    for (int k = 0; k < 9; ++k) atomicAdd(&s_pose[v * 12 + k], GW[k]);
                    for (int k = 0; k < 3; ++k) atomicAdd(&s_pose[v * 12 + 9 + k], gX[k]);
                }
            }
        }
    }
    if (want_pose) {
        __syncthreads();
        double *o = pose_blocks + (size_t)blockIdx.x * V * 12;
        for (int k = threadIdx.x; k < V * 12; k += blockDim.x) o[k] = s_pose[k];
    }
}

// Per Gaussian: its gradient is the sum of its records' contributions over
// the views, in a fixed order (deterministic): each half of the views in
// view order, then the two halves.  The loads of four views are in flight
// together.
__device__ __forceinline__ void gauss_sum_block(const ProjParams &pp, const ViewTable *__restrict__ vt,
                                                const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ inv,
                                                const float *__restrict__ rgrad, const GradOut &go,
                                                const int64_t *__restrict__ counters, int64_t blk) {
    const int V = vt->n_views;
    const uint32_t n_rec = (uint32_t)counters[kCntVisible];
    // two adjacent lanes per Gaussian, one per half of the views (each in
    // view order), their sums added by a lane exchange (a fixed order)
    const int64_t g = blk * blockDim.x + threadIdx.x;
    const int64_t i = g >> 1;
    const int half = (int)(g & 1);
    const int vh = (V + 1) / 2, va = half ? vh : 0, vb = half ? V : vh;
    float acc[kRecGrad];
    for (int k = 0; k < kRecGrad; ++k) acc[k] = 0.0f;
    for (int v0 = va; i < pp.n && v0 < vb; v0 += 4) {
        uint32_t sv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t gi = (int64_t)(v0 + k) * pp.n + i;
            const bool in = v0 + k < vb;
            const uint32_t c = in ? cnt[gi] : 0u;
            const uint32_t t = in ? inv[gi] : 0u;
            sv[k] = (c != 0u && t < n_rec) ? t : 0xffffffffu;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool vis = sv[k] != 0xffffffffu;
            const float *o = rgrad + kRecGrad * (size_t)(vis ? sv[k] : 0u);   // row 0 stands in, unused
            float row[kRecGrad];
#pragma unroll
            for (int c = 0; c < kRecGrad; ++c) row[c] = o[c];
#pragma unroll
            for (int c = 0; c < kRecGrad; ++c) acc[c] += vis ? row[c] : 0.0f;
        }
    }
#pragma unroll
    for (int k = 0; k < kRecGrad; ++k) {   // every lane takes part; the two halves added as (first + second)
        const float other = __shfl_xor(acc[k], 1, 64);
        acc[k] = half ? other + acc[k] : acc[k] + other;
    }
    if (i >= pp.n || half) return;
    if (go.gg.means)
        for (int k = 0; k < 3; ++k) go.gg.means[3 * i + k] = acc[k];
    if (go.gg.quats)
        for (int k = 0; k < 4; ++k) go.gg.quats[4 * i + k] = pp.iso ? 0.0f : acc[3 + k];
    if (go.gg.log_scales) {
        if (pp.iso)
            go.gg.log_scales[i] = acc[7];
        else
            for (int k = 0; k < 3; ++k) go.gg.log_scales[3 * i + k] = acc[7 + k];
    }
    if (go.gg.opacity_logits) go.gg.opacity_logits[i] = acc[10];
    if (go.gg.rgb)
        for (int k = 0; k < 3; ++k) go.gg.rgb[3 * i + k] = acc[11 + k];
}

// Per view (one block each): the pose partials (G_W, g_t) summed over the
// record blocks' rows in a fixed order (deterministic), then
// (G_W, g_t) -> dL/dq | t, dL/dt, dL/dq | C, dL/dC with C = -W^T t.
// A tracking loop's pose step, applied where the pose gradients are formed
// (st == nullptr: none).
struct PoseOpt {
    gsr_pose_adam hp;
    PoseOptState *st;
    float *quat, *trans;   // the poses the next iteration renders
    double *hist;          // per-iteration losses (may be null)
};

__device__ __forceinline__ void pose_final_view(const float *__restrict__ pq, const float *__restrict__ pt,
                                                bool centre, const PoseF64 *poses,
                                                const double *__restrict__ pose_blocks, int nblocks, int V,
                                                const gsr_pose_grads &pg, const PoseOpt &po, int v) {
    // What the lead thread needs after the reduction (the pose inputs, the
    // rotation and the optimiser state), one value per thread, requested
    // first so that these loads overlap the rows' loads, and put in LDS
    // after them (a value per thread keeps the registers of the kernel's other
    // block roles free).
    constexpr int kPreQ = 0, kPreT = 4, kPreW = 7, kPreS = 16;
    constexpr int kPre = kPreS + GSR_POSE_STATE_DOUBLES;
    __shared__ double s_red[12][4];
    __shared__ double s_pre[kPre];
    const int t = threadIdx.x;
    double pre = 0.0;
    if (t < kPreT)
        pre = pq[4 * v + t];
    else if (t < kPreW)
        pre = pt[3 * v + (t - kPreT)];
    else if (t < kPreS)
        pre = poses[v].W[t - kPreW];
    else if (t < kPre && po.st)
        pre = reinterpret_cast<const double *>(po.st + v)[t - kPreS];
    double acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
#pragma unroll 4   // loads in flight together; the additions keep their order
    for (int b = t; b < nblocks; b += 256) {
        const double *row = pose_blocks + ((size_t)b * V + v) * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] += row[k];
    }
    if (t < kPre) s_pre[t] = pre;
    // the block's rows summed in a fixed order: each wave's butterfly, then the four waves in order
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = wave_sum_f64(acc[k]);
    if ((t & 63) == 0)
        for (int k = 0; k < 12; ++k) s_red[k][t >> 6] = acc[k];
    __syncthreads();
    if (t != 0) return;
    const double *q = s_pre + kPreQ, *tin = s_pre + kPreT, *W = s_pre + kPreW;
    double GW[12];
    for (int k = 0; k < 12; ++k) GW[k] = ((s_red[k][0] + s_red[k][1]) + s_red[k][2]) + s_red[k][3];
    const double *gt = GW + 9;
    double gq[4];
    rot_grad_to_quat_f64(q, GW, gq);
    if (pg.dq_t)
        for (int k = 0; k < 4; ++k) pg.dq_t[4 * v + k] = (float)gq[k];
    if (pg.dt)
        for (int k = 0; k < 3; ++k) pg.dt[3 * v + k] = (float)gt[k];
    double C[3], gc[3];   // C = -W^T t (or given, with GSR_POSE_CENTRE); dL/dC = -W^T dL/dt
    for (int k = 0; k < 3; ++k) {
        C[k] = centre ? tin[k] : -(W[k] * tin[0] + W[3 + k] * tin[1] + W[6 + k] * tin[2]);
        gc[k] = -(W[k] * gt[0] + W[3 + k] * gt[1] + W[6 + k] * gt[2]);
    }
    if (pg.dc)
        for (int k = 0; k < 3; ++k) pg.dc[3 * v + k] = (float)gc[k];
    double G2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G2[3 * r + c] = GW[3 * r + c] - gt[r] * C[c];
    rot_grad_to_quat_f64(q, G2, gq);
    if (pg.dq_c)
        for (int k = 0; k < 4; ++k) pg.dq_c[4 * v + k] = (float)gq[k];
    if (po.st) {   // the step takes the gradients as written (FP32); pq and pt were read above
        double sq[4], sc[3];
        for (int k = 0; k < 4; ++k) sq[k] = (double)(float)gq[k];
        for (int k = 0; k < 3; ++k) sc[k] = (double)(float)gc[k];
        PoseOptState s0;
        double *sd = reinterpret_cast<double *>(&s0);
        for (int k = 0; k < GSR_POSE_STATE_DOUBLES; ++k) sd[k] = s_pre[kPreS + k];
        pose_adam_apply(v, sq, sc, po.hp, s0, po.st, po.quat, po.trans);
    }
}

// The last step of a backward, one launch: blocks [0, n_pose) finish the
// views' pose gradients, the next n_loss blocks the views' losses, the rest
// sum the Gaussians' gradients.  The three are independent (each reads what
// earlier kernels wrote), so their latencies overlap.
struct FinalArgs {
    int n_pose, n_loss;
    const float *pq, *pt;   // pose inputs
    int centre;             // pt holds the camera centre (GSR_POSE_CENTRE)
    const PoseF64 *poses;
    const double *pose_blocks;
    int pose_rows, V;
    gsr_pose_grads pg;
    PoseOpt po;
    const ViewTable *vt;   // loss
    const double *loss_tile;
    double *loss;
    ProjParams pp;   // Gaussian sums
    const uint32_t *cnt, *inv;
    const float *rgrad;
    GradOut go;
    const int64_t *counters;
    int64_t *loss_ticket;   // cleared by the call's set-up
};

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_finalize(FinalArgs a) {
    int b = (int)blockIdx.x;
    if (b < a.n_pose) {
        pose_final_view(a.pq, a.pt, a.centre != 0, a.poses, a.pose_blocks, a.pose_rows, a.V, a.pg, a.po, b);
        return;
    }
    b -= a.n_pose;
    if (b < a.n_loss) {
        loss_final_view(a.vt, a.loss_tile, a.loss, a.po.hist, a.loss_ticket, b);
        return;
    }
    b -= a.n_loss;
    gauss_sum_block(a.pp, a.vt, a.cnt, a.inv, a.rgrad, a.go, a.counters, b);
}

// Binning test hook: record fields in depth order.
template <bool ISO>
__global__ void k_debug_records(const int64_t *__restrict__ counters, const uint32_t *__restrict__ gid,
                                const float4 *__restrict__ rec, const uint2 *__restrict__ trect, int64_t max_rec,
                                uint32_t *o_gid, float *o_xy, float *o_rad, float *o_z, const ProjParams pp,
                                const ViewTable *__restrict__ vt, const PoseF64 *__restrict__ poses) {
    const int64_t M = counters[kCntVisible];
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < M && s < max_rec;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g = gid[s];
        o_gid[s] = g;
        o_xy[2 * s] = rec[3 * s].x;
        o_xy[2 * s + 1] = rec[3 * s].y;
        o_z[s] = rec[3 * s + 2].w;
        // the radius is recomputed exactly as the projection kernels do
        const int v = (int)(g / (uint64_t)pp.n);
        const int64_t i = (int64_t)g - (int64_t)v * pp.n;
        const GaussIn p = load_gauss<ISO>(pp.g, i);
        Proj r;
        project<true, ISO>(p, poses[v], vt->v[v], pp.z_near, pp.blur, r);
        o_rad[s] = r.radius;
    }
}

__global__ void k_debug_copy_u32(const uint32_t *src, const int64_t *counters, int which, int64_t max_n, uint32_t *dst,
                                 int64_t fixed_n) {
    const int64_t n0 = which >= 0 ? counters[which] : fixed_n;
    const int64_t n = n0 < max_n ? n0 : max_n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Tile ranges as [start, end), an empty one as (0, 0) (in the workspace it is
// (0xffffffff, 0), see the set-up).
__global__ void k_debug_ranges(const uint2 *__restrict__ src, int64_t n, uint2 *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint2 r = src[i];
        dst[i] = r.x < r.y ? r : make_uint2(0u, 0u);
    }
}

// Wave-primitive self test: 0 failures expected.
__global__ void k_selftest(int *fail) {
    const uint32_t lane = threadIdx.x;
    const float x = (float)(lane + 1);
    const float s = wave_sum(x);
    if (s != 2080.0f) atomicAdd(fail, 1);
    const float s63 = wave_sum_to63(lane == 17 ? 3.5f : 0.0f);
    if (lane == 63 && s63 != 3.5f) atomicAdd(fail, 1);
    const uint64_t m = ballot((lane % 3) == 0);
    const uint32_t r = rank_below(m);
    if ((lane % 3) == 0 && r != lane / 3) atomicAdd(fail, 1);
    if (lane_id() != lane) atomicAdd(fail, 1);
    const uint32_t mx = wave_max_u32(lane * 7 % 64);
    if (mx != 63u) atomicAdd(fail, 1);
    const double d = wave_sum_f64((double)lane);
    if (d != 2016.0) atomicAdd(fail, 1);
}

unsigned grid_for(int64_t n, int threads, int64_t max_blocks = 65536) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (unsigned)b;
}

// Calls that wait on the host (GSR_SYNC, gsr_plan) cannot be part of a graph.
gsr_status reject_capture(gsr_ctx *ctx, void *stream, const char *what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (ctx->capturing ||
        (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone))
        return fail(ctx, GSR_EINVAL, "%s waits on the host and cannot be captured into a graph", what);
    return GSR_OK;
}

// Copies the counters of the last call on the workspace to the host (waits
// for the stream); GSR_EHIP if a wait between blocks gave up.
gsr_status read_counters_sync(gsr_ctx *ctx, const gsr_workspace &ws, hipStream_t st, int64_t h[kNumCounters]) {
    gsr_status s = check_hip(ctx, hipMemcpyAsync(h, ws.ptr, sizeof(int64_t) * kNumCounters, hipMemcpyDeviceToHost, st),
                             "hipMemcpyAsync(counters)");
    if (s == GSR_OK) s = check_hip(ctx, hipStreamSynchronize(st), "hipStreamSynchronize");
    if (s != GSR_OK) return s;
    if (h[kCntSyncError] != 0)
        return fail(ctx, GSR_EHIP, "%lld waits between blocks of the binning gave up; outputs are undefined",
                    (long long)h[kCntSyncError]);
    return GSR_OK;
}

struct Call {
    bool count = false;
    bool hash = false;   // the forward writes the per-pixel decision hash
    bool keep_sticky = false;   // inside a tracking loop after its first iteration
    gsr_ctx *ctx;
    ViewTable tab;
    Layout L;
    gsr_workspace ws;
    hipStream_t st;
    ProjParams pp;
};

gsr_status prepare(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                   gsr_workspace ws, void *stream, Call &c) {
    if (!ctx) return GSR_EINVAL;
    if (!g) return fail(ctx, GSR_EINVAL, "gaussians must not be NULL");
    gsr_status s = validate_views(ctx, views, opts);
    if (s != GSR_OK) return s;
    if (opts->flags & GSR_SYNC) {
        s = reject_capture(ctx, stream, "GSR_SYNC");
        if (s != GSR_OK) return s;
    }
    if (g->n < 0) return fail(ctx, GSR_EINVAL, "n must be >= 0 (got %lld)", (long long)g->n);
    if ((int64_t)views->n_views * g->n >= (int64_t)0xffffffffLL)
        return fail(ctx, GSR_EUNSUPPORTED, "views x Gaussians must be < 2^32");
    const bool iso = (opts->flags & GSR_ISOTROPIC) != 0;   // isotropic Gaussians have no quaternions
    if (g->n > 0 && (!g->means || (!g->quats && !iso) || !g->log_scales || !g->opacity_logits || !g->rgb))
        return fail(ctx, GSR_EINVAL, "Gaussian parameter pointers must not be NULL");
    if (!views->quat || !views->trans) return fail(ctx, GSR_EINVAL, "pose pointers must not be NULL");
    if (!ws.ptr) return fail(ctx, GSR_EINVAL, "workspace pointer is NULL");
    if (ws.pair_capacity < 0 || ws.pair_capacity >= (int64_t)0xffffffffLL)
        return fail(ctx, GSR_EINVAL, "pair_capacity must be in [0, 2^32)");
    build_table(views, opts, c.tab);
    if (c.tab.total_tiles >= (1 << 24))   // a backward work item holds the tile in 24 bits
        return fail(ctx, GSR_EUNSUPPORTED, "more than 2^24 - 1 tiles in one call (got %d)", c.tab.total_tiles);
    c.L = make_layout(g->n, c.tab, ws.pair_capacity);
    if (ws.bytes < c.L.total)
        return fail(ctx, GSR_ENOMEM, "workspace has %zu bytes, this call needs %zu", ws.bytes, c.L.total);
    c.ctx = ctx;
    c.ws = ws;
    c.st = (hipStream_t)stream;
    c.pp.g = *g;
    c.pp.n = g->n;
    c.pp.z_near = opts->z_near;
    c.pp.blur = opts->blur2d;
    c.pp.iso = (opts->flags & GSR_ISOTROPIC) != 0;
    c.count = (opts->flags & GSR_COUNT_WORK) != 0;
    c.hash = (opts->flags & GSR_PIXEL_HASH) != 0;
    return GSR_OK;
}

// Projection, binning, sorting and ranges (forward up to the blend).
void enqueue_binning(Call &c, const gsr_views *views) {
    StageTimer timer(c.ctx, kStageBinning, c.st);
    const Layout &L = c.L;
    const gsr_workspace &ws = c.ws;
    hipStream_t st = c.st;
    ViewTable *vt = at<ViewTable>(ws, L.views);
    PoseF64 *poses = at<PoseF64>(ws, L.poses);
    int64_t *counters = at<int64_t>(ws, L.counters);
    uint32_t *cnt = at<uint32_t>(ws, L.cnt), *zkey = at<uint32_t>(ws, L.zkey);
    uint32_t *dk0 = at<uint32_t>(ws, L.dk0), *dv0 = at<uint32_t>(ws, L.dv0);
    uint32_t *dk1 = at<uint32_t>(ws, L.dk1), *dv1 = at<uint32_t>(ws, L.dv1);
    char *sync = at<char>(ws, L.sync);
    SyncState ss{reinterpret_cast<uint32_t *>(sync), reinterpret_cast<uint64_t *>(sync + L.sync_status),
                 counters + kCntSyncError};
    SortState so{at<uint32_t>(ws, L.scounts), at<uint32_t>(ws, L.stotals)};
    const int64_t sync16 = (int64_t)(L.sync_bytes / 16);
    {
        // one thread per Gaussian (none for an empty call: the set-up still runs)
        const unsigned grid = L.vn > 0 ? grid_for(c.pp.n, 256, 1ll << 30) : 1u;
        ProjParams pp = c.pp;
        if (L.vn == 0) pp.n = 0;
        hipLaunchKernelGGL(c.pp.iso ? k_setup_project<true> : k_setup_project<false>, dim3(grid), dim3(256), 0, st,
                           c.tab, vt, views->quat, views->trans, poses, counters, reinterpret_cast<uint4 *>(sync),
                           sync16, at<uint2>(ws, L.ranges), L.T, c.keep_sticky, pp, cnt, zkey);
    }
    SweepState sw{reinterpret_cast<uint32_t *>(sync + L.sync_sweep), reinterpret_cast<uint32_t *>(sync),
                  counters + kCntSyncError};
    uint32_t *dhist = reinterpret_cast<uint32_t *>(sync + L.sync_hist), *thist = dhist + 256 * kDepthPasses;
    // Tile-local binning: the visible (view, Gaussian) items compacted in
    // index order (their depth keys beside them, in dk0), counted.  Else the
    // visible records in depth order: stable sort on the float32 depth bits
    // (positive floats sort as integers), which also compacts and counts them.
    const bool wide = L.vn >= kCompactWideMin;
    const int64_t compact_chunk = (int64_t)kCompactThreads * (wide ? 8 : 4);
    auto compact = wide ? k_compact_hist<8> : k_compact_hist<4>;
    if (L.vn > 0 && L.tile_local) {
        hipLaunchKernelGGL(compact, dim3((unsigned)((L.vn + compact_chunk - 1) / compact_chunk)),
                           dim3(kCompactThreads), 0, st, (const uint32_t *)cnt, (const uint32_t *)zkey, L.vn, dk0, dv0,
                           ss, (uint32_t)kIdCompact, (uint32_t *)nullptr, counters + kCntVisible,
                           reinterpret_cast<uint32_t *>(sync + L.sync_vstart), c.pp.n);
    } else if (L.vn > 0) {
        if (L.depth_sweep) {
            hipLaunchKernelGGL(compact, dim3((unsigned)((L.vn + compact_chunk - 1) / compact_chunk)),
                               dim3(kCompactThreads), 0, st, (const uint32_t *)cnt, (const uint32_t *)zkey, L.vn, dk0,
                               dv0, ss, (uint32_t)kIdCompact, dhist, counters + kCntVisible, (uint32_t *)nullptr,
                               (int64_t)1);
            for (int p = 0; p < kDepthPasses; ++p) {   // (k0, v0) -> (k1, v1) -> ... -> (k0, v0)
                const bool from0 = p % 2 == 0;
                hipLaunchKernelGGL(k_sweep<PairIn>, dim3((unsigned)sweep_blocks(L.vn)), dim3(kSweepThreads), 0, st,
                                   PairIn{from0 ? dk0 : dk1, from0 ? dv0 : dv1}, from0 ? dk1 : dk0, from0 ? dv1 : dv0,
                                   (const int64_t *)(counters + kCntVisible), L.vn, 8 * p, 8,
                                   (const uint32_t *)(dhist + 256 * p), sw, (uint32_t)(kIdSweepDepth + p),
                                   (uint2 *)nullptr, (int64_t)0);
            }
        } else {
            radix_sort_visible(cnt, zkey, L.vn, dk0, dv0, dk1, dv1, counters + kCntVisible, so, st);
        }
    }
    const uint32_t *gid_sorted = dv0;
    float4 *rec = at<float4>(ws, L.rec);
    uint2 *trect = at<uint2>(ws, L.trect);
    uint32_t *cnt_s = at<uint32_t>(ws, L.cnt_s), *inv = at<uint32_t>(ws, L.inv);
    uint32_t *pk0 = at<uint32_t>(ws, L.pk0), *pv0 = at<uint32_t>(ws, L.pv0);
    uint32_t *pk1 = at<uint32_t>(ws, L.pk1), *pv1 = at<uint32_t>(ws, L.pv1);
    uint32_t *poff = at<uint32_t>(ws, L.poff);
    uint32_t *chunk_first = at<uint32_t>(ws, L.chunk);
    const int64_t n_chunks = (L.kcap + kEmitChunk - 1) / kEmitChunk;
    // records and their pair offsets; the last block checks the pair capacity
    float *rrows = c.tab.deterministic ? nullptr : at<float>(ws, L.rrows);
    OffSink osink{poff, chunk_first, n_chunks};
    if (L.depth_sweep) {   // few records: one launch
        if (L.vn > 0)
            hipLaunchKernelGGL(c.pp.iso ? k_gather_scan<true> : k_gather_scan<false>,
                               dim3((unsigned)((L.vn + 255) / 256)), dim3(256), 0, st, c.pp, vt, poses, counters,
                               gid_sorted, rec, trect, cnt_s, inv, c.pp.g.rgb, rrows, ss, (uint32_t)kIdOffsets,
                               osink, PairTotal{counters, L.kcap});
    } else {
        if (L.vn > 0)
            hipLaunchKernelGGL(c.pp.iso ? k_gather<true> : k_gather<false>, dim3(grid_for(L.vn, 256, 1ll << 24)),
                               dim3(256), 0, st, c.pp, vt, poses, counters, gid_sorted, rec, trect, cnt_s, inv,
                               c.pp.g.rgb, rrows);
        scan_exclusive(CntSrc{cnt_s}, osink, counters + kCntVisible, L.vn, ss, kIdOffsets,
                       PairTotal{counters, L.kcap}, st);
    }
    uint2 *ranges = at<uint2>(ws, L.ranges);
    if (L.tile_local) {
        // per-block tile counts, every tile's offsets over the blocks and its
        // total, the list ranges (and the work order), the pairs placed in
        // their lists, each list sorted
        uint32_t *torder = at<uint32_t>(ws, L.torder), *tcnt = at<uint32_t>(ws, L.tcnt);
        uint32_t *ttot = at<uint32_t>(ws, L.ttot), *tstart = at<uint32_t>(ws, L.tstart);
        const bool pairs = L.vn > 0 && L.kcap > 0;
        const uint32_t *vrec = reinterpret_cast<const uint32_t *>(sync + L.sync_vstart);
        if (pairs) {
            hipLaunchKernelGGL(k_emit_count, dim3((unsigned)n_chunks), dim3(kEmitThreads), 0, st,
                               (const int64_t *)counters, (const uint32_t *)poff, (const uint32_t *)chunk_first,
                               (const uint2 *)trect, gid_sorted, (const ViewTable *)vt, c.pp.n, L.T, L.tv_max, tcnt,
                               at<uint2>(ws, L.espan));
        }
        if (L.T > 0) {
            hipLaunchKernelGGL(k_tile_offsets, dim3((unsigned)((L.T * kOffsetsParts + 255) / 256)), dim3(256), 0, st,
                               (const ViewTable *)vt, (const int64_t *)counters, vrec, (const uint32_t *)poff, L.T,
                               L.tv_max, tcnt, ttot);
            hipLaunchKernelGGL(k_tile_ranges, dim3(1), dim3(kOrderThreads), 0, st, (const uint32_t *)ttot, L.T,
                               ranges, tstart, L.cp_slots, torder, at<uint32_t>(ws, L.cpoff), at<uint32_t>(ws, L.work),
                               at<int64_t>(ws, L.nwork), counters);
        }
        if (pairs) {
            hipLaunchKernelGGL(k_emit_place, dim3((unsigned)n_chunks), dim3(kEmitThreads), 0, st,
                               (const int64_t *)counters, (const uint32_t *)poff, (const uint32_t *)chunk_first,
                               (const uint2 *)trect, gid_sorted, (const ViewTable *)vt, c.pp.n, L.T, L.tv_max,
                               (const uint32_t *)tcnt, (const uint32_t *)tstart, (const uint2 *)at<uint2>(ws, L.espan),
                               (const uint32_t *)dk0, at<uint2>(ws, L.pkv));
            hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)std::min<int64_t>(L.T, kTileSortGrid)),
                               dim3(kTileSortThreads), 0, st, (const uint2 *)ranges, (const uint32_t *)torder, L.T, counters,
                               (const uint32_t *)dk0, (const uint2 *)at<uint2>(ws, L.pkv), pv1, pk0, pk1);
        }
        return;
    }
    if (L.vn > 0 && L.kcap > 0)
        hipLaunchKernelGGL(k_emit, dim3((unsigned)n_chunks), dim3(kEmitThreads), 0, st, counters, poff,
                           (const uint32_t *)chunk_first, trect, gid_sorted, vt, c.pp.n, pk0, pv0,
                           L.tile_sweep ? thist : nullptr, L.tile_bits);
    // tile order (stable: depth order within a tile); the values are the
    // pairs' records; the last pass also sets every tile's [start, end)
    if (L.tile_sweep) {
        const int passes = (L.tile_bits + 7) / 8;
        for (int p = 0; L.kcap > 0 && p < passes; ++p) {   // (k0, v0) -> (k1, v1) -> ...
            const bool from0 = p % 2 == 0, last = p == passes - 1;
            const int dbits = std::min(8, L.tile_bits - 8 * p);
            hipLaunchKernelGGL(k_sweep<PairIn>, dim3((unsigned)sweep_blocks(L.kcap)), dim3(kSweepThreads), 0, st,
                               PairIn{from0 ? pk0 : pk1, from0 ? pv0 : pv1}, from0 ? pk1 : pk0, from0 ? pv1 : pv0,
                               (const int64_t *)(counters + kCntPairsUsed), L.kcap, 8 * p, dbits,
                               (const uint32_t *)(thist + 256 * p), sw, (uint32_t)(kIdSweepTile + p),
                               last ? ranges : (uint2 *)nullptr, (int64_t)L.T);
        }
    } else {
        radix_sort(pk0, pv0, pk1, pv1, counters + kCntPairsUsed, L.kcap, L.tile_bits, so, st, ranges, L.T);
    }
    if (L.T > 0)
        hipLaunchKernelGGL(k_work_order, dim3(1), dim3(kOrderThreads), 0, st, (const uint2 *)ranges, L.T, L.cp_slots,
                           at<uint32_t>(ws, L.torder), at<uint32_t>(ws, L.cpoff), at<uint32_t>(ws, L.work),
                           at<int64_t>(ws, L.nwork), counters);
}

// record index of every sorted pair (the sort's result buffer is fixed by the key bits)
const uint32_t *pair_values(const Call &c) {
    if (c.L.tile_local) return at<uint32_t>(c.ws, c.L.pv1);   // where the per-tile sort writes
    const int passes = (c.L.tile_bits + 7) / 8;
    const bool in1 = (c.L.kcap > 0 && c.L.tile_bits > 0) ? (passes % 2 == 1) : false;
    return at<uint32_t>(c.ws, in1 ? c.L.pv1 : c.L.pv0);
}

// each record's view * N + index (records in depth order, or in that index
// order with tile-local binning)
const uint32_t *depth_sorted_gid(const Call &c) {
    return at<uint32_t>(c.ws, c.L.dv0);   // where the depth sort or the compaction leaves it
}

void enqueue_blend_fwd(Call &c, gsr_images out) {
    StageTimer timer(c.ctx, kStageBlendFwd, c.st);
    const Layout &L = c.L;
    BlendOut bo{out.rgb, out.depth, out.sil, at<float>(c.ws, L.tfinal), at<uint32_t>(c.ws, L.nlast),
                at<uint32_t>(c.ws, L.phash), at<uint64_t>(c.ws, L.cmask)};
    // the tiles' blocks, tile ranks dealt to the XCDs in turn (see locate_block)
    const int64_t nsub = (int64_t)(c.tab.tile_w / kBlk) * (c.tab.tile_h / kBlk);
    const unsigned grid = (unsigned)(8 * nsub * ((L.T + 7) / 8));
    if (grid > 0) {
        auto kern = c.count ? (c.hash ? k_blend_fwd<true, true> : k_blend_fwd<true, false>)
                            : (c.hash ? k_blend_fwd<false, true> : k_blend_fwd<false, false>);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, c.st, at<ViewTable>(c.ws, L.views),
                           at<float4>(c.ws, L.rec), pair_values(c), at<uint2>(c.ws, L.ranges),
                           at<uint32_t>(c.ws, L.torder), at<uint32_t>(c.ws, L.cpoff), at<float>(c.ws, L.cp),
                           at<int64_t>(c.ws, L.counters), bo);
    }
}

// The backward blend's instantiation for a call.
template <int NV, bool ATOMIC, int WAVES>
auto blend_bwd_kernel_w(bool fused, bool count) {
    return fused ? (count ? k_blend_bwd<true, true, NV, ATOMIC, WAVES> : k_blend_bwd<true, false, NV, ATOMIC, WAVES>)
                 : (count ? k_blend_bwd<false, true, NV, ATOMIC, WAVES> : k_blend_bwd<false, false, NV, ATOMIC, WAVES>);
}
template <int NV, bool ATOMIC>
auto blend_bwd_kernel(bool fused, bool count, int waves) {
    return waves <= kBwdWavesSmall ? blend_bwd_kernel_w<NV, ATOMIC, kBwdWavesSmall>(fused, count)
                                   : blend_bwd_kernel_w<NV, ATOMIC, kBwdWavesLarge>(fused, count);
}
template <int NV, bool ATOMIC>
auto record_bwd_kernel(bool iso) {
    return iso ? k_record_bwd<true, NV, ATOMIC> : k_record_bwd<false, NV, ATOMIC>;
}

void enqueue_backward(Call &c, const gsr_views *views, const gsr_options *opts, gsr_images out, LossIn li,
                      bool fused, gsr_gaussian_grads *gg, gsr_pose_grads *pg, const PoseOpt *po = nullptr) {
    const Layout &L = c.L;
    hipStream_t st = c.st;
    ViewTable *vt = at<ViewTable>(c.ws, L.views);
    int64_t *counters = at<int64_t>(c.ws, L.counters);
    // 2D gradient rows: per (tile, entry) pair (GSR_DETERMINISTIC) or per record (atomics)
    const bool atomic = !c.tab.deterministic;
    float *gpairs = atomic ? at<float>(c.ws, L.rrows) : at<float>(c.ws, L.gpairs);
    li.loss_tile = at<double>(c.ws, L.losst);
    GradOut go;
    memset(&go, 0, sizeof(go));
    if (gg) go.gg = *gg;
    go.want_gauss = gg && !(opts->flags & GSR_NO_GAUSS_GRADS) &&
                    (gg->means || gg->quats || gg->log_scales || gg->opacity_logits || gg->rgb);
    go.want_pose = pg && !(opts->flags & GSR_NO_POSE_GRADS) && (pg->dq_t || pg->dt || pg->dq_c || pg->dc);
    const bool pose_only = !go.want_gauss;   // 6 partials per entry reach the pose
    BlendOut bo{out.rgb, out.depth, out.sil, at<float>(c.ws, L.tfinal), at<uint32_t>(c.ws, L.nlast),
                at<uint32_t>(c.ws, L.phash), at<uint64_t>(c.ws, L.cmask)};
    {
        StageTimer timer(c.ctx, kStageBlendBwd, st);
        const unsigned grid = (unsigned)(((L.work_cap + 7) / 8) * 8);   // the items past n_work leave at once
        const unsigned threads = (unsigned)(64 * (opts->tile_w / kBlk) * (opts->tile_h / kBlk));
        if (grid > 0 && L.kcap > 0 && L.T > 0) {
            const int waves = (int)(threads / 64);
            auto kern = pose_only ? (atomic ? blend_bwd_kernel<6, true>(fused, c.count, waves)
                                            : blend_bwd_kernel<6, false>(fused, c.count, waves))
                                  : (atomic ? blend_bwd_kernel<10, true>(fused, c.count, waves)
                                            : blend_bwd_kernel<10, false>(fused, c.count, waves));
            hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, vt, at<float4>(c.ws, L.rec), pair_values(c),
                               at<uint32_t>(c.ws, L.poff), at<uint2>(c.ws, L.trect), at<uint2>(c.ws, L.ranges),
                               at<uint32_t>(c.ws, L.work), at<int64_t>(c.ws, L.nwork), at<uint32_t>(c.ws, L.cpoff),
                               at<float>(c.ws, L.cp), counters, bo, li, gpairs);
        }
    }
    if (fused && L.kcap == 0)   // no blend ran: every tile's partial is zero
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(L.T, 256)), dim3(256), 0, st, li.loss_tile, L.T);
    StageTimer timer(c.ctx, kStageProjectBwd, st);
    const unsigned rec_blocks = std::min<unsigned>(grid_for(L.vn, kRecBwdItemsPerBlock, 1ll << 30), kRecBwdMaxBlocks);
    double *pose_blocks = at<double>(c.ws, L.poseblk);
    // with atomics the record rows are also cleared here, so this runs whenever the blend did
    if (c.pp.n > 0 && (go.want_gauss || go.want_pose || (atomic && L.kcap > 0 && L.T > 0)))
        hipLaunchKernelGGL(pose_only ? (atomic ? record_bwd_kernel<6, true>(c.pp.iso)
                                               : record_bwd_kernel<6, false>(c.pp.iso))
                                     : (atomic ? record_bwd_kernel<10, true>(c.pp.iso)
                                               : record_bwd_kernel<10, false>(c.pp.iso)),
                           dim3(rec_blocks), dim3(256), 0, st,
                           c.pp, vt, at<PoseF64>(c.ws, L.poses),
                           depth_sorted_gid(c), at<uint32_t>(c.ws, L.poff), at<uint32_t>(c.ws, L.cnt_s), gpairs,
                           (const int64_t *)counters, at<float>(c.ws, L.rgrad), pose_blocks, go.want_gauss,
                           go.want_pose);
    if (go.want_pose && c.pp.n == 0)   // no record blocks ran: their rows are zero
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_for((int64_t)rec_blocks * 12 * views->n_views, 256)), dim3(256), 0,
                           st, pose_blocks, (int64_t)rec_blocks * 12 * views->n_views);
    FinalArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.n_pose = go.want_pose ? views->n_views : 0;
    fa.n_loss = fused ? views->n_views : 0;
    const int64_t n_gauss_blocks = (c.pp.n > 0 && go.want_gauss) ? grid_for(2 * c.pp.n, 256, 1ll << 30) : 0;   // two lanes per Gaussian
    fa.pq = views->quat;
    fa.pt = views->trans;
    fa.centre = c.tab.pose_centre;
    fa.poses = at<PoseF64>(c.ws, L.poses);
    fa.pose_blocks = pose_blocks;
    fa.pose_rows = (int)rec_blocks;
    fa.V = views->n_views;
    if (pg) fa.pg = *pg;
    if (po) fa.po = *po;
    fa.vt = vt;
    fa.loss_tile = li.loss_tile;
    fa.loss = li.loss;
    fa.pp = c.pp;
    fa.cnt = at<uint32_t>(c.ws, L.cnt);
    fa.inv = at<uint32_t>(c.ws, L.inv);
    fa.rgrad = at<float>(c.ws, L.rgrad);
    fa.go = go;
    fa.counters = counters;
    fa.loss_ticket = counters + kCntLossTicket;
    const int64_t n_final = fa.n_pose + fa.n_loss + n_gauss_blocks;
    if (n_final > 0) hipLaunchKernelGGL(k_finalize, dim3((unsigned)n_final), dim3(256), 0, st, fa);
    // with the Gaussian gradients off, or for N = 0, the outputs are still defined (zero)
    if (gg && !go.want_gauss && c.pp.n > 0) {
        float *ptrs[5] = {gg->means, gg->quats, gg->log_scales, gg->opacity_logits, gg->rgb};
        const int64_t sz[5] = {3 * c.pp.n, 4 * c.pp.n, (c.pp.iso ? 1 : 3) * c.pp.n, c.pp.n, 3 * c.pp.n};
        for (int k = 0; k < 5; ++k)
            if (ptrs[k])
                hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(sz[k], 256)), dim3(256), 0, st, (uint32_t *)ptrs[k],
                                   sz[k], 0u);
    }
}

gsr_status finish(Call &c, const char *what) {
    return check_hip(c.ctx, hipGetLastError(), what);
}

// GSR_SYNC: waits for the binning just enqueued and fails with GSR_ECAPACITY,
// enqueueing nothing more, if its pairs exceed the workspace's capacity.
gsr_status sync_capacity(Call &c) {
    gsr_status s = check_hip(c.ctx, hipGetLastError(), "binning launch");
    if (s != GSR_OK) return s;
    int64_t h[kNumCounters];
    s = read_counters_sync(c.ctx, c.ws, c.st, h);
    if (s != GSR_OK) return s;
    if (h[kCntOverflow] != 0)
        return fail(c.ctx, GSR_ECAPACITY,
                    "%lld (Gaussian, tile) pairs needed, the workspace holds %lld; no output was written",
                    (long long)h[kCntPairs], (long long)c.L.kcap);
    return GSR_OK;
}

gsr_status render_loss_grad_impl(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                 const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws,
                                 gsr_images out, double *loss, gsr_gaussian_grads *gg, gsr_pose_grads *pg,
                                 void *stream, bool keep_sticky = false, const PoseOpt *po = nullptr) {
    Call c;
    gsr_status s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    c.keep_sticky = keep_sticky;
    if (!out.rgb || !out.depth || !out.sil) return fail(ctx, GSR_EINVAL, "output images must not be NULL");
    if (!targets || !targets->rgb || !targets->depth) return fail(ctx, GSR_EINVAL, "targets rgb and depth are required");
    if (!loss) return fail(ctx, GSR_EINVAL, "loss must not be NULL");
    s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    enqueue_binning(c, views);
    if (opts->flags & GSR_SYNC) {
        s = sync_capacity(c);
        if (s != GSR_OK) return s;
    }
    enqueue_blend_fwd(c, out);
    LossIn li;
    memset(&li, 0, sizeof(li));
    li.t_rgb = targets->rgb;
    li.t_depth = targets->depth;
    li.t_sil = targets->sil;
    li.t_prior = targets->prior;
    li.t_weight = targets->weight;
    li.w_rgb = opts->w_rgb;
    li.w_depth = opts->w_depth;
    li.w_sil = opts->w_sil;
    li.w_prior = opts->w_prior;
    li.sil_thresh = opts->sil_mask_thresh;
    li.loss = loss;
    enqueue_backward(c, views, opts, out, li, true, gg, pg, po);
    return finish(c, "gsr_render_loss_grad launch");
}


// The tracking loop (enqueue only): iters x (render + loss + pose gradients,
// decoupled Adam step).
gsr_status track_impl(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int32_t V, float *quat,
                      float *trans, const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws,
                      gsr_images out, double *loss, gsr_pose_grads *pg, const gsr_pose_adam *hp, double *state,
                      int32_t iters, double *loss_hist, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!g || !cams || !opts || !hp || !state || !quat || !trans || !pg || !pg->dq_c || !pg->dc)
        return fail(ctx, GSR_EINVAL, "track: NULL argument (g, cams, opts, hp, state, quat, trans, pg->dq_c, pg->dc)");
    if (iters < 0) return fail(ctx, GSR_EINVAL, "track: iters must be >= 0 (got %d)", iters);
    if (V < 1 || V > GSR_MAX_VIEWS) return fail(ctx, GSR_EINVAL, "track: n_views must be in [1, %d]", GSR_MAX_VIEWS);
    if (opts->flags & GSR_POSE_CENTRE)
        return fail(ctx, GSR_EUNSUPPORTED, "track: the loop updates (q, t) poses; GSR_POSE_CENTRE is not accepted");
    const gsr_views views{V, cams, quat, trans};
    gsr_options o = *opts;
    o.flags |= GSR_NO_GAUSS_GRADS;
    o = resolve_tile(ctx, g->n, &views, &o);
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    for (int32_t it = 0; it < iters && s == GSR_OK; ++it) {
        // the pose step runs in the backward's last launch, where the pose
        // gradients are formed
        const PoseOpt po{*hp, reinterpret_cast<PoseOptState *>(state), quat, trans,
                         loss_hist ? loss_hist + (size_t)it * V : nullptr};
        s = render_loss_grad_impl(ctx, g, &views, &o, targets, ws, out, loss, nullptr, pg, stream, it > 0, &po);
    }
    return s;
}

// Moment-array layout of the mapping state: segment k of both arrays starts
// at moff[k] floats (256-byte aligned); returns the floats of one array.
int64_t map_layout(int64_t n, bool iso, int64_t moff[kMapSegs], int64_t cnt[kMapSegs]) {
    const int64_t per[kMapSegs] = {3, 4, iso ? 1 : 3, 1, 3};
    int64_t off = 0;
    for (int k = 0; k < kMapSegs; ++k) {
        cnt[k] = (k == 1 && iso) ? 0 : per[k] * n;
        moff[k] = off;
        off += (cnt[k] + (int64_t)kMapAlign - 1) / (int64_t)kMapAlign * (int64_t)kMapAlign;
    }
    return off;
}

// One Adam step of the map (enqueue only).
gsr_status map_step_impl(gsr_ctx *ctx, const gsr_gaussians_rw &params, const gsr_gaussian_grads *grads, bool iso,
                         const gsr_map_adam *hp, void *state, hipStream_t st) {
    if (!grads || !hp || !state) return fail(ctx, GSR_EINVAL, "map_opt_step: NULL argument");
    if (params.n < 0) return fail(ctx, GSR_EINVAL, "map_opt_step: n must be >= 0");
    float *xs[kMapSegs] = {params.means, iso ? nullptr : params.quats, params.log_scales, params.opacity_logits,
                           params.rgb};
    const float *gs[kMapSegs] = {grads->means, iso ? nullptr : grads->quats, grads->log_scales,
                                 grads->opacity_logits, grads->rgb};
    const float lrs[kMapSegs] = {hp->lr_means, hp->lr_quats, hp->lr_log_scales, hp->lr_opacity, hp->lr_rgb};
    int64_t moff[kMapSegs], cnt[kMapSegs];
    const int64_t per_array = map_layout(params.n, iso, moff, cnt);
    MapSegs segs;
    int64_t most = 0;
    for (int k = 0; k < kMapSegs; ++k) {
        if ((xs[k] == nullptr) != (gs[k] == nullptr))
            return fail(ctx, GSR_EINVAL, "map_opt_step: parameter array %d and its gradient must both be given", k);
        segs.s[k] = MapSeg{xs[k], gs[k], xs[k] ? cnt[k] : 0, moff[k], lrs[k]};
        most = std::max(most, segs.s[k].count);
    }
    MapHeader *h = reinterpret_cast<MapHeader *>(state);
    float *m = reinterpret_cast<float *>(static_cast<char *>(state) + kMapHeader);
    float *v = m + per_array;
    hipLaunchKernelGGL(k_map_opt_begin, dim3(1), dim3(64), 0, st, h, hp->beta1, hp->beta2);
    if (most > 0) {
        const unsigned gx = grid_for((most + 3) / 4, 256, 4096);
        hipLaunchKernelGGL(k_map_opt_step, dim3(gx, kMapSegs), dim3(256), 0, st, segs, m, v, (const MapHeader *)h,
                           hp->beta1, hp->beta2, hp->eps);
    }
    return check_hip(ctx, hipGetLastError(), "map step launch");
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// The mapping loop (enqueue only): iters x (render + loss + Gaussian
// gradients over the views, Adam step of the map).
gsr_status map_iterate_impl(gsr_ctx *ctx, const gsr_gaussians_rw &params, const gsr_views *views,
                            const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws, gsr_images out,
                            double *loss, gsr_gaussian_grads *gg, const gsr_map_adam *hp, void *state, int32_t iters,
                            double *loss_hist, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!views || !opts || !gg || !hp || !state)
        return fail(ctx, GSR_EINVAL, "map_iterate: NULL argument (views, opts, gg, hp, state)");
    if (iters < 0) return fail(ctx, GSR_EINVAL, "map_iterate: iters must be >= 0 (got %d)", iters);
    if (opts->flags & GSR_NO_GAUSS_GRADS)
        return fail(ctx, GSR_EINVAL, "map_iterate: GSR_NO_GAUSS_GRADS leaves nothing to update");
    const bool iso = (opts->flags & GSR_ISOTROPIC) != 0;
    const gsr_gaussians g{params.n, params.means, params.quats, params.log_scales, params.opacity_logits, params.rgb};
    gsr_options o = *opts;
    o.flags |= GSR_NO_POSE_GRADS;
    o = resolve_tile(ctx, g.n, views, &o);
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    for (int32_t it = 0; it < iters && s == GSR_OK; ++it) {
        s = render_loss_grad_impl(ctx, &g, views, &o, targets, ws, out, loss, gg, nullptr, stream, it > 0);
        if (s != GSR_OK) break;
        s = map_step_impl(ctx, params, gg, iso, hp, state, st);
        if (s == GSR_OK && loss_hist)
            hipLaunchKernelGGL(k_copy_f64, dim3(1), dim3(64), 0, st, (const double *)loss,
                               loss_hist + (size_t)it * views->n_views, views->n_views);
        if (s == GSR_OK) s = check_hip(ctx, hipGetLastError(), "gsr_map_iterate launch");
    }
    return s;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

gsr_status gsr_create(gsr_ctx **out, int device) {
    if (!out) {
        g_create_err = "out must not be NULL";
        return GSR_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) {
        g_create_err = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
        return GSR_EHIP;
    }
    if (device < 0 || device >= ndev) {
        g_create_err = "device ordinal out of range";
        return GSR_EINVAL;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        g_create_err = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
        return GSR_EHIP;
    }
    void *sp = nullptr;
    if (device < kMaxScratchDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            int prev = 0;
            e = hipGetDevice(&prev);
            if (e == hipSuccess) e = hipSetDevice(device);
            if (e == hipSuccess) e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
            if (e == hipSuccess) e = hipSetDevice(prev);
            if (e != hipSuccess) {
                g_create_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                return GSR_EHIP;
            }
            g_scratch_ptr[device] = sp;
        }
        sp = g_scratch_ptr[device];
    }
    gsr_ctx *c = new gsr_ctx;
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->scratch = sp;
    *out = c;
    return GSR_OK;
}

void gsr_destroy(gsr_ctx *ctx) {
    if (!ctx) return;
    for (auto &r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    delete ctx;
}

const char *gsr_last_error(const gsr_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

gsr_status gsr_workspace_size(gsr_ctx *ctx, int64_t n, const gsr_views *views, const gsr_options *opts,
                              int64_t pair_capacity, size_t *bytes) {
    // needs no device: with ctx == NULL errors go to the text gsr_last_error(NULL) returns
    if (!bytes) return fail(ctx, GSR_EINVAL, "bytes must not be NULL");
    gsr_options o_res;
    if (opts && views) {
        o_res = resolve_tile(ctx, n, views, opts);
        opts = &o_res;
    }
    gsr_status s = validate_views(ctx, views, opts);
    if (s != GSR_OK) return s;
    if (n < 0) return fail(ctx, GSR_EINVAL, "n must be >= 0");
    if (pair_capacity < 0 || pair_capacity >= (int64_t)0xffffffffLL)
        return fail(ctx, GSR_EINVAL, "pair_capacity must be in [0, 2^32)");
    if ((int64_t)views->n_views * n >= (int64_t)0xffffffffLL)
        return fail(ctx, GSR_EUNSUPPORTED, "views x Gaussians must be < 2^32");
    ViewTable tab;
    build_table(views, opts, tab);
    *bytes = make_layout(n, tab, pair_capacity).total;
    return GSR_OK;
}

gsr_status gsr_forward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                       gsr_workspace ws, gsr_images out, void *stream) {
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    Call c;
    gsr_status s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    if (!out.rgb || !out.depth || !out.sil) return fail(ctx, GSR_EINVAL, "output images must not be NULL");
    if (ctx->device >= 0) {
        s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        if (s != GSR_OK) return s;
    }
    enqueue_binning(c, views);
    if (opts->flags & GSR_SYNC) {
        s = sync_capacity(c);
        if (s != GSR_OK) return s;
    }
    enqueue_blend_fwd(c, out);
    return finish(c, "gsr_forward launch");
}

gsr_status gsr_backward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                        gsr_workspace ws, gsr_images out, const float *g_rgb, const float *g_depth,
                        const float *g_sil, gsr_gaussian_grads *gg, gsr_pose_grads *pg, void *stream) {
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    Call c;
    gsr_status s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    LossIn li;
    memset(&li, 0, sizeof(li));
    li.g_rgb = g_rgb;
    li.g_depth = g_depth;
    li.g_sil = g_sil;
    enqueue_backward(c, views, opts, out, li, false, gg, pg);
    return finish(c, "gsr_backward launch");
}

gsr_status gsr_render_loss_grad(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws,
                                gsr_images out, double *loss, gsr_gaussian_grads *gg, gsr_pose_grads *pg,
                                void *stream) {
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    return render_loss_grad_impl(ctx, g, views, opts, targets, ws, out, loss, gg, pg, stream);
}

// The fused call with the device's static scratch as its workspace: the pair
// capacity is the largest whose layout fits the scratch.  No allocation of
// any kind (no device memory, no events); GSR_SYNC is refused because the
// host wait it adds would copy through the runtime's staging memory.
gsr_status gsr_render_loss_grad_noalloc(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                        const gsr_options *opts, const gsr_targets *targets, gsr_images out,
                                        double *loss, gsr_gaussian_grads *gg, gsr_pose_grads *pg, void *stream,
                                        gsr_workspace *used) {
    if (!ctx) return GSR_EINVAL;
    if (!ctx->scratch) return fail(ctx, GSR_EUNSUPPORTED, "no static scratch on device %d", ctx->device);
    if (!g || !views || !opts) return fail(ctx, GSR_EINVAL, "g, views and opts must not be NULL");
    if (opts->flags & GSR_SYNC) return fail(ctx, GSR_EINVAL, "the static-scratch call does not accept GSR_SYNC");
    const gsr_options o = resolve_tile(ctx, g->n, views, opts);
    gsr_status s = validate_views(ctx, views, &o);
    if (s != GSR_OK) return s;
    if (g->n < 0) return fail(ctx, GSR_EINVAL, "n must be >= 0 (got %lld)", (long long)g->n);
    if ((int64_t)views->n_views * g->n >= (int64_t)0xffffffffLL)
        return fail(ctx, GSR_EUNSUPPORTED, "views x Gaussians must be < 2^32");
    ViewTable tab;
    build_table(views, &o, tab);
    const size_t base = make_layout(g->n, tab, 0).total;
    if (base > kStaticScratchBytes)
        return fail(ctx, GSR_ENOMEM,
                    "this call needs %zu bytes before any pair, the static scratch holds %zu (%zu MiB): use "
                    "gsr_render_loss_grad with a workspace",
                    base, kStaticScratchBytes, kStaticScratchBytes >> 20);
    // the largest pair capacity whose layout fits (the layout grows with it)
    int64_t lo = 0, hi = (int64_t)0xfffffffeLL;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (make_layout(g->n, tab, mid).total <= kStaticScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    const gsr_workspace ws{ctx->scratch, kStaticScratchBytes, lo};
    if (used) *used = ws;
    ctx->no_alloc = true;
    s = render_loss_grad_impl(ctx, g, views, &o, targets, ws, out, loss, gg, pg, stream);
    ctx->no_alloc = false;
    return s;
}

// Tile autotuner: every candidate is run once (checked against the pair
// capacity, one synchronisation), then timed over `reps` calls with HIP
// events; the fastest is kept for this input shape.
gsr_status gsr_autotune(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                        const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                        gsr_gaussian_grads *gg, gsr_pose_grads *pg, int32_t reps, int32_t *best_tile,
                        double *ms_per_call, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!g || !views || !opts || !best_tile || !ms_per_call) return fail(ctx, GSR_EINVAL, "autotune: NULL argument");
    if (reps < 1) return fail(ctx, GSR_EINVAL, "autotune: reps must be >= 1");
    static const int cand[kTuneCandidates][2] = {{16, 16}, {16, 8}, {8, 16}, {8, 8}, {32, 32}, {32, 16}, {16, 32}};
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s == GSR_OK) s = check_hip(ctx, hipEventCreate(&a), "hipEventCreate");
    if (s == GSR_OK) s = check_hip(ctx, hipEventCreate(&b), "hipEventCreate");
    double best = -1.0;
    int bw = 0, bh = 0;
    for (int k = 0; k < kTuneCandidates && s == GSR_OK; ++k) {
        gsr_options o = *opts;
        o.tile_w = cand[k][0];
        o.tile_h = cand[k][1];
        size_t need = 0;
        if (gsr_workspace_size(ctx, g->n, views, &o, ws.pair_capacity, &need) != GSR_OK || need > ws.bytes) continue;
        s = render_loss_grad_impl(ctx, g, views, &o, targets, ws, out, loss, gg, pg, stream);
        if (s != GSR_OK) break;
        int64_t m = 0, kk = 0;
        int32_t ovf = 0;
        s = gsr_read_counters(ctx, ws, stream, &m, &kk, &ovf);
        if (s != GSR_OK) break;
        if (ovf) continue;   // this tile needs more pairs than the workspace holds
        (void)hipEventRecord(a, st);
        for (int r = 0; r < reps && s == GSR_OK; ++r)
            s = render_loss_grad_impl(ctx, g, views, &o, targets, ws, out, loss, gg, pg, stream);
        (void)hipEventRecord(b, st);
        if (s != GSR_OK) break;
        s = check_hip(ctx, hipEventSynchronize(b), "hipEventSynchronize");
        float ms = 0.0f;
        if (s == GSR_OK) s = check_hip(ctx, hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
        const double per = (double)ms / reps;
        if (s == GSR_OK && (best < 0.0 || per < best)) {
            best = per;
            bw = o.tile_w;
            bh = o.tile_h;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s != GSR_OK) return s;
    if (best < 0.0) return fail(ctx, GSR_ECAPACITY, "autotune: no tile size fits the workspace's pair capacity");
    ctx->tuned[shape_key(g->n, views, opts->flags)] = {bw, bh};
    best_tile[0] = bw;
    best_tile[1] = bh;
    *ms_per_call = best;
    return GSR_OK;
}

gsr_status gsr_set_tile(gsr_ctx *ctx, int64_t n, const gsr_views *views, uint32_t flags, int32_t tile_w,
                        int32_t tile_h) {
    if (!ctx) return GSR_EINVAL;
    if (!views || !views->cams || views->n_views < 1 || views->n_views > GSR_MAX_VIEWS)
        return fail(ctx, GSR_EINVAL, "set_tile: invalid views");
    if (!tile_side_ok(tile_w) || !tile_side_ok(tile_h))
        return fail(ctx, GSR_EINVAL, "set_tile: each side must be 8, 16 or 32");
    ctx->tuned[shape_key(n, views, flags)] = {tile_w, tile_h};
    return GSR_OK;
}

// Graph capture of one fused call (forward, loss, backward): the sequence
// has no host synchronisation and no memset nodes, so it replays as is.
gsr_status gsr_graph_capture(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                             const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                             gsr_gaussian_grads *gg, gsr_pose_grads *pg, void *stream, int32_t *graph_id) {
    if (!ctx) return GSR_EINVAL;
    if (!graph_id) return fail(ctx, GSR_EINVAL, "graph_id must not be NULL");
    if (!stream) return fail(ctx, GSR_EINVAL, "graph capture needs a stream other than the null stream");
    if (opts && (opts->flags & GSR_SYNC))
        return fail(ctx, GSR_EINVAL, "GSR_SYNC waits on the host and cannot be captured into a graph");
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    // validate everything before the capture starts
    Call c;
    gsr_status s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (s != GSR_OK) return s;
    ctx->capturing = true;
    const gsr_status s_call = render_loss_grad_impl(ctx, g, views, opts, targets, ws, out, loss, gg, pg, stream);
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    s = check_hip(ctx, hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
    if (s_call != GSR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s_call;
    }
    if (s != GSR_OK) return s;
    hipGraphExec_t exec = nullptr;
    s = check_hip(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    (void)hipGraphDestroy(graph);
    if (s != GSR_OK) return s;
    const int32_t id = ctx->next_graph++;
    ctx->graphs[id] = exec;
    *graph_id = id;
    return GSR_OK;
}

gsr_status gsr_graph_launch(gsr_ctx *ctx, int32_t graph_id, void *stream) {
    if (!ctx) return GSR_EINVAL;
    auto it = ctx->graphs.find(graph_id);
    if (it == ctx->graphs.end()) return fail(ctx, GSR_EINVAL, "unknown graph id %d", graph_id);
    return check_hip(ctx, hipGraphLaunch(it->second, (hipStream_t)stream), "hipGraphLaunch");
}

gsr_status gsr_graph_destroy(gsr_ctx *ctx, int32_t graph_id) {
    if (!ctx) return GSR_EINVAL;
    auto it = ctx->graphs.find(graph_id);
    if (it == ctx->graphs.end()) return fail(ctx, GSR_EINVAL, "unknown graph id %d", graph_id);
    const gsr_status s = check_hip(ctx, hipGraphExecDestroy(it->second), "hipGraphExecDestroy");
    ctx->graphs.erase(it);
    return s;
}

gsr_status gsr_read_counters(gsr_ctx *ctx, gsr_workspace ws, void *stream, int64_t *n_visible, int64_t *n_pairs,
                             int32_t *overflow) {
    if (!ctx) return GSR_EINVAL;
    if (!ws.ptr) return fail(ctx, GSR_EINVAL, "workspace pointer is NULL");
    if (ws.bytes < sizeof(int64_t) * kNumCounters) return fail(ctx, GSR_EINVAL, "workspace too small");
    int64_t h[kNumCounters];
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    s = read_counters_sync(ctx, ws, (hipStream_t)stream, h);
    if (s != GSR_OK) return s;
    if (n_visible) *n_visible = h[kCntVisible];
    if (n_pairs) *n_pairs = h[kCntPairs];
    if (overflow) *overflow = (int32_t)(h[kCntOverflow] | h[kCntOverflowAny]);
    return GSR_OK;
}

gsr_status gsr_check_overflow(gsr_ctx *ctx, gsr_workspace ws, void *stream, int32_t *overflowed) {
    if (!ctx) return GSR_EINVAL;
    if (!overflowed) return fail(ctx, GSR_EINVAL, "overflowed must not be NULL");
    int64_t k = 0;
    const gsr_status s = gsr_read_counters(ctx, ws, stream, nullptr, &k, overflowed);
    if (s != GSR_OK) return s;
    if (*overflowed)
        return fail(ctx, GSR_ECAPACITY, "the pair capacity overflowed (%lld pairs needed by the last call)",
                    (long long)k);
    return GSR_OK;
}

gsr_status gsr_plan(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                    gsr_workspace ws, int64_t *pairs_needed, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!pairs_needed) return fail(ctx, GSR_EINVAL, "pairs_needed must not be NULL");
    gsr_status s = reject_capture(ctx, stream, "gsr_plan");
    if (s != GSR_OK) return s;
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    Call c;
    s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    enqueue_binning(c, views);
    s = check_hip(ctx, hipGetLastError(), "gsr_plan launch");
    if (s != GSR_OK) return s;
    int64_t h[kNumCounters];
    s = read_counters_sync(ctx, ws, c.st, h);
    if (s != GSR_OK) return s;
    *pairs_needed = h[kCntPairs];
    if (h[kCntOverflow] != 0)
        return fail(ctx, GSR_ECAPACITY, "%lld (Gaussian, tile) pairs needed, the workspace holds %lld",
                    (long long)h[kCntPairs], (long long)ws.pair_capacity);
    return GSR_OK;
}

gsr_status gsr_read_work(gsr_ctx *ctx, gsr_workspace ws, void *stream, int64_t *work) {
    if (!ctx) return GSR_EINVAL;
    if (!ws.ptr || !work) return fail(ctx, GSR_EINVAL, "workspace and work must not be NULL");
    if (ws.bytes < sizeof(int64_t) * kNumCounters) return fail(ctx, GSR_EINVAL, "workspace too small");
    int64_t h[kNumCounters];
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipMemcpyAsync(h, ws.ptr, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream),
                  "hipMemcpyAsync(counters)");
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    if (s != GSR_OK) return s;
    for (int k = 0; k < 5; ++k) work[k] = h[kCntEvalFwd + k];
    work[5] = h[kCntWorkItems];
    return GSR_OK;
}

gsr_status gsr_set_timing(gsr_ctx *ctx, int32_t enable) {
    if (!ctx) return GSR_EINVAL;
    ctx->timing = enable != 0;
    return GSR_OK;
}

gsr_status gsr_read_timing(gsr_ctx *ctx, double *ms, int64_t *launches) {
    if (!ctx) return GSR_EINVAL;
    if (!ms || !launches) return fail(ctx, GSR_EINVAL, "ms and launches must not be NULL");
    for (int k = 0; k < kNumStages; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    gsr_status status = GSR_OK;
    for (auto &r : ctx->recs) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess && status == GSR_OK) status = check_hip(ctx, e, "hipEventElapsedTime");
        ms[r.stage] += t;
        launches[r.stage] += 1;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    return status;
}

gsr_status gsr_debug_binning(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views, const gsr_options *opts,
                             gsr_workspace ws, int64_t max_rec, int64_t max_tiles, int64_t max_pairs,
                             uint32_t *rec_gid, float *rec_xy, float *rec_radius, float *rec_z, uint32_t *ranges,
                             uint32_t *pair_rec, void *stream) {
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    Call c;
    gsr_status s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    if (!rec_gid || !rec_xy || !rec_radius || !rec_z || !ranges || !pair_rec)
        return fail(ctx, GSR_EINVAL, "debug output pointers must not be NULL");
    s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    const Layout &L = c.L;
    const int64_t *counters = at<int64_t>(ws, L.counters);
    hipLaunchKernelGGL(c.pp.iso ? k_debug_records<true> : k_debug_records<false>, dim3(grid_for(L.vn, 256, 4096)),
                       dim3(256), 0, c.st, counters,
                       depth_sorted_gid(c), at<float4>(ws, L.rec), at<uint2>(ws, L.trect), max_rec, rec_gid, rec_xy,
                       rec_radius, rec_z, c.pp, at<ViewTable>(ws, L.views), at<PoseF64>(ws, L.poses));
    hipLaunchKernelGGL(k_debug_ranges, dim3(grid_for(L.T, 256, 4096)), dim3(256), 0, c.st, at<uint2>(ws, L.ranges),
                       std::min<int64_t>(L.T, max_tiles), reinterpret_cast<uint2 *>(ranges));
    hipLaunchKernelGGL(k_debug_copy_u32, dim3(grid_for(L.kcap, 256, 4096)), dim3(256), 0, c.st, pair_values(c),
                       counters, (int)kCntPairsUsed, max_pairs, pair_rec, (int64_t)0);
    return finish(c, "gsr_debug_binning launch");
}

gsr_status gsr_debug_pixel_state(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_views *views,
                                 const gsr_options *opts, gsr_workspace ws, float *t_final, uint32_t *n_last,
                                 uint32_t *hash, void *stream) {
    gsr_options o_res;
    if (opts && views && g) {
        o_res = resolve_tile(ctx, g->n, views, opts);
        opts = &o_res;
    }
    Call c;
    gsr_status s = prepare(ctx, g, views, opts, ws, stream, c);
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    const size_t bytes = 4 * (size_t)c.L.P;
    if (t_final) s = check_hip(ctx, hipMemcpyAsync(t_final, at<float>(ws, c.L.tfinal), bytes, hipMemcpyDeviceToDevice,
                                                   c.st), "copy t_final");
    if (s == GSR_OK && n_last)
        s = check_hip(ctx, hipMemcpyAsync(n_last, at<uint32_t>(ws, c.L.nlast), bytes, hipMemcpyDeviceToDevice, c.st),
                      "copy n_last");
    if (s == GSR_OK && hash)
        s = check_hip(ctx, hipMemcpyAsync(hash, at<uint32_t>(ws, c.L.phash), bytes, hipMemcpyDeviceToDevice, c.st),
                      "copy hash");
    return s;
}

gsr_status gsr_selftest(gsr_ctx *ctx, int32_t *failures, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!failures) return fail(ctx, GSR_EINVAL, "failures must not be NULL");
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, (hipStream_t)stream, (uint32_t *)failures, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_selftest, dim3(1), dim3(64), 0, (hipStream_t)stream, (int *)failures);
    return check_hip(ctx, hipGetLastError(), "gsr_selftest launch");
}


// ---------------------------------------------------------------------------
// optimisation steps
// ---------------------------------------------------------------------------

gsr_status gsr_pose_opt_init(gsr_ctx *ctx, int32_t n_views, const float *quat, const float *trans, double *state,
                             void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!quat || !trans || !state) return fail(ctx, GSR_EINVAL, "pose_opt_init: NULL argument");
    if (n_views < 1 || n_views > GSR_MAX_VIEWS)
        return fail(ctx, GSR_EINVAL, "pose_opt_init: n_views must be in [1, %d]", GSR_MAX_VIEWS);
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    hipLaunchKernelGGL(k_pose_opt_init, dim3(1), dim3(64), 0, (hipStream_t)stream, n_views, quat, trans,
                       reinterpret_cast<PoseOptState *>(state));
    return check_hip(ctx, hipGetLastError(), "gsr_pose_opt_init launch");
}

gsr_status gsr_pose_opt_step(gsr_ctx *ctx, int32_t n_views, const float *dq_c, const float *dc,
                             const gsr_pose_adam *hp, double *state, float *quat, float *trans, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!dq_c || !dc || !hp || !state || !quat || !trans) return fail(ctx, GSR_EINVAL, "pose_opt_step: NULL argument");
    if (n_views < 1 || n_views > GSR_MAX_VIEWS)
        return fail(ctx, GSR_EINVAL, "pose_opt_step: n_views must be in [1, %d]", GSR_MAX_VIEWS);
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    hipLaunchKernelGGL(k_pose_opt_step, dim3(1), dim3(64), 0, (hipStream_t)stream, n_views, dq_c, dc, *hp,
                       reinterpret_cast<PoseOptState *>(state), quat, trans, (const double *)nullptr,
                       (double *)nullptr);
    return check_hip(ctx, hipGetLastError(), "gsr_pose_opt_step launch");
}

gsr_status gsr_track(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views, float *quat,
                     float *trans, const gsr_options *opts, const gsr_targets *targets, gsr_workspace ws,
                     gsr_images out, double *loss, gsr_pose_grads *pg, const gsr_pose_adam *hp, double *state,
                     int32_t iters, double *loss_hist, void *stream) {
    return track_impl(ctx, g, cams, n_views, quat, trans, opts, targets, ws, out, loss, pg, hp, state, iters,
                      loss_hist, stream);
}

gsr_status gsr_track_capture(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                             float *quat, float *trans, const gsr_options *opts, const gsr_targets *targets,
                             gsr_workspace ws, gsr_images out, double *loss, gsr_pose_grads *pg,
                             const gsr_pose_adam *hp, double *state, int32_t iters, double *loss_hist, void *stream,
                             int32_t *graph_id) {
    if (!ctx) return GSR_EINVAL;
    if (!graph_id) return fail(ctx, GSR_EINVAL, "graph_id must not be NULL");
    if (!stream) return fail(ctx, GSR_EINVAL, "graph capture needs a stream other than the null stream");
    // validate before the capture starts (one render's worth of checks)
    if (!g || !cams || !opts || n_views < 1 || n_views > GSR_MAX_VIEWS)
        return fail(ctx, GSR_EINVAL, "track_capture: bad arguments");
    if (opts->flags & GSR_SYNC)
        return fail(ctx, GSR_EINVAL, "GSR_SYNC waits on the host and cannot be captured into a graph");
    {
        const gsr_views views{n_views, cams, quat, trans};
        gsr_options o = *opts;
        o.flags |= GSR_NO_GAUSS_GRADS;
        o = resolve_tile(ctx, g->n, &views, &o);
        Call c;
        const gsr_status sv = prepare(ctx, g, &views, &o, ws, stream, c);
        if (sv != GSR_OK) return sv;
    }
    hipStream_t st = (hipStream_t)stream;
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (s != GSR_OK) return s;
    ctx->capturing = true;
    const gsr_status s_call = track_impl(ctx, g, cams, n_views, quat, trans, opts, targets, ws, out, loss, pg, hp,
                                         state, iters, loss_hist, stream);
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    s = check_hip(ctx, hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
    if (s_call != GSR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s_call;
    }
    if (s != GSR_OK) return s;
    hipGraphExec_t exec = nullptr;
    s = check_hip(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    (void)hipGraphDestroy(graph);
    if (s != GSR_OK) return s;
    const int32_t id = ctx->next_graph++;
    ctx->graphs[id] = exec;
    *graph_id = id;
    return GSR_OK;
}


size_t gsr_map_state_size(int64_t n, int32_t isotropic) {
    if (n < 0) return 0;
    int64_t moff[kMapSegs], cnt[kMapSegs];
    return kMapHeader + 2 * sizeof(float) * (size_t)map_layout(n, isotropic != 0, moff, cnt);
}

gsr_status gsr_map_opt_init(gsr_ctx *ctx, int64_t n, int32_t isotropic, void *state, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!state || n < 0) return fail(ctx, GSR_EINVAL, "map_opt_init: NULL state or n < 0");
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    const int64_t words = (int64_t)(gsr_map_state_size(n, isotropic) / 4);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, 256, 65536)), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t *)state, words, 0u);
    return check_hip(ctx, hipGetLastError(), "gsr_map_opt_init launch");
}

gsr_status gsr_map_opt_step(gsr_ctx *ctx, gsr_gaussians_rw params, const gsr_gaussian_grads *grads,
                            int32_t isotropic, const gsr_map_adam *hp, void *state, void *stream) {
    if (!ctx) return GSR_EINVAL;
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    return map_step_impl(ctx, params, grads, isotropic != 0, hp, state, (hipStream_t)stream);
}

gsr_status gsr_map_iterate(gsr_ctx *ctx, gsr_gaussians_rw params, const gsr_views *views, const gsr_options *opts,
                           const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                           gsr_gaussian_grads *gg, const gsr_map_adam *hp, void *state, int32_t iters,
                           double *loss_hist, void *stream) {
    return map_iterate_impl(ctx, params, views, opts, targets, ws, out, loss, gg, hp, state, iters, loss_hist,
                            stream);
}

gsr_status gsr_map_capture(gsr_ctx *ctx, gsr_gaussians_rw params, const gsr_views *views, const gsr_options *opts,
                           const gsr_targets *targets, gsr_workspace ws, gsr_images out, double *loss,
                           gsr_gaussian_grads *gg, const gsr_map_adam *hp, void *state, int32_t iters,
                           double *loss_hist, void *stream, int32_t *graph_id) {
    if (!ctx) return GSR_EINVAL;
    if (!graph_id) return fail(ctx, GSR_EINVAL, "graph_id must not be NULL");
    if (!stream) return fail(ctx, GSR_EINVAL, "graph capture needs a stream other than the null stream");
    if (!views || !opts) return fail(ctx, GSR_EINVAL, "map_capture: views and opts must not be NULL");
    if (opts->flags & GSR_SYNC)
        return fail(ctx, GSR_EINVAL, "GSR_SYNC waits on the host and cannot be captured into a graph");
    {   // validate before the capture starts (one render's worth of checks)
        const gsr_gaussians g{params.n, params.means, params.quats, params.log_scales, params.opacity_logits,
                              params.rgb};
        gsr_options o = *opts;
        o.flags |= GSR_NO_POSE_GRADS;
        o = resolve_tile(ctx, g.n, views, &o);
        Call c;
        const gsr_status sv = prepare(ctx, &g, views, &o, ws, stream, c);
        if (sv != GSR_OK) return sv;
    }
    hipStream_t st = (hipStream_t)stream;
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    s = check_hip(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (s != GSR_OK) return s;
    ctx->capturing = true;
    const gsr_status s_call = map_iterate_impl(ctx, params, views, opts, targets, ws, out, loss, gg, hp, state, iters,
                                               loss_hist, stream);
    ctx->capturing = false;
    hipGraph_t graph = nullptr;
    s = check_hip(ctx, hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
    if (s_call != GSR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s_call;
    }
    if (s != GSR_OK) return s;
    hipGraphExec_t exec = nullptr;
    s = check_hip(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    (void)hipGraphDestroy(graph);
    if (s != GSR_OK) return s;
    const int32_t id = ctx->next_graph++;
    ctx->graphs[id] = exec;
    *graph_id = id;
    return GSR_OK;
}

size_t gsr_densify_work_size(int32_t width, int32_t height) {
    if (width < 1 || height < 1) return 0;
    const int64_t P = (int64_t)width * height;
    const int64_t nb = (P + kChunk - 1) / kChunk;
    return kSyncTickets + align_up(8 * (size_t)nb) + 256;   // tickets, look-back words, pose (12 doubles), error
}

gsr_status gsr_densify(gsr_ctx *ctx, gsr_camera cam, const float *quat, const float *trans, const float *rgb,
                       const float *depth, const float *sil, float sil_thresh, gsr_gaussians_rw out,
                       int32_t isotropic, int64_t offset, int64_t capacity, int64_t *n_new, void *work,
                       size_t work_bytes, void *stream) {
    if (!ctx) return GSR_EINVAL;
    if (!quat || !trans || !rgb || !depth || !n_new || !work)
        return fail(ctx, GSR_EINVAL, "densify: NULL argument (quat, trans, rgb, depth, n_new, work)");
    if (cam.width < 1 || cam.height < 1 || cam.width > 16384 || cam.height > 16384)
        return fail(ctx, GSR_EINVAL, "densify: image size %dx%d out of range", cam.width, cam.height);
    if (!(cam.fx > 0.0f) || !(cam.fy > 0.0f)) return fail(ctx, GSR_EINVAL, "densify: focal lengths must be > 0");
    if (offset < 0 || capacity < offset) return fail(ctx, GSR_EINVAL, "densify: need 0 <= offset <= capacity");
    const bool iso = isotropic != 0;
    if (capacity > offset && (!out.means || !out.log_scales || !out.opacity_logits || !out.rgb || (!iso && !out.quats)))
        return fail(ctx, GSR_EINVAL, "densify: output arrays must not be NULL");
    const size_t need = gsr_densify_work_size(cam.width, cam.height);
    if (work_bytes < need) return fail(ctx, GSR_EINVAL, "densify: work needs %zu bytes (got %zu)", need, work_bytes);
    gsr_status s = check_hip(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (s != GSR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int64_t P = (int64_t)cam.width * cam.height;
    char *w = static_cast<char *>(work);
    const size_t sync_bytes = kSyncTickets + align_up(8 * (size_t)((P + kChunk - 1) / kChunk));
    double *Rt = reinterpret_cast<double *>(w + sync_bytes);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((int64_t)(sync_bytes / 4), 256, 4096)), dim3(256), 0, st,
                       (uint32_t *)w, (int64_t)(sync_bytes / 4), 0u);
    hipLaunchKernelGGL(k_densify_setup, dim3(1), dim3(64), 0, st, quat, trans, Rt);
    int64_t *err = reinterpret_cast<int64_t *>(Rt + 12);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)err, (int64_t)2, 0u);
    SyncState ss{reinterpret_cast<uint32_t *>(w), reinterpret_cast<uint64_t *>(w + kSyncTickets), err};
    NewSink sink{cam, Rt, rgb, depth, P, offset, capacity, out.means, iso ? nullptr : out.quats, out.log_scales,
                 out.opacity_logits, out.rgb, iso};
    scan_exclusive(NewSrc{depth, sil, sil_thresh}, sink, nullptr, P, ss, 0u, TotalTo{n_new}, st);
    hipLaunchKernelGGL(k_densify_finish, dim3(1), dim3(64), 0, st, (const int64_t *)err, n_new);
    return check_hip(ctx, hipGetLastError(), "gsr_densify launch");
}
}  // extern "C"
