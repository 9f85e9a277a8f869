// Optimisation steps around the rasteriser: the decoupled pose update of
// tracking, the Adam step of mapping, and the creation of Gaussians from an
// RGB-D frame.  All of them run on the device from device state, so a
// whole tracking or mapping loop can be enqueued or captured without a host
// round trip.
//
// Update rule (the paper prescribes gradient-based optimisation with rotation
// and translation handled separately, but no rule): Adam (Kingma & Ba 2015)
// per parameter block.  Pose: one step on the raw quaternion with dL/dq at a
// fixed camera centre and one on the centre C = -R^T t with dL/dC, then
// t = -R(q/|q|) C.
#pragma once

#include "gsr_common.hpp"
#include "gsr_project.hpp"
#include "gsr_scan_sort.hpp"

namespace gsr {

// ---------------------------------------------------------------------------
// pose
// ---------------------------------------------------------------------------

// Per-view optimiser state (FP64): q 4, C 3, m_q 4, v_q 4, m_C 3, v_C 3, step,
// and beta1^step, beta2^step (the bias corrections' powers, kept as running
// products).
struct PoseOptState {
    double q[4], C[3], mq[4], vq[4], mc[3], vc[3], step, b1p, b2p;
};
static_assert(sizeof(PoseOptState) == GSR_POSE_STATE_DOUBLES * sizeof(double), "pose state layout");

// (contraction off: the fused tracking step and the separate step kernel
// then round alike wherever the compiler inlines them)
__device__ __forceinline__ double adam_update(double &x, double g, double &m, double &v, double lr, double b1, double b2,
                                              double eps, double c1, double c2) {
#pragma clang fp contract(off)
    m = b1 * m + (1.0 - b1) * g;
    v = b2 * v + (1.0 - b2) * g * g;
    const double m_hat = m / c1, v_hat = v / c2;
    x = x - lr * m_hat / (sqrt(v_hat) + eps);
    return x;
}

__global__ void k_pose_opt_init(int V, const float *__restrict__ quat, const float *__restrict__ trans,
                                PoseOptState *__restrict__ st) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    PoseOptState s;
    for (int k = 0; k < 4; ++k) s.q[k] = (double)quat[4 * v + k];
    double R[9];
    quat_to_rot_f64(s.q[0], s.q[1], s.q[2], s.q[3], R);
    for (int k = 0; k < 3; ++k)   // C = -R^T t
        s.C[k] = -(R[k] * (double)trans[3 * v] + R[3 + k] * (double)trans[3 * v + 1] + R[6 + k] * (double)trans[3 * v + 2]);
    for (int k = 0; k < 4; ++k) s.mq[k] = s.vq[k] = 0.0;
    for (int k = 0; k < 3; ++k) s.mc[k] = s.vc[k] = 0.0;
    s.step = 0.0;
    s.b1p = s.b2p = 1.0;
    st[v] = s;
}

// One decoupled Adam step of view v from its gradients (dL/dq | C, dL/dC);
// writes the pose the next render reads (FP32).
// s: the view's state as read from st[v] (the caller may read it early).
__device__ __forceinline__ void pose_adam_apply(int v, const double dq_c[4], const double dc[3], const gsr_pose_adam &hp,
                                                PoseOptState s, PoseOptState *__restrict__ st,
                                                float *__restrict__ quat, float *__restrict__ trans) {
#pragma clang fp contract(off)
    s.step += 1.0;
    const double b1 = hp.beta1, b2 = hp.beta2, eps = hp.eps;
    s.b1p *= b1;
    s.b2p *= b2;
    const double c1 = 1.0 - s.b1p, c2 = 1.0 - s.b2p;
    for (int k = 0; k < 4; ++k) adam_update(s.q[k], dq_c[k], s.mq[k], s.vq[k], (double)hp.lr_rot, b1, b2, eps, c1, c2);
    for (int k = 0; k < 3; ++k) adam_update(s.C[k], dc[k], s.mc[k], s.vc[k], (double)hp.lr_pos, b1, b2, eps, c1, c2);
    st[v] = s;
    double R[9];
    quat_to_rot_f64(s.q[0], s.q[1], s.q[2], s.q[3], R);
    for (int k = 0; k < 4; ++k) quat[4 * v + k] = (float)s.q[k];
    for (int k = 0; k < 3; ++k)   // t = -R C
        trans[3 * v + k] = (float)(-(R[3 * k] * s.C[0] + R[3 * k + 1] * s.C[1] + R[3 * k + 2] * s.C[2]));
}

// One decoupled Adam step per view from the gradient arrays; if hist is set,
// also copies the view's loss into it.
__global__ void k_pose_opt_step(int V, const float *__restrict__ dq_c, const float *__restrict__ dc,
                                gsr_pose_adam hp, PoseOptState *__restrict__ st, float *__restrict__ quat,
                                float *__restrict__ trans, const double *__restrict__ loss, double *__restrict__ hist) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    double gq[4], gc[3];
    for (int k = 0; k < 4; ++k) gq[k] = (double)dq_c[4 * v + k];
    for (int k = 0; k < 3; ++k) gc[k] = (double)dc[3 * v + k];
    pose_adam_apply(v, gq, gc, hp, st[v], st, quat, trans);
    if (hist) hist[v] = loss[v];
}

// ---------------------------------------------------------------------------
// map: Adam over the raw parameter arrays
// ---------------------------------------------------------------------------

constexpr int kMapSegs = 5;          // means, quats, log_scales, opacity_logits, rgb
constexpr size_t kMapAlign = 64;     // floats: every moment segment starts 256-byte aligned
constexpr size_t kMapHeader = 256;   // bytes: step count and bias factors

struct MapSeg {
    float *x;
    const float *g;
    int64_t count;   // floats
    int64_t moff;    // offset of the segment in the moment arrays (floats)
    float lr;
};
struct MapSegs {
    MapSeg s[kMapSegs];
};

struct MapHeader {
    int32_t step;
    float c1, c2;   // 1 / (1 - beta^step)
    int32_t pad;
};

__global__ void k_map_opt_begin(MapHeader *h, float b1, float b2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int k = h->step + 1;
    h->step = k;
    h->c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)k)));
    h->c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)k)));
}

// blockIdx.y = segment; four floats a thread (float4 where the segment allows).
__global__ __launch_bounds__(256) void k_map_opt_step(MapSegs segs, float *__restrict__ m, float *__restrict__ v,
                                                      const MapHeader *__restrict__ h, float b1, float b2, float eps) {
    const MapSeg sg = segs.s[blockIdx.y];
    if (!sg.x || sg.count == 0) return;
    const float c1 = h->c1, c2 = h->c2;
    float *ms = m + sg.moff, *vs = v + sg.moff;
    const bool vec = ((reinterpret_cast<uintptr_t>(sg.x) | reinterpret_cast<uintptr_t>(sg.g)) & 15u) == 0;
    const int64_t n4 = vec ? sg.count / 4 : 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        float4 x = reinterpret_cast<float4 *>(sg.x)[i];
        const float4 g = reinterpret_cast<const float4 *>(sg.g)[i];
        float4 mm = reinterpret_cast<float4 *>(ms)[i];
        float4 vv = reinterpret_cast<float4 *>(vs)[i];
        float *xp = &x.x, *mp = &mm.x, *vp = &vv.x;
        const float *gp = &g.x;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            mp[k] = b1 * mp[k] + (1.0f - b1) * gp[k];
            vp[k] = b2 * vp[k] + (1.0f - b2) * gp[k] * gp[k];
            xp[k] = xp[k] - sg.lr * (mp[k] * c1) / (sqrtf(vp[k] * c2) + eps);
        }
        reinterpret_cast<float4 *>(sg.x)[i] = x;
        reinterpret_cast<float4 *>(ms)[i] = mm;
        reinterpret_cast<float4 *>(vs)[i] = vv;
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sg.count; i += stride) {
        const float g = sg.g[i];
        const float mm = b1 * ms[i] + (1.0f - b1) * g;
        const float vv = b2 * vs[i] + (1.0f - b2) * g * g;
        sg.x[i] = sg.x[i] - sg.lr * (mm * c1) / (sqrtf(vv * c2) + eps);
        ms[i] = mm;
        vs[i] = vv;
    }
}

// ---------------------------------------------------------------------------
// new Gaussians from an RGB-D frame (raster order, compacted by a scan)
// ---------------------------------------------------------------------------

struct NewSrc {   // 1 for a pixel that gets a Gaussian
    const float *depth, *sil;
    float thresh;
    __device__ uint32_t operator()(int64_t i) const {
        return (depth[i] > 0.0f && (!sil || sil[i] < thresh)) ? 1u : 0u;
    }
};

// Pose of the frame in FP64, [R (9), t (3)], for the sink.
__global__ void k_densify_setup(const float *__restrict__ quat, const float *__restrict__ trans, double *Rt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    quat_to_rot_f64((double)quat[0], (double)quat[1], (double)quat[2], (double)quat[3], Rt);
    for (int k = 0; k < 3; ++k) Rt[9 + k] = (double)trans[k];
}

// A scan wait that gave up (never expected) turns the count into -1.
__global__ void k_densify_finish(const int64_t *err, int64_t *n_new) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *err != 0) *n_new = -1;
}

struct NewSink {   // writes the Gaussian of pixel i at row offset + prefix
    gsr_camera cam;
    const double *Rt;
    const float *rgb, *depth;
    int64_t P, offset, capacity;
    float *means, *quats, *log_scales, *opacity, *col;
    bool iso;
    __device__ void operator()(int64_t i, uint32_t pre, uint32_t flag) const {
        if (!flag) return;
        const int64_t o = offset + (int64_t)pre;
        if (o >= capacity) return;   // the count still reports it
        const double *R = Rt, *t = Rt + 9;
        const double D = (double)depth[i];
        const double u = (double)(i % cam.width), w = (double)(i / cam.width);
        const double Xc[3] = {(u - (double)cam.cx) * D / (double)cam.fx, (w - (double)cam.cy) * D / (double)cam.fy, D};
        const double d[3] = {Xc[0] - t[0], Xc[1] - t[1], Xc[2] - t[2]};
        for (int k = 0; k < 3; ++k)   // mu = R^T (X_c - t)
            means[3 * o + k] = (float)(R[k] * d[0] + R[3 + k] * d[1] + R[6 + k] * d[2]);
        if (quats) {
            quats[4 * o] = 1.0f;
            quats[4 * o + 1] = quats[4 * o + 2] = quats[4 * o + 3] = 0.0f;
        }
        const float ls = (float)log(D / (0.5 * ((double)cam.fx + (double)cam.fy)));
        if (iso) {
            log_scales[o] = ls;
        } else {
            for (int k = 0; k < 3; ++k) log_scales[3 * o + k] = ls;
        }
        opacity[o] = 0.0f;   // sigmoid(0) = 0.5
        for (int c = 0; c < 3; ++c) col[3 * o + c] = rgb[(int64_t)c * P + i];
    }
};

}  // namespace gsr
