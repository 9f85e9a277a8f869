// Per-(view, Gaussian) projection and its chain rule, evaluated in FP64 on
// the GPU.  The work is per Gaussian (not per pixel), so FP64 costs nothing
// measurable here, and rounding the results once to FP32 keeps the depth keys
// and screen positions exact to the last bit that FP32 can hold.
//
// Forward (per view v, Gaussian i):
//   q^ = q/|q| -> R (Gaussian rotation), s = exp(log_s), o = sigmoid(logit)
//   Sigma = R diag(s^2) R^T            (Introduction, anisotropic covariance)
//   X = W mu + t                       (world to camera, W = R_cw)
//   J = d pi_m / dX at X               (pi_m: Visual Geometry Residual)
//   Sigma' = J W Sigma W^T J^T + b I   (Introduction, EWA projection; b = blur)
//   m = pi_m(X), depth d = X_z         (eq. 3 uses the camera-frame depth)
// The inverse of Sigma' is stored as a scaled Cholesky-type factor (l11, l21,
// l22) with  -(l11 dx + l21 dy)^2 - (l22 dy)^2 = log2(e) * (-1/2 d^T Sigma'^-1 d),
// so one exp2 gives the Gaussian of eq. 1 and the sum of squares cannot
// cancel for thin ellipses.
#pragma once

#include "gsr_common.hpp"

namespace gsr {

// sqrt(0.5 * log2(e))
constexpr double kLScale = 0.84932180028801907;
constexpr double kLn2 = 0.69314718055994531;

struct PoseF64 {
    double W[9];    // R_cw from the normalised pose quaternion
    double t[3];
};

__device__ __forceinline__ void quat_to_rot_f64(double w, double x, double y, double z, double *R) {
    const double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// dL/dq for an unnormalised quaternion q, given dL/dR of R(q/|q|).
__device__ __forceinline__ void rot_grad_to_quat_f64(const double *q, const double *G, double *gq) {
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    // dR/dw, dR/dx, dR/dy, dR/dz contracted with G (R as above, row-major)
    const double gw = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    const double gx = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                             2.0 * x * G[8]);
    const double gy = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                             2.0 * y * G[8]);
    const double gz = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0 * z * G[4] + y * G[5] +
                             x * G[6] + y * G[7]);
    const double dot = gw * w + gx * x + gy * y + gz * z;
    gq[0] = (gw - w * dot) / n;
    gq[1] = (gx - x * dot) / n;
    gq[2] = (gy - y * dot) / n;
    gq[3] = (gz - z * dot) / n;
}

struct GaussIn {
    double mu[3];
    double q[4];
    double ls[3];
    double logit;
};

// ISO: the isotropic parameterization (one log-scale per Gaussian, no
// rotation): quaternions are not read.
template <bool ISO>
__device__ __forceinline__ GaussIn load_gauss(const gsr_gaussians &g, int64_t i) {
    GaussIn p;
    for (int k = 0; k < 3; ++k) p.mu[k] = (double)g.means[3 * i + k];
    if constexpr (ISO) {
        const double l = (double)g.log_scales[i];
        p.ls[0] = p.ls[1] = p.ls[2] = l;
        p.q[0] = 1.0;
        p.q[1] = p.q[2] = p.q[3] = 0.0;
    } else {
        for (int k = 0; k < 4; ++k) p.q[k] = (double)g.quats[4 * i + k];
        for (int k = 0; k < 3; ++k) p.ls[k] = (double)g.log_scales[3 * i + k];
    }
    p.logit = (double)g.opacity_logits[i];
    return p;
}

// Everything the forward pass and the chain rule need about one projection.
struct Proj {
    bool visible;
    double X[3];
    double o;
    double s2[3];      // squared scales
    double Rg[9];      // Gaussian rotation
    double Sig[9];     // world covariance
    double M[9];       // W Sigma W^T
    double J[6];       // 2x3 Jacobian of pi_m
    double a, b, c;    // Sigma' (with blur)
    double det;
    double mx, my;
    double l11, l21, l22;
    float mxh, myh, mxl, myl, radius, z32;
    int32_t px0, px1, py0, py1;   // clamped pixel rectangle of the binning radius (inclusive)
};

// The view-independent part of a projection: opacity, squared scales,
// rotation and world covariance (the same FP64 operations whichever view).
struct GaussPre {
    double o;
    double qmax;   // 2 ln(255 o): the alpha >= 1/255 level of the exponent (used when 255 o > 1)
    double s2[3];
    double Rg[9];
    double Sig[9];
};

template <bool ISO>
__device__ __forceinline__ void prep_gauss(const GaussIn &p, GaussPre &g) {
    g.o = 1.0 / (1.0 + exp(-p.logit));
    g.qmax = 2.0 * log(255.0 * g.o);
    if constexpr (ISO) {
        g.s2[0] = g.s2[1] = g.s2[2] = exp(2.0 * p.ls[0]);
    } else {
        for (int k = 0; k < 3; ++k) g.s2[k] = exp(2.0 * p.ls[k]);
        quat_to_rot_f64(p.q[0], p.q[1], p.q[2], p.q[3], g.Rg);
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                const double v = g.Rg[3 * i] * g.s2[0] * g.Rg[3 * j] + g.Rg[3 * i + 1] * g.s2[1] * g.Rg[3 * j + 1] +
                                 g.Rg[3 * i + 2] * g.s2[2] * g.Rg[3 * j + 2];
                g.Sig[3 * i + j] = v;
                g.Sig[3 * j + i] = v;
            }
    }
}

// Project Gaussian p (view-independent part g) into view (pose, camera).
// Culls: z <= z_near, 255 o <= 1, det(Sigma') <= 0, non-finite values,
// rectangle outside the image.  FULL: the record's conic factor is formed
// (else only the culling decisions, the rectangle and the depth).  With ISO, Sigma = s^2 I, so
// M = W Sigma W^T = s^2 I (W is a rotation) and no rotation or covariance
// product is formed.
template <bool FULL, bool ISO>
__device__ __forceinline__ void project_pre(const GaussIn &p, const GaussPre &g, const PoseF64 &pose,
                                            const ViewInfo &cam, double z_near, double blur, Proj &r) {
    r.visible = false;
    const double *W = pose.W;
    for (int k = 0; k < 3; ++k)
        r.X[k] = W[3 * k] * p.mu[0] + W[3 * k + 1] * p.mu[1] + W[3 * k + 2] * p.mu[2] + pose.t[k];
    const double x = r.X[0], y = r.X[1], z = r.X[2];
    r.z32 = (float)z;
    if (!(z > z_near)) return;
    r.o = g.o;
    if (!(255.0 * r.o > 1.0)) return;
    for (int k = 0; k < 3; ++k) r.s2[k] = g.s2[k];
    if constexpr (ISO) {
        for (int k = 0; k < 9; ++k) r.M[k] = (k % 4 == 0) ? r.s2[0] : 0.0;
    } else {
        for (int k = 0; k < 9; ++k) {
            r.Rg[k] = g.Rg[k];
            r.Sig[k] = g.Sig[k];
        }
        // M = W Sigma W^T
        double WS[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                WS[3 * i + j] = W[3 * i] * r.Sig[j] + W[3 * i + 1] * r.Sig[3 + j] + W[3 * i + 2] * r.Sig[6 + j];
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                const double v = WS[3 * i] * W[3 * j] + WS[3 * i + 1] * W[3 * j + 1] + WS[3 * i + 2] * W[3 * j + 2];
                r.M[3 * i + j] = v;
                r.M[3 * j + i] = v;
            }
    }
    const double fx = cam.fx, fy = cam.fy;
    const double iz = 1.0 / z;
    r.J[0] = fx * iz; r.J[1] = 0.0; r.J[2] = -fx * x * iz * iz;
    r.J[3] = 0.0; r.J[4] = fy * iz; r.J[5] = -fy * y * iz * iz;
    // Sigma' = J M J^T + b I  (J has two zeros)
    const double *M = r.M;
    const double j0 = r.J[0], j2 = r.J[2], j4 = r.J[4], j5 = r.J[5];
    const double m0 = j0 * M[0] + j2 * M[6], m1 = j0 * M[1] + j2 * M[7], m2 = j0 * M[2] + j2 * M[8];
    const double n1 = j4 * M[4] + j5 * M[7], n2 = j4 * M[5] + j5 * M[8];
    r.a = m0 * j0 + m2 * j2 + blur;
    r.b = m1 * j4 + m2 * j5;
    r.c = n1 * j4 + n2 * j5 + blur;
    r.det = r.a * r.c - r.b * r.b;
    if (!(r.det > 0.0) || !isfinite(r.det)) return;
    r.mx = fx * x * iz + cam.cx;
    r.my = fy * y * iz + cam.cy;
    if (!isfinite(r.mx) || !isfinite(r.my)) return;
    // The conic's scaled Cholesky factor.  Without FULL (culling only) just
    // whether l11 and l21 are finite, which they are for c and det in
    // [1e-100, 1e200] and |b| <= 1e200 (c / det <= 1e300; c det >= 1e-200, or
    // it overflows and l21 = -0): only outside those bounds are they formed.
    const bool surely_finite = r.c >= 1e-100 && r.c <= 1e200 && r.det >= 1e-100 && fabs(r.b) <= 1e200;
    if (FULL || !surely_finite) {
        r.l11 = kLScale * sqrt(r.c / r.det);
        r.l21 = -kLScale * r.b / sqrt(r.c * r.det);
        r.l22 = kLScale / sqrt(r.c);
        if (!isfinite(r.l11) || !isfinite(r.l21)) return;
    }
    // Binning radius: a circle holding the whole alpha >= 1/255 ellipse
    // (d^T Sigma'^-1 d <= 2 ln(255 o)), widened by 2^-10 relatively and
    // absolutely so that FP32 rounding never clips a contributing pixel.
    const double qmax = g.qmax;
    const double mid = 0.5 * (r.a + r.c);
    const double lmax = mid + sqrt(fmax(mid * mid - r.det, 0.0));
    r.radius = (float)((1.0 + 0x1p-10) * sqrt(qmax * lmax) + 0x1p-10);
    r.mxh = (float)r.mx;
    r.myh = (float)r.my;
    r.mxl = (float)(r.mx - (double)r.mxh);
    r.myl = (float)(r.my - (double)r.myh);
    // pixel rectangle in FP32: [ceil(m - r), floor(m + r)] clamped to the image
    float xl = ceilf(r.mxh - r.radius), xh = floorf(r.mxh + r.radius);
    float yl = ceilf(r.myh - r.radius), yh = floorf(r.myh + r.radius);
    xl = fmaxf(xl, 0.0f);
    yl = fmaxf(yl, 0.0f);
    xh = fminf(xh, (float)(cam.W - 1));
    yh = fminf(yh, (float)(cam.H - 1));
    if (!(xl <= xh && yl <= yh)) return;
    r.px0 = (int32_t)xl; r.px1 = (int32_t)xh;
    r.py0 = (int32_t)yl; r.py1 = (int32_t)yh;
    r.visible = true;
}

template <bool FULL, bool ISO>
__device__ __forceinline__ void project(const GaussIn &p, const PoseF64 &pose, const ViewInfo &cam, double z_near,
                                        double blur, Proj &r) {
    GaussPre g;
    prep_gauss<ISO>(p, g);
    project_pre<FULL, ISO>(p, g, pose, cam, z_near, blur, r);
}

// Chain rule from the per-record 2D gradient (dmx, dmy, dl11, dl21, dl22, do,
// dr, dg, db, dz) to the raw parameters of Gaussian p and to the pose
// partials of this view: gX (dL/dX, which sums to dL/dt) and
// GW = dL/dW = gX mu^T + 2 dM W Sigma.
struct ParamGrad {
    double mu[3], q[4], ls[3], logit, rgb[3];
};

// GAUSS = false: only the pose partials (gX, GW) are formed, not the
// Gaussian's own parameter gradients.
template <bool ISO, bool GAUSS = true>
__device__ __forceinline__ void project_backward(const GaussIn &p, const PoseF64 &pose, const ViewInfo &cam,
                                                 const Proj &r, const float *g2, ParamGrad &pg, double gX[3],
                                                 double GW[9]) {
    const double *W = pose.W;
    for (int k = 0; k < 3; ++k) pg.rgb[k] += (double)g2[6 + k];
    pg.logit += (double)g2[5] * r.o * (1.0 - r.o);
    // (l11, l21, l22) -> Sigma' = (a, b, c)
    const double a = r.a, b = r.b, c = r.c, det = r.det;
    const double dl11 = g2[2], dl21 = g2[3], dl22 = g2[4];
    const double rs = kLScale / sqrt(c * det);   // = l11 / c = -l21 / b
    double da = dl11 * (-0.5 * r.l11 * c / det) + dl21 * (-0.5 * r.l21 * c / det);
    double db = dl11 * (r.l11 * b / det) + dl21 * (-rs * (1.0 + b * b / det));
    double dc = dl11 * r.l11 * (0.5 / c - 0.5 * a / det) + dl21 * r.l21 * (-0.5 / c - 0.5 * a / det) +
                dl22 * (-0.5 * r.l22 / c);
    // Sigma' = J M J^T: dM = J^T G J, dJ = 2 G J M with G = [[da, db/2], [db/2, dc]]
    const double G00 = da, G01 = 0.5 * db, G11 = dc;
    const double *J = r.J;
    double GJ[6];
    for (int k = 0; k < 3; ++k) {
        GJ[k] = G00 * J[k] + G01 * J[3 + k];
        GJ[3 + k] = G01 * J[k] + G11 * J[3 + k];
    }
    double dM[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dM[3 * i + j] = J[i] * GJ[j] + J[3 + i] * GJ[3 + j];
    double dJ[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            dJ[3 * i + j] = 2.0 * (GJ[3 * i] * r.M[j] + GJ[3 * i + 1] * r.M[3 + j] + GJ[3 * i + 2] * r.M[6 + j]);
    const double x = r.X[0], y = r.X[1], z = r.X[2];
    const double fx = cam.fx, fy = cam.fy;
    const double iz = 1.0 / z, iz2 = iz * iz, iz3 = iz2 * iz;
    const double dmx = g2[0], dmy = g2[1], dz = g2[9];
    gX[0] = dJ[2] * (-fx * iz2) + dmx * fx * iz;
    gX[1] = dJ[5] * (-fy * iz2) + dmy * fy * iz;
    gX[2] = dJ[0] * (-fx * iz2) + dJ[2] * (2.0 * fx * x * iz3) + dJ[4] * (-fy * iz2) + dJ[5] * (2.0 * fy * y * iz3) -
            dmx * fx * x * iz2 - dmy * fy * y * iz2 + dz;
    if constexpr (GAUSS)
        for (int k = 0; k < 3; ++k) pg.mu[k] += W[k] * gX[0] + W[3 + k] * gX[1] + W[6 + k] * gX[2];
    // M = W Sigma W^T: dSigma = W^T dM W; dW = 2 dM W Sigma (+ gX mu^T from X = W mu + t)
    if constexpr (ISO) {
        // Sigma = s^2 I: dW = gX mu^T + 2 s^2 dM W, and dL/dlog s = 2 s^2 tr(W^T dM W) = 2 s^2 tr(dM)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                GW[3 * i + j] = gX[i] * p.mu[j] + 2.0 * r.s2[0] *
                                                      (dM[3 * i] * W[j] + dM[3 * i + 1] * W[3 + j] + dM[3 * i + 2] * W[6 + j]);
        if constexpr (GAUSS) pg.ls[0] += 2.0 * r.s2[0] * (dM[0] + dM[4] + dM[8]);
        return;
    } else {
    double WSg[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            WSg[3 * i + j] = W[3 * i] * r.Sig[j] + W[3 * i + 1] * r.Sig[3 + j] + W[3 * i + 2] * r.Sig[6 + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            GW[3 * i + j] = gX[i] * p.mu[j] +
                            2.0 * (dM[3 * i] * WSg[j] + dM[3 * i + 1] * WSg[3 + j] + dM[3 * i + 2] * WSg[6 + j]);
    if constexpr (!GAUSS) return;
    double T1[9], dS[9];
    for (int i = 0; i < 3; ++i)   // T1 = W^T dM
        for (int j = 0; j < 3; ++j) T1[3 * i + j] = W[i] * dM[j] + W[3 + i] * dM[3 + j] + W[6 + i] * dM[6 + j];
    for (int i = 0; i < 3; ++i)   // dS = T1 W
        for (int j = 0; j < 3; ++j)
            dS[3 * i + j] = T1[3 * i] * W[j] + T1[3 * i + 1] * W[3 + j] + T1[3 * i + 2] * W[6 + j];
    // Sigma = Rg diag(s^2) Rg^T
    const double *Rg = r.Rg;
    double dSR[9];   // dS Rg
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dSR[3 * i + j] = dS[3 * i] * Rg[j] + dS[3 * i + 1] * Rg[3 + j] + dS[3 * i + 2] * Rg[6 + j];
    for (int k = 0; k < 3; ++k) {   // (Rg^T dS Rg)_kk
        const double v = Rg[k] * dSR[k] + Rg[3 + k] * dSR[3 + k] + Rg[6 + k] * dSR[6 + k];
        pg.ls[k] += 2.0 * r.s2[k] * v;
    }
    double dRg[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dRg[3 * i + j] = 2.0 * dSR[3 * i + j] * r.s2[j];
    double gq[4];
    rot_grad_to_quat_f64(p.q, dRg, gq);
    for (int k = 0; k < 4; ++k) pg.q[k] += gq[k];
    }
}

}  // namespace gsr
