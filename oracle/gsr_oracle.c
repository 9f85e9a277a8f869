/*
 * gsr_oracle.c -- plain FP64 CPU oracle for the differentiable Gaussian
 * rasteriser (renders RGB, depth and silhouette; loss; gradients to the
 * Gaussians and to the camera pose).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * What it computes, and where the paper defines it
 *   - Gaussian (eq. 1) generalised to the anisotropic form whose covariance
 *     is R S S^T R^T (Introduction, commented formula) with S = diag(exp(log_s)).
 *   - Projection of the covariance to the image, Sigma' = J W Sigma W^T J^T
 *     (Introduction, commented formula) with W the world-to-camera rotation
 *     and J the Jacobian of the pinhole map pi_m (Preliminaries, Visual
 *     Geometry Residual), evaluated at the camera-frame mean.
 *   - alpha compositing of colour (eq. 2), depth (eq. 3) and silhouette
 *     (eq. 4) over the Gaussians sorted front to back, with the usual
 *     cut-offs: alpha = min(0.99, o G), skip alpha < 1/255, stop before a
 *     Gaussian that would take transmittance below 1e-4.
 *   - The combined photometric + depth + silhouette (+ depth prior) L1 loss
 *     (Abstract; Proposed Approach, Pose Estimation; depth priors in the
 *     Abstract and Conclusions), and its exact derivative by the chain rule.
 *   - Pose gradients in both parameterisations: (q, t) and the decoupled
 *     (q with camera centre C fixed, C) used by the rotation-translation
 *     decoupled update (Proposed Approach, Pose Estimation).
 *
 * Everything is evaluated pixel by pixel over every Gaussian (the plain
 * definition); there are no tiles.  The only speed-up is a per-row list of
 * the Gaussians whose exact alpha >= 1/255 bounding box covers that row,
 * kept in depth order, which does not change any result.
 *
 * Readings of the paper that this file fixes are listed next to the code
 * that uses them (pixel centres at integer coordinates, sigmoid opacity,
 * exp log-scales, (w,x,y,z) quaternions, black background, 0.3 px^2 screen
 * blur, depth key = camera-frame z rounded to float32, ties by index).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_ALPHA_MAX 0.99
#define OR_T_MIN 1e-4

typedef struct {
    int64_t n;
    const double *means, *quats, *log_scales, *opacity_logits, *rgb;
    int32_t isotropic;
    int32_t n_views;
    const int32_t *width, *height;
    const double *fx, *fy, *cx, *cy;
    const double *pose_q, *pose_t;  /* [V,4] w2c quaternion (w,x,y,z), [V,3] */
    double z_near, blur2d;
    double w_rgb, w_depth, w_sil, w_prior, sil_mask_thresh;
    /* targets, concatenated over views; NULL t_rgb means "no loss" */
    const double *t_rgb, *t_depth, *t_sil, *t_prior, *t_weight;
    const uint8_t *pixel_mask;      /* NULL = every pixel */
    double margin;                  /* relative margin that flags a decision as ambiguous */
    int32_t mask_ambiguous;         /* zero the loss weight at ambiguous pixels */
    int32_t want_grads;
    int32_t n_threads;
    double res_margin;              /* relative margin that flags a residual sign as ambiguous */
} or_in;

typedef struct {
    double *rgb, *depth, *sil, *t_final;   /* [3*sumP] planar per view, [sumP] ... */
    int32_t *n_contrib;                    /* contributing Gaussians per pixel */
    uint8_t *ambiguous;                    /* per pixel */
    double *loss;                          /* [V] */
    double *g_means, *g_quats, *g_log_scales, *g_opacity, *g_rgb;
    double *g_q_t, *g_t, *g_q_c, *g_c;     /* [V,4],[V,3],[V,4],[V,3] */
    uint64_t *decision_hash;               /* [V] */
    double *grad2d;                        /* optional [V,N,10] */
    /* the two kinds of ambiguity, per pixel (NULL = not wanted):
     *   decision_amb: an alpha, clamp or transmittance decision within the
     *     margin of its threshold, so the image itself may differ between
     *     precisions;
     *   residual_amb: the sign of a weighted L1 residual, or the tracking
     *     mask [S > thresh], within its margin: the image is well defined
     *     there, only the loss derivative's sign may differ.
     * `ambiguous` is their union. */
    uint8_t *decision_amb, *residual_amb;
} or_out;

/* per (view, Gaussian) projection */
typedef struct {
    int visible;
    double X[3];          /* camera-frame mean */
    float z32;            /* sort key */
    double m[2];          /* projected mean (pixels) */
    double cov[3];        /* Sigma' = (a, b, c) incl. the screen blur */
    double con[3];        /* its inverse (A, B, C) */
    double o;             /* opacity */
    double ex, ey;        /* half extents of the alpha >= 1/255 ellipse */
    double radius;        /* circumscribed screen radius used for binning */
    int32_t rect[4];      /* x_lo, x_hi, y_lo, y_hi pixel rectangle (inclusive) */
    double Rg[9], s[3];   /* Gaussian rotation and scales */
    double Sig[9];        /* world covariance */
    double M[9];          /* W Sigma W^T */
    double J[6];          /* 2x3 Jacobian of pi_m */
} or_proj;

/* ------------------------------------------------------------------------ */
/* small dense helpers (3x3 row-major)                                       */
/* ------------------------------------------------------------------------ */
static void mat3_mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}
static void mat3_mul_bt(const double *A, const double *B, double *C) { /* A B^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * j + k];
            C[3 * i + j] = s;
        }
}
static void mat3_mul_at(const double *A, const double *B, double *C) { /* A^T B */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * k + i] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

/* Unit quaternion (w,x,y,z) to rotation matrix.  The quaternion is first
 * normalised (reading: parameters are unconstrained, the rotation uses q/|q|). */
static void quat_to_rot(const double *q_raw, double *R, double *qn) {
    double nrm = sqrt(q_raw[0] * q_raw[0] + q_raw[1] * q_raw[1] + q_raw[2] * q_raw[2] + q_raw[3] * q_raw[3]);
    double w = q_raw[0] / nrm, x = q_raw[1] / nrm, y = q_raw[2] / nrm, z = q_raw[3] / nrm;
    if (qn) { qn[0] = w; qn[1] = x; qn[2] = y; qn[3] = z; }
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* dL/dq_raw from dL/dR, through R(qhat) and qhat = q/|q|. */
static void rot_grad_to_quat(const double *q_raw, const double *G, double *gq) {
    double nrm = sqrt(q_raw[0] * q_raw[0] + q_raw[1] * q_raw[1] + q_raw[2] * q_raw[2] + q_raw[3] * q_raw[3]);
    double w = q_raw[0] / nrm, x = q_raw[1] / nrm, y = q_raw[2] / nrm, z = q_raw[3] / nrm;
    /* partial derivatives of the nine entries of R with respect to w, x, y, z */
    const double dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    const double dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    const double dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    const double dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    double g[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k) {
        g[0] += G[k] * dw[k]; g[1] += G[k] * dx[k]; g[2] += G[k] * dy[k]; g[3] += G[k] * dz[k];
    }
    double qh[4] = {w, x, y, z};
    double dot = g[0] * w + g[1] * x + g[2] * y + g[3] * z;
    for (int k = 0; k < 4; ++k) gq[k] = (g[k] - qh[k] * dot) / nrm;
}

/* ------------------------------------------------------------------------ */
/* projection of one Gaussian into one view                                  */
/* ------------------------------------------------------------------------ */
static void project_one(const or_in *in, int v, int64_t i, const double *W, const double *t, or_proj *p) {
    memset(p, 0, sizeof(*p));
    const double *mu = in->means + 3 * i;
    /* camera-frame mean: X_c = R_cw mu + t_cw (pose as in the reprojection residual) */
    for (int r = 0; r < 3; ++r) p->X[r] = W[3 * r] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + t[r];
    const double x = p->X[0], y = p->X[1], z = p->X[2];
    p->z32 = (float)z;  /* reading: depth key = camera-frame z rounded to float32 */
    if (!(z > in->z_near)) return;                        /* near-plane cull */
    /* opacity o in [0,1] from a logit (reading) */
    p->o = 1.0 / (1.0 + exp(-in->opacity_logits[i]));
    if (!(255.0 * p->o > 1.0)) return;                    /* alpha <= o < 1/255 everywhere */
    /* scales from log-scales; isotropic uses one scale for all axes (eq. 1's radius) */
    for (int k = 0; k < 3; ++k) p->s[k] = exp(in->isotropic ? in->log_scales[i] : in->log_scales[3 * i + k]);
    quat_to_rot(in->quats + 4 * i, p->Rg, NULL);
    /* Sigma = R diag(s^2) R^T */
    double RD[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) RD[3 * r + c] = p->Rg[3 * r + c] * p->s[c] * p->s[c];
    mat3_mul_bt(RD, p->Rg, p->Sig);
    /* M = W Sigma W^T */
    double WS[9];
    mat3_mul(W, p->Sig, WS);
    mat3_mul_bt(WS, W, p->M);
    /* J = d pi_m / d X at the mean */
    const double fx = in->fx[v], fy = in->fy[v];
    p->J[0] = fx / z; p->J[1] = 0.0;    p->J[2] = -fx * x / (z * z);
    p->J[3] = 0.0;    p->J[4] = fy / z; p->J[5] = -fy * y / (z * z);
    /* Sigma' = J M J^T + blur I */
    double JM[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            JM[3 * r + c] = p->J[3 * r] * p->M[c] + p->J[3 * r + 1] * p->M[3 + c] + p->J[3 * r + 2] * p->M[6 + c];
    double a = JM[0] * p->J[0] + JM[1] * p->J[1] + JM[2] * p->J[2];
    double b = JM[0] * p->J[3] + JM[1] * p->J[4] + JM[2] * p->J[5];
    double c = JM[3] * p->J[3] + JM[4] * p->J[4] + JM[5] * p->J[5];
    a += in->blur2d;
    c += in->blur2d;
    p->cov[0] = a; p->cov[1] = b; p->cov[2] = c;
    double det = a * c - b * b;
    if (!(det > 0.0) || !isfinite(det)) return;
    p->con[0] = c / det; p->con[1] = -b / det; p->con[2] = a / det;
    /* mean: pi_m(X_c) = (fx X/Z + cx, fy Y/Z + cy); pixel (u,v) sits at (u,v) */
    p->m[0] = fx * x / z + in->cx[v];
    p->m[1] = fy * y / z + in->cy[v];
    /* alpha >= 1/255  <=>  d^T Sigma'^-1 d <= qmax */
    double qmax = 2.0 * log(255.0 * p->o);
    p->ex = sqrt(qmax * a) * (1.0 + 1e-9) + 1e-9;
    p->ey = sqrt(qmax * c) * (1.0 + 1e-9) + 1e-9;
    /* binning radius: circle around the mean that holds the ellipse above, widened by 2^-10 */
    double mid = 0.5 * (a + c);
    double lmax = mid + sqrt(fmax(mid * mid - det, 0.0));
    p->radius = (1.0 + 0x1p-10) * sqrt(qmax * lmax) + 0x1p-10;
    const int Wd = in->width[v], Hd = in->height[v];
    double xl = ceil(p->m[0] - p->radius), xh = floor(p->m[0] + p->radius);
    double yl = ceil(p->m[1] - p->radius), yh = floor(p->m[1] + p->radius);
    if (xl < 0) xl = 0;
    if (yl < 0) yl = 0;
    if (xh > Wd - 1) xh = Wd - 1;
    if (yh > Hd - 1) yh = Hd - 1;
    if (!(xl <= xh && yl <= yh)) return;
    p->rect[0] = (int32_t)xl; p->rect[1] = (int32_t)xh; p->rect[2] = (int32_t)yl; p->rect[3] = (int32_t)yh;
    if (!isfinite(p->m[0]) || !isfinite(p->m[1]) || !isfinite(p->con[0])) return;
    p->visible = 1;
}

/* depth order: (float32 depth, index) ascending */
typedef struct { float z; int64_t i; } or_key;
static int key_cmp(const void *A, const void *B) {
    const or_key *a = (const or_key *)A, *b = (const or_key *)B;
    if (a->z < b->z) return -1;
    if (a->z > b->z) return 1;
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

static inline uint64_t mix_hash(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

static inline double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* one contributing Gaussian at a pixel, kept for the backward pass */
typedef struct { int64_t k; double alpha, T, G, dx, dy; int clamped; } or_hit;

/* ------------------------------------------------------------------------ */
/* public: projection fields of one view, for tests and for binning checks   */
/* ------------------------------------------------------------------------ */
int oracle_project_view(const or_in *in, int v, int32_t *visible, double *mean2d, double *cov2d,
                        double *conic, double *opacity, double *radius, int32_t *rect, float *z32,
                        double *Xc) {
    double W[9], qn[4];
    quat_to_rot(in->pose_q + 4 * v, W, qn);
    const double *t = in->pose_t + 3 * v;
    for (int64_t i = 0; i < in->n; ++i) {
        or_proj p;
        project_one(in, v, i, W, t, &p);
        visible[i] = p.visible;
        mean2d[2 * i] = p.m[0]; mean2d[2 * i + 1] = p.m[1];
        for (int k = 0; k < 3; ++k) { cov2d[3 * i + k] = p.cov[k]; conic[3 * i + k] = p.con[k]; Xc[3 * i + k] = p.X[k]; }
        opacity[i] = p.o;
        radius[i] = p.radius;
        for (int k = 0; k < 4; ++k) rect[4 * i + k] = p.rect[k];
        z32[i] = p.z32;
    }
    return 0;
}

int oracle_quat_to_rot(const double *q, double *R) { quat_to_rot(q, R, NULL); return 0; }

/* ------------------------------------------------------------------------ */
/* public: render + loss + gradients                                         */
/* ------------------------------------------------------------------------ */
int oracle_run(const or_in *in, or_out *out) {
    const int64_t N = in->n;
    const int V = in->n_views;
    int64_t off = 0;
    if (out->g_means) {
        memset(out->g_means, 0, sizeof(double) * 3 * N);
        memset(out->g_quats, 0, sizeof(double) * 4 * N);
        memset(out->g_log_scales, 0, sizeof(double) * (in->isotropic ? 1 : 3) * N);
        memset(out->g_opacity, 0, sizeof(double) * N);
        memset(out->g_rgb, 0, sizeof(double) * 3 * N);
    }
    if (out->grad2d) memset(out->grad2d, 0, sizeof(double) * 10 * N * V);
#ifdef _OPENMP
    int nthr = in->n_threads > 0 ? in->n_threads : omp_get_max_threads();
#else
    int nthr = 1;
#endif

    for (int v = 0; v < V; ++v) {
        const int Wd = in->width[v], Hd = in->height[v];
        const int64_t P = (int64_t)Wd * Hd;
        if (in->pixel_mask) {   /* a view with no selected pixel contributes nothing: skip its work */
            int any = 0;
            for (int64_t p = 0; p < P && !any; ++p) any = in->pixel_mask[off + p] != 0;
            if (!any) {
                for (int64_t p = 0; p < P; ++p) {
                    if (out->rgb) { out->rgb[3 * off + p] = 0; out->rgb[3 * off + P + p] = 0; out->rgb[3 * off + 2 * P + p] = 0; }
                    if (out->depth) out->depth[off + p] = 0;
                    if (out->sil) out->sil[off + p] = 0;
                    if (out->t_final) out->t_final[off + p] = 1.0;
                    if (out->n_contrib) out->n_contrib[off + p] = 0;
                    if (out->ambiguous) out->ambiguous[off + p] = 0;
                    if (out->decision_amb) out->decision_amb[off + p] = 0;
                    if (out->residual_amb) out->residual_amb[off + p] = 0;
                }
                if (out->loss) out->loss[v] = 0.0;
                if (out->decision_hash) out->decision_hash[v] = 0;
                if (in->want_grads && in->t_rgb && out->g_q_t)
                    for (int k = 0; k < 4; ++k) { out->g_q_t[4 * v + k] = 0; out->g_q_c[4 * v + k] = 0; }
                if (in->want_grads && in->t_rgb && out->g_t)
                    for (int k = 0; k < 3; ++k) { out->g_t[3 * v + k] = 0; out->g_c[3 * v + k] = 0; }
                off += P;
                continue;
            }
        }
        double W[9];
        quat_to_rot(in->pose_q + 4 * v, W, NULL);
        const double *t = in->pose_t + 3 * v;

        /* 1. project every Gaussian */
        or_proj *proj = (or_proj *)malloc(sizeof(or_proj) * (size_t)(N > 0 ? N : 1));
        int64_t nvis = 0;
#pragma omp parallel for num_threads(nthr) schedule(static) reduction(+ : nvis)
        for (int64_t i = 0; i < N; ++i) {
            project_one(in, v, i, W, t, &proj[i]);
            nvis += proj[i].visible;
        }
        /* 2. depth order of the visible ones */
        or_key *keys = (or_key *)malloc(sizeof(or_key) * (size_t)(nvis > 0 ? nvis : 1));
        int64_t nk = 0;
        for (int64_t i = 0; i < N; ++i)
            if (proj[i].visible) { keys[nk].z = proj[i].z32; keys[nk].i = i; ++nk; }
        qsort(keys, (size_t)nk, sizeof(or_key), key_cmp);
        /* rank of each visible Gaussian in depth order (gradient buffers are indexed by it) */
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nk > 0 ? nk : 1));
        for (int64_t r = 0; r < nk; ++r) order[r] = keys[r].i;
        /* per-row candidate lists (ellipse bounding box covers the row), in depth order */
        int64_t *row_cnt = (int64_t *)calloc((size_t)Hd + 1, sizeof(int64_t));
        for (int64_t r = 0; r < nk; ++r) {
            const or_proj *p = &proj[order[r]];
            int y0 = (int)ceil(p->m[1] - p->ey), y1 = (int)floor(p->m[1] + p->ey);
            if (y0 < 0) y0 = 0;
            if (y1 > Hd - 1) y1 = Hd - 1;
            for (int y = y0; y <= y1; ++y) row_cnt[y + 1]++;
        }
        for (int y = 0; y < Hd; ++y) row_cnt[y + 1] += row_cnt[y];
        int64_t *row_list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(row_cnt[Hd] > 0 ? row_cnt[Hd] : 1));
        int64_t *row_fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Hd > 0 ? Hd : 1));
        for (int y = 0; y < Hd; ++y) row_fill[y] = row_cnt[y];
        for (int64_t r = 0; r < nk; ++r) {
            const or_proj *p = &proj[order[r]];
            int y0 = (int)ceil(p->m[1] - p->ey), y1 = (int)floor(p->m[1] + p->ey);
            if (y0 < 0) y0 = 0;
            if (y1 > Hd - 1) y1 = Hd - 1;
            for (int y = y0; y <= y1; ++y) row_list[row_fill[y]++] = r;
        }

        /* 3. per pixel: composite, loss, exact per-pixel gradient */
        const int want_g = in->want_grads && in->t_rgb != NULL;
        double *g2d_thr = NULL;   /* per thread [nk,10]: dm0 dm1 dA dB dC do dr dg db dz */
        if (want_g) g2d_thr = (double *)calloc((size_t)nthr * (size_t)(nk > 0 ? nk : 1) * 10, sizeof(double));
        double *loss_thr = (double *)calloc((size_t)nthr, sizeof(double));
        uint64_t *hash_row = (uint64_t *)calloc((size_t)Hd + 1, sizeof(uint64_t));
        const double inv_P = 1.0 / (double)(P > 0 ? P : 1);

#pragma omp parallel num_threads(nthr)
        {
#ifdef _OPENMP
            const int tid = omp_get_thread_num();
#else
            const int tid = 0;
#endif
            or_hit *hits = (or_hit *)malloc(sizeof(or_hit) * 4096);
            int64_t hcap = 4096;
#pragma omp for schedule(dynamic, 1)
            for (int py = 0; py < Hd; ++py) {
                uint64_t hrow = 1469598103934665603ull;
                for (int px = 0; px < Wd; ++px) {
                    const int64_t pix = (int64_t)py * Wd + px;
                    const int64_t gp = off + pix;
                    double acc[5] = {0, 0, 0, 0, 0};  /* r, g, b, depth, silhouette */
                    double T = 1.0;
                    int amb = 0;     /* decisions of the compositing */
                    int amb_r = 0;   /* residual signs and the tracking mask */
                    int64_t nh = 0;
                    if (in->pixel_mask && !in->pixel_mask[gp]) {
                        if (out->rgb) { out->rgb[3 * off + pix] = 0; out->rgb[3 * off + P + pix] = 0; out->rgb[3 * off + 2 * P + pix] = 0; }
                        if (out->depth) out->depth[gp] = 0;
                        if (out->sil) out->sil[gp] = 0;
                        if (out->t_final) out->t_final[gp] = 1.0;
                        if (out->n_contrib) out->n_contrib[gp] = 0;
                        if (out->ambiguous) out->ambiguous[gp] = 0;
                        if (out->decision_amb) out->decision_amb[gp] = 0;
                        if (out->residual_amb) out->residual_amb[gp] = 0;
                        continue;
                    }
                    const double m = in->margin;
                    for (int64_t c = row_cnt[py]; c < row_cnt[py + 1]; ++c) {
                        const int64_t r = row_list[c];
                        const or_proj *p = &proj[order[r]];
                        const double dx = (double)px - p->m[0], dy = (double)py - p->m[1];
                        if (fabs(dx) > p->ex || fabs(dy) > p->ey) continue;  /* outside the ellipse box */
                        /* eq. 1 in its projected form: G = exp(-1/2 d^T Sigma'^-1 d) */
                        const double power = -0.5 * (p->con[0] * dx * dx + 2.0 * p->con[1] * dx * dy + p->con[2] * dy * dy);
                        const double G = exp(power);
                        const double og = p->o * G;
                        if (fabs(og - OR_ALPHA_MIN) <= m * OR_ALPHA_MIN) amb = 1;
                        if (og < OR_ALPHA_MIN) continue;                       /* skip faint */
                        if (fabs(og - OR_ALPHA_MAX) <= m * OR_ALPHA_MAX) amb = 1;
                        const int clamped = og > OR_ALPHA_MAX;
                        const double alpha = clamped ? OR_ALPHA_MAX : og;
                        const double Tn = T * (1.0 - alpha);
                        if (fabs(Tn - OR_T_MIN) <= m * OR_T_MIN) amb = 1;
                        if (Tn < OR_T_MIN) { hrow = mix_hash(hrow, 0xfffffffull); break; }  /* stop, not blended */
                        const double w = alpha * T;
                        const double *col = in->rgb + 3 * order[r];
                        acc[0] += col[0] * w; acc[1] += col[1] * w; acc[2] += col[2] * w;
                        acc[3] += p->X[2] * w;  /* eq. 3: d_i is the camera-frame depth */
                        acc[4] += w;            /* eq. 4 */
                        if (nh == hcap) { hcap *= 2; hits = (or_hit *)realloc(hits, sizeof(or_hit) * hcap); }
                        hits[nh].k = r; hits[nh].alpha = alpha; hits[nh].T = T; hits[nh].G = G;
                        hits[nh].dx = dx; hits[nh].dy = dy; hits[nh].clamped = clamped;
                        ++nh;
                        hrow = mix_hash(hrow, (uint64_t)order[r] * 2u + (uint64_t)clamped);
                        T = Tn;
                    }
                    hrow = mix_hash(hrow, (uint64_t)nh);
                    if (out->rgb) {
                        out->rgb[3 * off + pix] = acc[0];
                        out->rgb[3 * off + P + pix] = acc[1];
                        out->rgb[3 * off + 2 * P + pix] = acc[2];
                    }
                    if (out->depth) out->depth[gp] = acc[3];
                    if (out->sil) out->sil[gp] = acc[4];
                    if (out->t_final) out->t_final[gp] = T;
                    if (out->n_contrib) out->n_contrib[gp] = (int32_t)nh;
                    if (out->decision_amb) out->decision_amb[gp] = (uint8_t)amb;
                    if (!in->t_rgb) {
                        if (out->ambiguous) out->ambiguous[gp] = (uint8_t)amb;
                        if (out->residual_amb) out->residual_amb[gp] = 0;
                        continue;
                    }

                    /* loss at this pixel (reading of the combined loss: L1 terms, 1/P per view) */
                    double wgt = in->t_weight ? in->t_weight[gp] : 1.0;
                    const double trk = (in->sil_mask_thresh >= 0.0) ? (acc[4] > in->sil_mask_thresh ? 1.0 : 0.0) : 1.0;
                    const double dm = in->t_depth[gp] > 0.0 ? 1.0 : 0.0;
                    const double dpr = (in->t_prior && in->t_prior[gp] > 0.0) ? 1.0 : 0.0;
                    double tv[5];
                    tv[0] = in->t_rgb[3 * off + pix];
                    tv[1] = in->t_rgb[3 * off + P + pix];
                    tv[2] = in->t_rgb[3 * off + 2 * P + pix];
                    tv[3] = in->t_depth[gp];
                    tv[4] = in->t_sil ? in->t_sil[gp] : 0.0;
                    const double tpr = in->t_prior ? in->t_prior[gp] : 0.0;
                    double res[5];
                    for (int ch = 0; ch < 5; ++ch) res[ch] = acc[ch] - tv[ch];
                    const double rpr = acc[3] - tpr;
                    /* sign(residual) and the tracking mask are decisions too: flag
                     * the pixel when a residual that carries weight is within the
                     * relative margin of zero (but not both sides exactly zero) */
                    const double wch[5] = {trk * dm * in->w_rgb, trk * dm * in->w_rgb, trk * dm * in->w_rgb,
                                           trk * dm * in->w_depth, in->w_sil};
                    for (int ch = 0; ch < 5; ++ch)
                        if (wch[ch] != 0.0 && (acc[ch] != 0.0 || tv[ch] != 0.0) &&
                            fabs(res[ch]) <= in->res_margin * (fabs(acc[ch]) + fabs(tv[ch])))
                            amb_r = 1;
                    if (trk * dpr * in->w_prior != 0.0 && (acc[3] != 0.0 || tpr != 0.0) &&
                        fabs(rpr) <= in->res_margin * (fabs(acc[3]) + fabs(tpr)))
                        amb_r = 1;
                    if (in->sil_mask_thresh >= 0.0 &&
                        fabs(acc[4] - in->sil_mask_thresh) <= m * fmax(fabs(acc[4]), in->sil_mask_thresh))
                        amb_r = 1;
                    if (out->ambiguous) out->ambiguous[gp] = (uint8_t)(amb | amb_r);
                    if (out->residual_amb) out->residual_amb[gp] = (uint8_t)amb_r;
                    if (in->mask_ambiguous && (amb | amb_r)) wgt = 0.0;
                    if (wgt == 0.0) continue;
                    const double lp = wgt * inv_P *
                        (trk * dm * (in->w_rgb * (fabs(res[0]) + fabs(res[1]) + fabs(res[2])) + in->w_depth * fabs(res[3])) +
                         in->w_sil * fabs(res[4]) + trk * dpr * in->w_prior * fabs(rpr));
                    loss_thr[tid] += lp;
                    if (!want_g) continue;
                    double g[5];
                    g[0] = wgt * inv_P * trk * dm * in->w_rgb * sgn(res[0]);
                    g[1] = wgt * inv_P * trk * dm * in->w_rgb * sgn(res[1]);
                    g[2] = wgt * inv_P * trk * dm * in->w_rgb * sgn(res[2]);
                    g[3] = wgt * inv_P * (trk * dm * in->w_depth * sgn(res[3]) + trk * dpr * in->w_prior * sgn(rpr));
                    g[4] = wgt * inv_P * in->w_sil * sgn(res[4]);

                    /* exact derivative of eqs. 2-4 at this pixel:
                     * out_ch = sum_k f_k,ch a_k T_k, T_k = prod_{j<k}(1-a_j)
                     * d out_ch / d a_k = f_k,ch T_k - (sum_{j>k} f_j,ch a_j T_j) / (1 - a_k) */
                    double suffix[5] = {0, 0, 0, 0, 0};
                    double *g2 = g2d_thr + (size_t)tid * (size_t)nk * 10;
                    for (int64_t h = nh - 1; h >= 0; --h) {
                        const or_hit *e = &hits[h];
                        const or_proj *p = &proj[order[e->k]];
                        const double *col = in->rgb + 3 * order[e->k];
                        const double f[5] = {col[0], col[1], col[2], p->X[2], 1.0};
                        double dalpha = 0.0;
                        for (int ch = 0; ch < 5; ++ch)
                            dalpha += g[ch] * (f[ch] * e->T - suffix[ch] / (1.0 - e->alpha));
                        const double w = e->alpha * e->T;
                        for (int ch = 0; ch < 5; ++ch) suffix[ch] += f[ch] * w;
                        double *gg = g2 + 10 * e->k;
                        gg[6] += g[0] * w; gg[7] += g[1] * w; gg[8] += g[2] * w;
                        gg[9] += g[3] * w;                       /* through d_i = z (eq. 3) */
                        if (e->clamped) continue;                /* alpha = 0.99 is constant */
                        gg[5] += dalpha * e->G;                  /* d alpha / d o = G */
                        const double dpow = dalpha * e->alpha;   /* d alpha / d power = o G */
                        gg[0] += dpow * (p->con[0] * e->dx + p->con[1] * e->dy);  /* d power / d m_x */
                        gg[1] += dpow * (p->con[1] * e->dx + p->con[2] * e->dy);
                        gg[2] += dpow * (-0.5 * e->dx * e->dx);
                        gg[3] += dpow * (-e->dx * e->dy);
                        gg[4] += dpow * (-0.5 * e->dy * e->dy);
                    }
                }
                hash_row[py] = hrow;
            }
            free(hits);
        }
        double L = 0.0;
        for (int k = 0; k < nthr; ++k) L += loss_thr[k];
        if (out->loss) out->loss[v] = L;
        if (out->decision_hash) {
            uint64_t h = 1469598103934665603ull;
            for (int y = 0; y < Hd; ++y) h = mix_hash(h, hash_row[y]);
            out->decision_hash[v] = h;
        }

        /* 4. chain rule per Gaussian back to the raw parameters and the pose */
        if (want_g) {
            double GW[9] = {0}, gt[3] = {0, 0, 0};
            for (int64_t r = 0; r < nk; ++r) {
                const int64_t i = order[r];
                const or_proj *p = &proj[i];
                double d[10] = {0};
                for (int k = 0; k < nthr; ++k)
                    for (int c = 0; c < 10; ++c) d[c] += g2d_thr[((size_t)k * (size_t)nk + (size_t)r) * 10 + c];
                if (out->grad2d)
                    for (int c = 0; c < 10; ++c) out->grad2d[((size_t)v * (size_t)N + (size_t)i) * 10 + c] = d[c];
                /* colour and opacity */
                for (int c = 0; c < 3; ++c) out->g_rgb[3 * i + c] += d[6 + c];
                out->g_opacity[i] += d[5] * p->o * (1.0 - p->o);
                /* conic (A,B,C) = inverse of Sigma' (a,b,c) */
                const double a = p->cov[0], b = p->cov[1], c = p->cov[2];
                const double det = a * c - b * b, id2 = 1.0 / (det * det);
                const double dA = d[2], dB = d[3], dC = d[4];
                const double da = (dA * (-c * c) + dB * (b * c) + dC * (-b * b)) * id2;
                const double db = (dA * (2 * b * c) + dB * (-(a * c + b * b)) + dC * (2 * a * b)) * id2;
                const double dc = (dA * (-b * b) + dB * (a * b) + dC * (-a * a)) * id2;
                /* Sigma' = J M J^T:  dM = J^T G' J,  dJ = 2 G' J M  with G' symmetric */
                const double Gp[4] = {da, 0.5 * db, 0.5 * db, dc};
                double GJ[6];
                for (int rr = 0; rr < 2; ++rr)
                    for (int cc = 0; cc < 3; ++cc) GJ[3 * rr + cc] = Gp[2 * rr] * p->J[cc] + Gp[2 * rr + 1] * p->J[3 + cc];
                double dM[9];
                for (int rr = 0; rr < 3; ++rr)
                    for (int cc = 0; cc < 3; ++cc) dM[3 * rr + cc] = p->J[rr] * GJ[cc] + p->J[3 + rr] * GJ[3 + cc];
                double dJ[6];
                for (int rr = 0; rr < 2; ++rr)
                    for (int cc = 0; cc < 3; ++cc) {
                        double s = 0;
                        for (int k = 0; k < 3; ++k) s += GJ[3 * rr + k] * p->M[3 * k + cc];
                        dJ[3 * rr + cc] = 2.0 * s;
                    }
                /* camera-frame mean: through J, pi_m and the depth channel */
                const double x = p->X[0], y = p->X[1], z = p->X[2];
                const double fx = in->fx[v], fy = in->fy[v];
                double gX[3];
                gX[0] = dJ[2] * (-fx / (z * z)) + d[0] * fx / z;
                gX[1] = dJ[5] * (-fy / (z * z)) + d[1] * fy / z;
                gX[2] = dJ[0] * (-fx / (z * z)) + dJ[2] * (2.0 * fx * x / (z * z * z)) +
                        dJ[4] * (-fy / (z * z)) + dJ[5] * (2.0 * fy * y / (z * z * z)) -
                        d[0] * fx * x / (z * z) - d[1] * fy * y / (z * z) + d[9];
                /* X = W mu + t */
                const double *mu = in->means + 3 * i;
                for (int k = 0; k < 3; ++k)
                    out->g_means[3 * i + k] += W[k] * gX[0] + W[3 + k] * gX[1] + W[6 + k] * gX[2];
                for (int rr = 0; rr < 3; ++rr) {
                    gt[rr] += gX[rr];
                    for (int cc = 0; cc < 3; ++cc) GW[3 * rr + cc] += gX[rr] * mu[cc];
                }
                /* M = W Sigma W^T: dSigma = W^T dM W, dW += 2 dM W Sigma */
                double tmp[9], dSig[9], WSg[9], dMWS[9];
                mat3_mul_at(W, dM, tmp);
                mat3_mul(tmp, W, dSig);
                mat3_mul(W, p->Sig, WSg);
                mat3_mul(dM, WSg, dMWS);
                for (int k = 0; k < 9; ++k) GW[k] += 2.0 * dMWS[k];
                /* Sigma = Rg diag(s^2) Rg^T */
                double RtdS[9], RtdSR[9];
                mat3_mul_at(p->Rg, dSig, RtdS);
                mat3_mul(RtdS, p->Rg, RtdSR);
                if (in->isotropic) {
                    out->g_log_scales[i] += 2.0 * p->s[0] * p->s[0] * (RtdSR[0] + RtdSR[4] + RtdSR[8]);
                } else {
                    for (int k = 0; k < 3; ++k) out->g_log_scales[3 * i + k] += 2.0 * p->s[k] * p->s[k] * RtdSR[4 * k];
                }
                double dRg[9];
                for (int rr = 0; rr < 3; ++rr)
                    for (int cc = 0; cc < 3; ++cc) {
                        double s = 0;
                        for (int k = 0; k < 3; ++k) s += dSig[3 * rr + k] * p->Rg[3 * k + cc];
                        dRg[3 * rr + cc] = 2.0 * s * p->s[cc] * p->s[cc];
                    }
                double gq[4];
                rot_grad_to_quat(in->quats + 4 * i, dRg, gq);
                for (int k = 0; k < 4; ++k) out->g_quats[4 * i + k] += gq[k];
            }
            /* pose: coupled (q, t) and decoupled (q with centre fixed, centre) */
            double gq[4];
            rot_grad_to_quat(in->pose_q + 4 * v, GW, gq);
            for (int k = 0; k < 4; ++k) out->g_q_t[4 * v + k] = gq[k];
            for (int k = 0; k < 3; ++k) out->g_t[3 * v + k] = gt[k];
            double C[3];  /* C = -W^T t */
            for (int k = 0; k < 3; ++k) C[k] = -(W[k] * t[0] + W[3 + k] * t[1] + W[6 + k] * t[2]);
            for (int k = 0; k < 3; ++k) out->g_c[3 * v + k] = -(W[k] * gt[0] + W[3 + k] * gt[1] + W[6 + k] * gt[2]);
            double GWc[9];
            for (int rr = 0; rr < 3; ++rr)
                for (int cc = 0; cc < 3; ++cc) GWc[3 * rr + cc] = GW[3 * rr + cc] - gt[rr] * C[cc];
            rot_grad_to_quat(in->pose_q + 4 * v, GWc, gq);
            for (int k = 0; k < 4; ++k) out->g_q_c[4 * v + k] = gq[k];
        }
        free(g2d_thr);
        free(loss_thr);
        free(hash_row);
        free(row_cnt);
        free(row_list);
        free(row_fill);
        free(order);
        free(keys);
        free(proj);
        off += P;
    }
    return 0;
}
