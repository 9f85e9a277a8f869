"""ctypes binding of the FP64 oracle (gsr_oracle.c) and a dense numpy brute force.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Nothing here
imports the HIP package, and the HIP package never imports this.

Inputs are duck-typed: any object with `means, quats, log_scales,
opacity_logits, rgb` arrays (Gaussians) and `cams, quat, trans` (views,
each camera with `width, height, fx, fy, cx, cy`).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)
_u64p = C.POINTER(C.c_uint64)
_fp = C.POINTER(C.c_float)


class _In(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("means", _dp), ("quats", _dp), ("log_scales", _dp), ("opacity_logits", _dp), ("rgb", _dp),
        ("isotropic", C.c_int32), ("n_views", C.c_int32),
        ("width", _ip), ("height", _ip),
        ("fx", _dp), ("fy", _dp), ("cx", _dp), ("cy", _dp),
        ("pose_q", _dp), ("pose_t", _dp),
        ("z_near", C.c_double), ("blur2d", C.c_double),
        ("w_rgb", C.c_double), ("w_depth", C.c_double), ("w_sil", C.c_double), ("w_prior", C.c_double),
        ("sil_mask_thresh", C.c_double),
        ("t_rgb", _dp), ("t_depth", _dp), ("t_sil", _dp), ("t_prior", _dp), ("t_weight", _dp),
        ("pixel_mask", _u8p),
        ("margin", C.c_double),
        ("mask_ambiguous", C.c_int32), ("want_grads", C.c_int32), ("n_threads", C.c_int32),
        ("res_margin", C.c_double),
    ]


class _Out(C.Structure):
    _fields_ = [
        ("rgb", _dp), ("depth", _dp), ("sil", _dp), ("t_final", _dp),
        ("n_contrib", _ip), ("ambiguous", _u8p), ("loss", _dp),
        ("g_means", _dp), ("g_quats", _dp), ("g_log_scales", _dp), ("g_opacity", _dp), ("g_rgb", _dp),
        ("g_q_t", _dp), ("g_t", _dp), ("g_q_c", _dp), ("g_c", _dp),
        ("decision_hash", _u64p), ("grad2d", _dp),
        ("decision_amb", _u8p), ("residual_amb", _u8p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _lib.oracle_run.argtypes = [C.POINTER(_In), C.POINTER(_Out)]
        _lib.oracle_run.restype = C.c_int
        _lib.oracle_project_view.argtypes = [C.POINTER(_In), C.c_int, _ip, _dp, _dp, _dp, _dp, _dp, _ip, _fp, _dp]
        _lib.oracle_project_view.restype = C.c_int
        _lib.oracle_quat_to_rot.argtypes = [_dp, _dp]
        _lib.oracle_quat_to_rot.restype = C.c_int
    return _lib


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Options:
    z_near: float = 0.2
    blur2d: float = 0.3
    w_rgb: float = 0.5
    w_depth: float = 1.0
    w_sil: float = 1.0
    w_prior: float = 0.0
    sil_mask_thresh: float = -1.0


@dataclass
class Targets:
    rgb: np.ndarray               # [3*sumP] (planar per view)
    depth: np.ndarray             # [sumP]
    sil: Optional[np.ndarray] = None
    prior: Optional[np.ndarray] = None
    weight: Optional[np.ndarray] = None


@dataclass
class Result:
    rgb: np.ndarray
    depth: np.ndarray
    sil: np.ndarray
    t_final: np.ndarray
    n_contrib: np.ndarray
    ambiguous: np.ndarray           # union of the two flags below
    loss: np.ndarray
    decision_hash: np.ndarray
    grads: Optional[dict] = None
    grad2d: Optional[np.ndarray] = None
    # a compositing decision (alpha vs 1/255 or 0.99, transmittance vs 1e-4)
    # within `margin` of its threshold: the image itself may differ
    decision_ambiguous: Optional[np.ndarray] = None
    # a weighted L1 residual's sign or the tracking mask within its margin:
    # the image is well defined, only the sign of the loss derivative is not
    residual_ambiguous: Optional[np.ndarray] = None


def _make_in(g, views, opts: Options, keep: list):
    n = int(np.asarray(g.means).shape[0])
    ls = np.asarray(g.log_scales)
    iso = int(ls.ndim == 2 and ls.shape[1] == 1)
    arrs = dict(
        means=_f64(np.asarray(g.means).reshape(-1)), quats=_f64(np.asarray(g.quats).reshape(-1)),
        log_scales=_f64(ls.reshape(-1)), opacity_logits=_f64(np.asarray(g.opacity_logits).reshape(-1)),
        rgb=_f64(np.asarray(g.rgb).reshape(-1)),
        width=np.array([c.width for c in views.cams], np.int32),
        height=np.array([c.height for c in views.cams], np.int32),
        fx=_f64([c.fx for c in views.cams]), fy=_f64([c.fy for c in views.cams]),
        cx=_f64([c.cx for c in views.cams]), cy=_f64([c.cy for c in views.cams]),
        pose_q=_f64(np.asarray(views.quat).reshape(-1)), pose_t=_f64(np.asarray(views.trans).reshape(-1)),
    )
    keep.append(arrs)
    s = _In()
    s.n = n
    for k in ("means", "quats", "log_scales", "opacity_logits", "rgb", "fx", "fy", "cx", "cy", "pose_q", "pose_t"):
        setattr(s, k, _p(arrs[k]))
    s.width = _p(arrs["width"], _ip)
    s.height = _p(arrs["height"], _ip)
    s.isotropic = iso
    s.n_views = len(views.cams)
    s.z_near = opts.z_near
    s.blur2d = opts.blur2d
    s.w_rgb, s.w_depth, s.w_sil, s.w_prior = opts.w_rgb, opts.w_depth, opts.w_sil, opts.w_prior
    s.sil_mask_thresh = opts.sil_mask_thresh
    return s, n, iso


def run(g, views, opts: Options = Options(), targets: Optional[Targets] = None, want_grads: bool = False,
        pixel_mask: Optional[np.ndarray] = None, margin: float = 1e-5, mask_ambiguous: bool = False,
        threads: int = 0, want_grad2d: bool = False, res_margin: Optional[float] = None) -> Result:
    """Render every view; with targets also the loss; with want_grads the gradients.

    A pixel is flagged ambiguous when a decision on its path lies within a
    relative margin of its threshold.  Two kinds are reported apart:
    decision_ambiguous (alpha vs 1/255 and vs 0.99, the next transmittance vs
    1e-4; `margin`), where the image itself may differ between FP32 and FP64,
    and residual_ambiguous (the sign of a weighted loss residual, the tracking
    mask; `res_margin`, default `margin`), where only the sign of the loss
    derivative may.  `ambiguous` is their union; mask_ambiguous gives those
    pixels loss weight 0."""
    keep = []
    s, n, iso = _make_in(g, views, opts, keep)
    V = len(views.cams)
    P = int(sum(c.width * c.height for c in views.cams))
    tg = {}
    if targets is not None:
        tg = dict(rgb=_f64(targets.rgb).reshape(-1), depth=_f64(targets.depth).reshape(-1),
                  sil=_f64(targets.sil).reshape(-1) if targets.sil is not None else None,
                  prior=_f64(targets.prior).reshape(-1) if targets.prior is not None else None,
                  weight=_f64(targets.weight).reshape(-1) if targets.weight is not None else None)
        assert tg["rgb"].size == 3 * P and tg["depth"].size == P
        s.t_rgb, s.t_depth = _p(tg["rgb"]), _p(tg["depth"])
        s.t_sil, s.t_prior, s.t_weight = _p(tg["sil"]), _p(tg["prior"]), _p(tg["weight"])
    pm = None
    if pixel_mask is not None:
        pm = np.ascontiguousarray(pixel_mask.reshape(-1), dtype=np.uint8)
        assert pm.size == P
        s.pixel_mask = _p(pm, _u8p)
    s.margin = margin
    s.res_margin = margin if res_margin is None else res_margin
    s.mask_ambiguous = int(mask_ambiguous)
    s.want_grads = int(want_grads)
    s.n_threads = threads
    o = _Out()
    res = Result(rgb=np.zeros(3 * P), depth=np.zeros(P), sil=np.zeros(P), t_final=np.zeros(P),
                 n_contrib=np.zeros(P, np.int32), ambiguous=np.zeros(P, np.uint8), loss=np.zeros(V),
                 decision_hash=np.zeros(V, np.uint64), decision_ambiguous=np.zeros(P, np.uint8),
                 residual_ambiguous=np.zeros(P, np.uint8))
    o.rgb, o.depth, o.sil, o.t_final = _p(res.rgb), _p(res.depth), _p(res.sil), _p(res.t_final)
    o.decision_amb = _p(res.decision_ambiguous, _u8p)
    o.residual_amb = _p(res.residual_ambiguous, _u8p)
    o.n_contrib = _p(res.n_contrib, _ip)
    o.ambiguous = _p(res.ambiguous, _u8p)
    o.loss = _p(res.loss)
    o.decision_hash = _p(res.decision_hash, _u64p)
    if want_grads:
        gr = dict(means=np.zeros((n, 3)), quats=np.zeros((n, 4)), log_scales=np.zeros((n, 1 if iso else 3)),
                  opacity_logits=np.zeros(n), rgb=np.zeros((n, 3)),
                  dq_t=np.zeros((V, 4)), dt=np.zeros((V, 3)), dq_c=np.zeros((V, 4)), dc=np.zeros((V, 3)))
        o.g_means, o.g_quats, o.g_log_scales = _p(gr["means"]), _p(gr["quats"]), _p(gr["log_scales"])
        o.g_opacity, o.g_rgb = _p(gr["opacity_logits"]), _p(gr["rgb"])
        o.g_q_t, o.g_t, o.g_q_c, o.g_c = _p(gr["dq_t"]), _p(gr["dt"]), _p(gr["dq_c"]), _p(gr["dc"])
        res.grads = gr
        if want_grad2d:
            res.grad2d = np.zeros((V, n, 10))
            o.grad2d = _p(res.grad2d)
    rc = lib().oracle_run(C.byref(s), C.byref(o))
    if rc != 0:
        raise RuntimeError(f"oracle_run failed: {rc}")
    return res


@dataclass
class Projection:
    visible: np.ndarray
    mean2d: np.ndarray
    cov2d: np.ndarray
    conic: np.ndarray
    opacity: np.ndarray
    radius: np.ndarray
    rect: np.ndarray
    z32: np.ndarray
    Xc: np.ndarray


def project_view(g, views, v: int, opts: Options = Options()) -> Projection:
    keep = []
    s, n, _ = _make_in(g, views, opts, keep)
    pr = Projection(np.zeros(n, np.int32), np.zeros((n, 2)), np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n),
                    np.zeros(n), np.zeros((n, 4), np.int32), np.zeros(n, np.float32), np.zeros((n, 3)))
    lib().oracle_project_view(C.byref(s), v, _p(pr.visible, _ip), _p(pr.mean2d), _p(pr.cov2d), _p(pr.conic),
                              _p(pr.opacity), _p(pr.radius), _p(pr.rect, _ip), _p(pr.z32, _fp), _p(pr.Xc))
    return pr


def quat_to_rot(q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    R = np.zeros(9)
    lib().oracle_quat_to_rot(_p(q), _p(R))
    return R.reshape(3, 3)


def bin_view(pr: Projection, width: int, height: int, tile_w: int, tile_h: int):
    """Per-tile Gaussian lists of one view from the binning rule: a Gaussian is
    listed in every tile that its clamped pixel rectangle touches, ordered by
    (float32 depth, index).  Returns (tile_start[T+1], ids[K])."""
    tx = (width + tile_w - 1) // tile_w
    ty = (height + tile_h - 1) // tile_h
    vis = np.nonzero(pr.visible)[0]
    order = vis[np.lexsort((vis, pr.z32[vis]))]
    lists = [[] for _ in range(tx * ty)]
    for i in order:
        x0, x1, y0, y1 = pr.rect[i]
        for by in range(y0 // tile_h, y1 // tile_h + 1):
            for bx in range(x0 // tile_w, x1 // tile_w + 1):
                lists[by * tx + bx].append(int(i))
    start = np.zeros(tx * ty + 1, np.int64)
    for t in range(tx * ty):
        start[t + 1] = start[t] + len(lists[t])
    ids = np.array([i for l in lists for i in l], np.int64)
    return start, ids


def rect_boundary_margin(pr: Projection) -> np.ndarray:
    """Distance of m -/+ r to the nearest integer, per Gaussian (for flagging
    rectangles whose integer bounds could round either way)."""
    lo = np.concatenate([pr.mean2d - pr.radius[:, None], pr.mean2d + pr.radius[:, None]], 1)
    return np.abs(lo - np.round(lo)).min(1)


# ----------------------------------------------------------------------------
# dense brute force (numpy): every Gaussian at every pixel, explicit sort and
# front-to-back loop; for a few dozen Gaussians on tiny images.  Rotations come
# from scipy, independently of the C oracle.
# ----------------------------------------------------------------------------

def brute_render(g, views, opts: Options = Options()):
    from scipy.spatial.transform import Rotation
    means = np.asarray(g.means, np.float64)
    n = means.shape[0]
    quats = np.asarray(g.quats, np.float64)
    ls = np.asarray(g.log_scales, np.float64)
    s = np.exp(np.repeat(ls, 3, axis=1) if ls.shape[1] == 1 else ls)
    o = 1.0 / (1.0 + np.exp(-np.asarray(g.opacity_logits, np.float64)))
    col = np.asarray(g.rgb, np.float64)
    Rg = Rotation.from_quat(np.concatenate([quats[:, 1:], quats[:, :1]], 1)).as_matrix() if n else np.zeros((0, 3, 3))
    Sig = Rg @ (s[:, :, None] ** 2 * np.transpose(Rg, (0, 2, 1)))
    out = []
    for v, cam in enumerate(views.cams):
        qv = np.asarray(views.quat[v], np.float64)
        W = Rotation.from_quat(np.r_[qv[1:], qv[:1]]).as_matrix()
        X = means @ W.T + np.asarray(views.trans[v], np.float64)
        z = X[:, 2]
        Jm = np.zeros((n, 2, 3))
        Jm[:, 0, 0] = cam.fx / z
        Jm[:, 0, 2] = -cam.fx * X[:, 0] / z ** 2
        Jm[:, 1, 1] = cam.fy / z
        Jm[:, 1, 2] = -cam.fy * X[:, 1] / z ** 2
        cov = Jm @ (W @ Sig @ W.T) @ np.transpose(Jm, (0, 2, 1)) + opts.blur2d * np.eye(2)
        m = np.stack([cam.fx * X[:, 0] / z + cam.cx, cam.fy * X[:, 1] / z + cam.cy], 1)
        ok = (z > opts.z_near) & (255.0 * o > 1.0)
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        pix = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float64)
        P = pix.shape[0]
        order = sorted([i for i in range(n) if ok[i]], key=lambda i: (np.float32(z[i]), i))
        T = np.ones(P)
        done = np.zeros(P, bool)
        acc = np.zeros((P, 5))
        for i in order:
            d = pix - m[i]
            q = np.einsum("pi,ij,pj->p", d, np.linalg.inv(cov[i]), d)
            a = np.minimum(ALPHA_MAX, o[i] * np.exp(-0.5 * q))
            use = (~done) & (a >= ALPHA_MIN)
            Tn = T * (1 - a)
            stop = use & (Tn < T_MIN)
            done |= stop
            use &= ~stop
            w = np.where(use, a * T, 0.0)
            acc += w[:, None] * np.r_[col[i], z[i], 1.0][None, :]
            T = np.where(use, Tn, T)
        out.append(dict(rgb=acc[:, :3].T.reshape(3, cam.height, cam.width),
                        depth=acc[:, 3].reshape(cam.height, cam.width),
                        sil=acc[:, 4].reshape(cam.height, cam.width),
                        t_final=T.reshape(cam.height, cam.width)))
    return out
