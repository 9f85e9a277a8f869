"""FP64 oracle of the optimisation steps around the rasteriser: Adam, the
decoupled pose update and tracking loop, the map update, and the creation
of Gaussians from an RGB-D frame.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Readings (the paper names "gradient-based optimization" and a
rotation-translation decoupled strategy but no update rule, step sizes or
thresholds):
- Adam (Kingma & Ba, 2015, Algorithm 1) with bias correction, applied per
  parameter block.
- Tracking: each iteration renders once at the current pose, takes the
  decoupled gradients (dL/dq at a fixed camera centre C = -R^T t, and
  dL/dC), and makes one Adam step on q (step size lr_rot) and one on C
  (lr_pos); then t = -R(q/|q|) C.  The renderer reads the pose rounded to
  FP32; the optimiser state stays in FP64.  q is not renormalised (the
  renderer normalises it).
- Mapping: one Adam step per raw parameter array with its own step size.
- New Gaussians (initialisation section): a pixel with target depth D > 0
  (and, when densifying, rendered silhouette S < threshold) gives one
  Gaussian at the unprojected point R^T (X_c - t), X_c = ((u - cx) D / fx,
  (v - cy) D / fy, D), with the pixel's colour, opacity 0.5 (logit 0),
  identity rotation and radius D / f with f = (fx + fy) / 2 (log-scale
  log(D / f) on every axis).  Pixels are taken in raster order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


# ----------------------------------------------------------------------------
# Adam (Kingma & Ba 2015, Algorithm 1)
# ----------------------------------------------------------------------------

def adam_step(x, g, m, v, step: int, lr: float, beta1: float, beta2: float, eps: float):
    """One Adam update of x with gradient g at 1-based step `step`.
    Returns (x', m', v'); inputs are not modified."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return x - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


# ----------------------------------------------------------------------------
# poses: world-to-camera (q, t); camera centre C = -R^T t
# ----------------------------------------------------------------------------

def rot(q) -> np.ndarray:
    """Rotation of the normalised (w, x, y, z) quaternion (scipy's routine)."""
    from scipy.spatial.transform import Rotation
    q = np.asarray(q, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def centre_of(q, t) -> np.ndarray:
    return -rot(q).T @ np.asarray(t, np.float64)


def trans_of(q, C) -> np.ndarray:
    return -rot(q) @ np.asarray(C, np.float64)


@dataclass
class PoseAdam:
    lr_rot: float = 2e-3
    lr_pos: float = 2e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


@dataclass
class PoseState:
    """Optimiser state of one view: raw quaternion, camera centre, moments."""
    q: np.ndarray
    C: np.ndarray
    mq: np.ndarray = field(default_factory=lambda: np.zeros(4))
    vq: np.ndarray = field(default_factory=lambda: np.zeros(4))
    mc: np.ndarray = field(default_factory=lambda: np.zeros(3))
    vc: np.ndarray = field(default_factory=lambda: np.zeros(3))
    step: int = 0

    @staticmethod
    def from_pose(q, t) -> "PoseState":
        q = np.asarray(q, np.float64).copy()
        return PoseState(q=q, C=centre_of(q, t))

    def pose(self):
        """The pose the renderer reads: (q, t = -R C), rounded to FP32."""
        return self.q.astype(np.float32), trans_of(self.q, self.C).astype(np.float32)


def pose_step(st: PoseState, dq_c, dc, hp: PoseAdam) -> PoseState:
    """One decoupled step: rotation about the fixed camera centre from
    dL/dq|C, then the centre itself from dL/dC."""
    k = st.step + 1
    q, mq, vq = adam_step(st.q, dq_c, st.mq, st.vq, k, hp.lr_rot, hp.beta1, hp.beta2, hp.eps)
    C, mc, vc = adam_step(st.C, dc, st.mc, st.vc, k, hp.lr_pos, hp.beta1, hp.beta2, hp.eps)
    return PoseState(q=q, C=C, mq=mq, vq=vq, mc=mc, vc=vc, step=k)


@dataclass
class Views:
    cams: list
    quat: np.ndarray
    trans: np.ndarray


def track(g, cams, q0, t0, targets, opts, hp: PoseAdam, iters: int, **run_kw):
    """The tracking loop over all views at once (each view has its own
    state).  Returns (states after every iteration, loss per iteration [iters, V])."""
    from . import oracle
    V = len(cams)
    states = [PoseState.from_pose(q0[v], t0[v]) for v in range(V)]
    hist, losses = [], []
    for _ in range(iters):
        poses = [s.pose() for s in states]
        views = Views(cams, np.stack([p[0] for p in poses]), np.stack([p[1] for p in poses]))
        r = oracle.run(g, views, opts, targets, want_grads=True, **run_kw)
        losses.append(r.loss.copy())
        states = [pose_step(states[v], r.grads["dq_c"][v], r.grads["dc"][v], hp) for v in range(V)]
        hist.append(states)
    return hist, np.array(losses)


# ----------------------------------------------------------------------------
# mapping step
# ----------------------------------------------------------------------------

MAP_KEYS = ("means", "quats", "log_scales", "opacity_logits", "rgb")


@dataclass
class MapAdam:
    lr_means: float = 1e-4
    lr_quats: float = 1e-3
    lr_log_scales: float = 1e-3
    lr_opacity: float = 5e-2
    lr_rgb: float = 2.5e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    def lr(self, key: str) -> float:
        return {"means": self.lr_means, "quats": self.lr_quats, "log_scales": self.lr_log_scales,
                "opacity_logits": self.lr_opacity, "rgb": self.lr_rgb}[key]


def map_step(params: dict, grads: dict, m: dict, v: dict, step: int, hp: MapAdam):
    """Adam over every raw parameter array (1-based step).  Returns new
    (params, m, v) dicts."""
    P, Mo, Vo = {}, {}, {}
    for k in params:
        P[k], Mo[k], Vo[k] = adam_step(params[k], grads[k], m[k], v[k], step, hp.lr(k), hp.beta1, hp.beta2, hp.eps)
    return P, Mo, Vo


# ----------------------------------------------------------------------------
# new Gaussians from an RGB-D frame
# ----------------------------------------------------------------------------

def new_gaussians(cam, q, t, rgb, depth, sil: Optional[np.ndarray] = None, sil_thresh: float = 0.5,
                  isotropic: bool = True):
    """rgb [3, H*W] planar, depth [H*W], sil [H*W] or None (initialisation:
    every pixel with depth).  Returns (pixel indices, dict of parameters)."""
    depth = np.asarray(depth, np.float64).reshape(-1)
    rgb = np.asarray(rgb, np.float64).reshape(3, -1)
    sel = depth > 0.0
    if sil is not None:
        sel &= np.asarray(sil).reshape(-1) < sil_thresh
    pix = np.nonzero(sel)[0]
    u = (pix % cam.width).astype(np.float64)
    vv = (pix // cam.width).astype(np.float64)
    D = depth[pix]
    Xc = np.stack([(u - cam.cx) * D / cam.fx, (vv - cam.cy) * D / cam.fy, D], 1)
    R = rot(q)
    mu = (Xc - np.asarray(t, np.float64)[None, :]) @ R   # rows: R^T (X_c - t)
    f = 0.5 * (cam.fx + cam.fy)
    ls = np.log(D / f)
    n = pix.size
    out = dict(means=mu, quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
               log_scales=ls[:, None] if isotropic else np.repeat(ls[:, None], 3, 1),
               opacity_logits=np.zeros(n), rgb=rgb[:, pix].T.copy())
    return pix, out
