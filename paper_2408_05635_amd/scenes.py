"""Seeded synthetic inputs shaped like the paper's RGB-D workloads.

This module only draws inputs: Gaussian parameters, pinhole cameras and
world-to-camera poses.  It holds none of the renderer's arithmetic (no
projection, no compositing, no loss), so both the HIP path and the FP64
oracle can consume what it produces without sharing method code.

The paper evaluates on TUM-RGBD (Evaluation, Experiment Setup): 640x480
RGB-D at 30 Hz from a Kinect in office-scale rooms.  That dataset is not
available here; the generators below stand in for it with indoor rooms of
the same scale seen by a 640x480 camera with f = 525 px.

Conventions (shared with the C-ABI):
  * Gaussian parameters are raw: means [N,3] (world, metres), quats [N,4]
    (w,x,y,z, not normalised), log_scales [N,3] (or [N,1] if isotropic),
    opacity_logits [N], rgb [N,3].
  * A pose is world-to-camera (R_cw, t_cw) as in the paper's reprojection
    residual (Preliminaries, Visual Geometry Residual): X_c = R_cw X + t_cw,
    stored as a (w,x,y,z) quaternion and a translation.
  * Camera frame is the OpenCV one: x right, y down, z forward.  World z is up.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "Camera", "Gaussians", "Views", "Workload",
    "random_unit_quats", "pose_from_center", "perturb_pose",
    "smooth_trajectory", "room_gaussians", "multiroom_gaussians",
    "config1", "config2", "config3", "config4", "config5", "tiny_scene",
]


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclass
class Gaussians:
    means: np.ndarray          # [N,3] float32
    quats: np.ndarray          # [N,4] float32 (w,x,y,z)
    log_scales: np.ndarray     # [N,3] or [N,1] float32
    opacity_logits: np.ndarray  # [N] float32
    rgb: np.ndarray            # [N,3] float32

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def isotropic(self) -> bool:
        return self.log_scales.shape[1] == 1

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.means[idx].copy(), self.quats[idx].copy(),
                         self.log_scales[idx].copy(), self.opacity_logits[idx].copy(),
                         self.rgb[idx].copy())

    def permuted(self, perm) -> "Gaussians":
        return self.subset(np.asarray(perm))


@dataclass
class Views:
    cams: List[Camera]
    quat: np.ndarray   # [V,4] float32, w2c (w,x,y,z)
    trans: np.ndarray  # [V,3] float32, w2c

    @property
    def n(self) -> int:
        return len(self.cams)

    def pixel_offsets(self) -> np.ndarray:
        off = np.zeros(self.n + 1, dtype=np.int64)
        for v, c in enumerate(self.cams):
            off[v + 1] = off[v] + c.width * c.height
        return off

    def select(self, idx) -> "Views":
        idx = list(idx)
        return Views([self.cams[i] for i in idx], self.quat[idx].copy(), self.trans[idx].copy())


@dataclass
class Workload:
    """A scene, the poses the renderer is called at, and the poses whose
    renders serve as targets (true poses), plus optional depth-prior noise."""
    name: str
    gaussians: Gaussians
    views: Views                 # poses the renderer is evaluated at
    target_views: Views          # poses the targets are rendered at
    prior_noise: Optional[np.ndarray] = None  # per-pixel multiplicative N(0, sigma) draws, concatenated
    weights: dict = field(default_factory=dict)
    target_gaussians: Optional[Gaussians] = None  # scene the targets are rendered from (None: `gaussians`)

    @property
    def truth(self) -> Gaussians:
        return self.gaussians if self.target_gaussians is None else self.target_gaussians


# ----------------------------------------------------------------------------
# random rotations and poses
# ----------------------------------------------------------------------------

def _wxyz_from_matrix(R: np.ndarray) -> np.ndarray:
    q = Rotation.from_matrix(R).as_quat()  # (x,y,z,w)
    q = np.concatenate([q[..., 3:4], q[..., 0:3]], axis=-1)
    q = np.where(q[..., :1] < 0, -q, q)
    return q


def _matrix_from_wxyz(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:4], q[..., 0:1]], axis=-1)).as_matrix()


def random_unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def pose_from_center(center, yaw: float, pitch: float) -> Tuple[np.ndarray, np.ndarray]:
    """World-to-camera (quat wxyz, t) for a camera at `center` looking along
    yaw (about world z) and pitch (positive looks up), roll 0."""
    cy_, sy_ = np.cos(yaw), np.sin(yaw)
    cp, sp = np.cos(pitch), np.sin(pitch)
    fwd = np.array([cp * cy_, cp * sy_, sp])
    right = np.array([sy_, -cy_, 0.0])
    down = np.cross(fwd, right)
    R_cw = np.stack([right, down, fwd], axis=0)
    t = -R_cw @ np.asarray(center, dtype=np.float64)
    return _wxyz_from_matrix(R_cw), t


def perturb_pose(q_wxyz, t, rot_deg: float, trans_m: float, rng_axis, rng_dir):
    """Left-multiply a rotation of `rot_deg` about a random axis and add a
    translation of `trans_m` in a random direction (camera frame)."""
    axis = rng_axis.standard_normal(3)
    axis /= np.linalg.norm(axis)
    d = rng_dir.standard_normal(3)
    d /= np.linalg.norm(d)
    Rd = Rotation.from_rotvec(axis * np.deg2rad(rot_deg)).as_matrix()
    R = _matrix_from_wxyz(q_wxyz)
    R2 = Rd @ R
    t2 = Rd @ np.asarray(t, dtype=np.float64) + trans_m * d
    return _wxyz_from_matrix(R2), t2


def smooth_trajectory(rng: np.random.Generator, n: int, lo, hi, max_step=0.3, max_turn_deg=15.0,
                      height=(1.2, 1.8)):
    """n camera poses inside the box [lo, hi] (x,y) with consecutive centres at most
    `max_step` m apart and view directions at most `max_turn_deg` apart."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(*height)])
    yaw = rng.uniform(0, 2 * np.pi)
    pitch = rng.uniform(-np.deg2rad(15), np.deg2rad(15))
    out = []
    for k in range(n):
        out.append(pose_from_center(c, yaw, pitch))
        for _ in range(100):
            d = rng.standard_normal(3)
            d *= rng.uniform(0.05, max_step) / np.linalg.norm(d)
            c2 = c + d
            if lo[0] <= c2[0] <= hi[0] and lo[1] <= c2[1] <= hi[1] and height[0] <= c2[2] <= height[1]:
                c = c2
                break
        # split the turn budget between yaw and pitch so the total stays below max_turn_deg
        turn = np.deg2rad(rng.uniform(2.0, max_turn_deg))
        ang = rng.uniform(0, 2 * np.pi)
        yaw += turn * np.cos(ang) * 0.7
        pitch = float(np.clip(pitch + turn * np.sin(ang) * 0.7, -np.deg2rad(15), np.deg2rad(15)))
    q = np.stack([p[0] for p in out]).astype(np.float32)
    t = np.stack([p[1] for p in out]).astype(np.float32)
    return q, t


def random_room_poses(rng, n, lo, hi, height=(1.2, 1.8)):
    out = []
    for _ in range(n):
        c = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(*height)])
        out.append(pose_from_center(c, rng.uniform(0, 2 * np.pi),
                                    rng.uniform(-np.deg2rad(15), np.deg2rad(15))))
    return (np.stack([p[0] for p in out]).astype(np.float32),
            np.stack([p[1] for p in out]).astype(np.float32))


# ----------------------------------------------------------------------------
# surface samplers
# ----------------------------------------------------------------------------

def _faces_of_box(lo, hi, inward: bool, skip_bottom: bool = False):
    """Axis-aligned box faces as (origin, edge_u, edge_v, normal)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    s = hi - lo
    faces = []
    for ax in range(3):
        u_ax, v_ax = [a for a in range(3) if a != ax]
        for side in (0, 1):
            if skip_bottom and ax == 2 and side == 0:
                continue
            o = lo.copy()
            o[ax] = lo[ax] if side == 0 else hi[ax]
            eu = np.zeros(3)
            eu[u_ax] = s[u_ax]
            ev = np.zeros(3)
            ev[v_ax] = s[v_ax]
            n = np.zeros(3)
            n[ax] = -1.0 if side == 0 else 1.0
            if inward:
                n = -n
            faces.append((o, eu, ev, n))
    return faces


def _wall_with_door(x0, y0, x1, y1, height, door_center, door_width=1.0, door_height=2.0):
    """A vertical wall segment from (x0,y0) to (x1,y1) with a rectangular doorway,
    split into rectangles (double-sided: two normals)."""
    p0 = np.array([x0, y0, 0.0])
    p1 = np.array([x1, y1, 0.0])
    L = np.linalg.norm(p1 - p0)
    dirv = (p1 - p0) / L
    nrm = np.array([-dirv[1], dirv[0], 0.0])
    a = door_center - door_width / 2
    b = door_center + door_width / 2
    rects = [(0.0, a, 0.0, height), (b, L, 0.0, height), (a, b, door_height, height)]
    faces = []
    for (u0, u1, h0, h1) in rects:
        o = p0 + dirv * u0 + np.array([0, 0, h0])
        eu = dirv * (u1 - u0)
        ev = np.array([0, 0, h1 - h0])
        faces.append((o, eu, ev, nrm))
        faces.append((o, eu, ev, -nrm))
    return faces


def _sample_faces(rng, faces, n, offset_sigma):
    areas = np.array([np.linalg.norm(np.cross(f[1], f[2])) for f in faces])
    counts = rng.multinomial(n, areas / areas.sum())
    pts = []
    for f, k in zip(faces, counts):
        if k == 0:
            continue
        uv = rng.uniform(0, 1, size=(k, 2))
        p = f[0] + uv[:, :1] * f[1] + uv[:, 1:] * f[2] + rng.normal(0, offset_sigma, size=(k, 1)) * f[3]
        pts.append(p)
    pts = np.concatenate(pts, axis=0)
    return pts[rng.permutation(pts.shape[0])]


def room_gaussians(rng, n, size=(4.0, 4.0, 3.0), n_boxes=3, log_scale=(-4.0, 0.5),
                   opacity=(1.0, 1.0), offset_sigma=0.01) -> Tuple[Gaussians, list]:
    """Noisy samples on the inner faces of a room plus boxes standing on its floor."""
    faces = _faces_of_box([0, 0, 0], size, inward=True)
    for _ in range(n_boxes):
        s = rng.uniform(0.3, 1.0, size=3)
        x = rng.uniform(0.2, size[0] - 0.2 - s[0])
        y = rng.uniform(0.2, size[1] - 0.2 - s[1])
        faces += _faces_of_box([x, y, 0.0], [x + s[0], y + s[1], s[2]], inward=False, skip_bottom=True)
    means = _sample_faces(rng, faces, n, offset_sigma)
    g = Gaussians(
        means=means.astype(np.float32),
        quats=random_unit_quats(rng, n),
        log_scales=rng.normal(log_scale[0], log_scale[1], size=(n, 3)).astype(np.float32),
        opacity_logits=rng.normal(opacity[0], opacity[1], size=n).astype(np.float32),
        rgb=rng.uniform(0, 1, size=(n, 3)).astype(np.float32),
    )
    return g, faces


def multiroom_gaussians(rng, n) -> Gaussians:
    """10x8x3 m shell with interior walls at x=5 and y=4 (each with a 1 m doorway),
    ten boxes, and heavy anisotropy: one random axis has log-scale N(-6,0.5), the
    other two N(-3,0.5)."""
    W, D, H = 10.0, 8.0, 3.0
    faces = _faces_of_box([0, 0, 0], [W, D, H], inward=True)
    faces += _wall_with_door(5.0, 0.0, 5.0, D, H, door_center=2.0)
    faces += _wall_with_door(0.0, 4.0, W, 4.0, H, door_center=7.5)
    for _ in range(10):
        s = rng.uniform(0.3, 1.0, size=3)
        x = rng.uniform(0.2, W - 0.2 - s[0])
        y = rng.uniform(0.2, D - 0.2 - s[1])
        faces += _faces_of_box([x, y, 0.0], [x + s[0], y + s[1], s[2]], inward=False, skip_bottom=True)
    means = _sample_faces(rng, faces, n, 0.01)
    ls = rng.normal(-3.0, 0.5, size=(n, 3))
    thin = rng.integers(0, 3, size=n)
    ls[np.arange(n), thin] = rng.normal(-6.0, 0.5, size=n)
    return Gaussians(
        means=means.astype(np.float32),
        quats=random_unit_quats(rng, n),
        log_scales=ls.astype(np.float32),
        opacity_logits=rng.normal(1.0, 1.0, size=n).astype(np.float32),
        rgb=rng.uniform(0, 1, size=(n, 3)).astype(np.float32),
    )


def _perturbed_views(target: Views, seed_axis: int, seed_dir: int, deg=2.0, m=0.02) -> Views:
    qs, ts = [], []
    ra = np.random.default_rng(seed_axis)
    rd = np.random.default_rng(seed_dir)
    for v in range(target.n):
        q, t = perturb_pose(target.quat[v], target.trans[v], deg, m, ra, rd)
        qs.append(q)
        ts.append(t)
    return Views(list(target.cams), np.stack(qs).astype(np.float32), np.stack(ts).astype(np.float32))


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def config1() -> Workload:
    """2,000 Gaussians in front of a 128x96 camera; target at a pose 2 deg / 2 cm away."""
    rng = np.random.default_rng(1)
    n = 2000
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(1.5, 4.0, n)], 1)
    g = Gaussians(
        means=means.astype(np.float32),
        quats=random_unit_quats(rng, n),
        log_scales=rng.normal(-3.0, 0.3, size=(n, 3)).astype(np.float32),
        opacity_logits=rng.normal(0.0, 1.0, size=n).astype(np.float32),
        rgb=rng.uniform(0, 1, size=(n, 3)).astype(np.float32),
    )
    cam = Camera(128, 96, 110.0, 110.0, 64.0, 48.0)
    views = Views([cam], np.array([[1, 0, 0, 0]], np.float32), np.zeros((1, 3), np.float32))
    target = _perturbed_views(views, 11, 12)
    return Workload("config1_2k_128x96", g, views, target,
                    weights=dict(w_rgb=0.5, w_depth=1.0, w_sil=1.0, w_prior=0.0))


def _room_cam(W=640, H=480):
    f = 525.0 * W / 640.0
    return Camera(W, H, f, f, (W - 1) / 2.0, (H - 1) / 2.0)


def config2(n_views: int = 8, n: int = 200_000) -> Workload:
    """Tracking: 200k-Gaussian room, 640x480, poses along a smooth trajectory;
    the renderer is called at each true pose perturbed by 2 deg / 2 cm."""
    rng = np.random.default_rng(2)
    g, _ = room_gaussians(rng, n)
    q, t = smooth_trajectory(np.random.default_rng(31), n_views, (0.5, 0.5), (3.5, 3.5))
    target = Views([_room_cam()] * n_views, q, t)
    views = _perturbed_views(target, 11, 12)
    return Workload("config2_200k_640x480", g, views, target,
                    weights=dict(w_rgb=0.5, w_depth=1.0, w_sil=1.0, w_prior=0.0))


def perturbed_map(g: Gaussians, rng: np.random.Generator) -> Gaussians:
    """The map being optimised: every parameter of the true scene off by a
    small seeded amount (5 mm, 0.1 in log-scale, 0.3 in opacity logit, 0.05
    in colour and in each quaternion component)."""
    n = g.n
    return Gaussians(
        means=(g.means + rng.normal(0.0, 0.005, size=(n, 3))).astype(np.float32),
        quats=(g.quats + rng.normal(0.0, 0.05, size=(n, 4))).astype(np.float32),
        log_scales=(g.log_scales + rng.normal(0.0, 0.1, size=g.log_scales.shape)).astype(np.float32),
        opacity_logits=(g.opacity_logits + rng.normal(0.0, 0.3, size=n)).astype(np.float32),
        rgb=(g.rgb + rng.normal(0.0, 0.05, size=(n, 3))).astype(np.float32),
    )


def config3(n: int = 500_000, n_views: int = 8) -> Workload:
    """Mapping: 500k-Gaussian room, 8 keyframes on a smooth trajectory, depth
    prior.  Poses are the true ones; the map is a perturbed copy of the scene
    (sub-seed 33) and the targets are renders of the true scene."""
    rng = np.random.default_rng(3)
    g, _ = room_gaussians(rng, n)
    q, t = smooth_trajectory(np.random.default_rng(31), n_views, (0.5, 0.5), (3.5, 3.5))
    views = Views([_room_cam()] * n_views, q, t)
    P = sum(c.width * c.height for c in views.cams)
    noise = np.random.default_rng(32).normal(0.0, 0.02, size=P).astype(np.float32)
    return Workload("config3_500k_8x640x480_prior", perturbed_map(g, np.random.default_rng(33)), views, views,
                    prior_noise=noise, weights=dict(w_rgb=0.5, w_depth=1.0, w_sil=1.0, w_prior=1.0),
                    target_gaussians=g)


def config4(n: int = 1_000_000, n_views: int = 32) -> Workload:
    """Uneven batch: 1M-Gaussian room, 32 poses at mixed resolutions."""
    rng = np.random.default_rng(4)
    g, _ = room_gaussians(rng, n)
    res = [(320, 240), (640, 480), (960, 540), (1200, 680)]
    rr = np.random.default_rng(41)
    cams = [_room_cam(*res[k]) for k in rr.integers(0, 4, size=n_views)]
    q, t = random_room_poses(np.random.default_rng(42), n_views, (0.5, 0.5), (3.5, 3.5))
    target = Views(cams, q, t)
    views = _perturbed_views(target, 11, 12)
    return Workload("config4_1M_32xmixed", g, views, target,
                    weights=dict(w_rgb=0.5, w_depth=1.0, w_sil=1.0, w_prior=0.0))


def config5(n: int = 3_000_000, n_views: int = 16) -> Workload:
    """Large: 3M anisotropic Gaussians in a 10x8x3 m multi-room layout, 16 views at 1200x680."""
    rng = np.random.default_rng(5)
    g = multiroom_gaussians(rng, n)
    cam = Camera(1200, 680, 600.0, 600.0, 599.5, 339.5)
    q, t = smooth_trajectory(np.random.default_rng(52), n_views, (0.5, 0.5), (9.5, 7.5))
    target = Views([cam] * n_views, q, t)
    views = _perturbed_views(target, 11, 12)
    P = sum(c.width * c.height for c in views.cams)
    noise = np.random.default_rng(53).normal(0.0, 0.02, size=P).astype(np.float32)
    return Workload("config5_3M_16x1200x680_aniso", g, views, target, prior_noise=noise,
                    weights=dict(w_rgb=0.5, w_depth=1.0, w_sil=1.0, w_prior=1.0))


def tiny_scene(seed: int, n: int = 24, width: int = 32, height: int = 24, isotropic: bool = False,
               log_scale=(-2.3, 0.3), z=(1.5, 3.0), spread=0.5, opacity=(0.5, 1.0)) -> Workload:
    """A handful of Gaussians in front of a small camera, for brute force and
    finite-difference checks."""
    rng = np.random.default_rng(1000 + seed)
    means = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread * 0.75, spread * 0.75, n),
                      rng.uniform(z[0], z[1], n)], 1)
    ls = rng.normal(log_scale[0], log_scale[1], size=(n, 1 if isotropic else 3))
    g = Gaussians(
        means=means.astype(np.float32),
        quats=random_unit_quats(rng, n),
        log_scales=ls.astype(np.float32),
        opacity_logits=rng.normal(opacity[0], opacity[1], size=n).astype(np.float32),
        rgb=rng.uniform(0, 1, size=(n, 3)).astype(np.float32),
    )
    f = 1.1 * width
    cam = Camera(width, height, f, f, (width - 1) / 2.0, (height - 1) / 2.0)
    views = Views([cam], np.array([[1, 0, 0, 0]], np.float32), np.zeros((1, 3), np.float32))
    target = _perturbed_views(views, 2000 + seed, 3000 + seed)
    return Workload(f"tiny_{seed}", g, views, target,
                    weights=dict(w_rgb=0.5, w_depth=1.0, w_sil=1.0, w_prior=0.0))
