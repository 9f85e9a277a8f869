"""Helpers shared by the GPU parity tests: move seeded scenes to the device,
build oracle targets, and measure errors the way the parity bar states them
(images: max abs error over pixels without an ambiguous compositing decision
/ max |oracle| per channel; gradients: ||gpu - oracle||_inf / ||oracle||_inf
per parameter group).

Every comparison states how many pixels it compared and fails when that
number is zero or below the floor the test sets, so a parity test cannot pass
by comparing nothing.
"""
from __future__ import annotations

import numpy as np

import oracle

IMG_TOL = 1e-5
GRAD_TOL = 1e-4
# residual-sign decisions are flagged within this relative margin (a few
# times the FP32 error of an accumulated image value near 1)
RES_MARGIN = 4e-6
# elementwise relative error of the gradient entries above 1e-3 of their
# group's largest magnitude (reported beside the group bar; the bound allows
# for the cancellation of many per-pixel terms into a small entry)
GRAD_ELEM_TOL = 1e-2


class ParityCoverageError(AssertionError):
    """A parity comparison covered no pixel, or fewer than its floor."""


def require_coverage(mask: np.ndarray, floor: float, label: str) -> int:
    """Number of True entries of mask; raises if it is 0 or below floor * size."""
    mask = np.asarray(mask, bool)
    n = int(mask.sum())
    size = int(mask.size)
    frac = n / size if size else 0.0
    print(f"{label}: compared {n}/{size} pixels ({100.0 * frac:.2f}%, floor {100.0 * floor:.0f}%)", flush=True)
    if n == 0:
        raise ParityCoverageError(f"{label}: no pixel was compared")
    if frac < floor:
        raise ParityCoverageError(f"{label}: compared {n}/{size} pixels, below the floor of {100.0 * floor:.0f}%")
    return n


def dev_params(g, device="cuda"):
    import torch
    from paper_2408_05635_amd.raster import GaussianParams
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)  # noqa: E731
    return GaussianParams(t(g.means), t(g.quats), t(g.log_scales), t(g.opacity_logits).reshape(-1), t(g.rgb))


def dev_poses(views, device="cuda"):
    import torch
    q = torch.from_numpy(np.ascontiguousarray(views.quat, dtype=np.float32)).to(device)
    t = torch.from_numpy(np.ascontiguousarray(views.trans, dtype=np.float32)).to(device)
    return q, t


def oracle_targets(w, prior_noise=None):
    """Targets = oracle render at the target poses, rounded to float32 (the
    inputs both sides see)."""
    r = oracle.run(w.truth, w.target_views)
    f = lambda a: np.asarray(a, np.float32)  # noqa: E731
    tg = dict(rgb=f(r.rgb), depth=f(r.depth), sil=f(r.sil))
    if prior_noise is not None:
        tg["prior"] = f(r.depth * (1.0 + prior_noise.astype(np.float64)))
    return tg


def to_dev(d, device="cuda"):
    import torch
    return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device))
            for k, v in d.items()}


def _np(a):
    return a.detach().double().cpu().numpy() if hasattr(a, "double") else np.asarray(a, np.float64)


def _channel_planes(rgb: np.ndarray, cams) -> list:
    """The three colour planes over all views (images are planar per view)."""
    planes = [[], [], []]
    off = 0
    for c in cams:
        p = c.width * c.height
        for k in range(3):
            planes[k].append(rgb[3 * off + k * p: 3 * off + (k + 1) * p])
        off += p
    return [np.concatenate(pl) for pl in planes]


def image_errors(gpu: dict, orc, cams, ok: np.ndarray, floor: float = 0.0, label: str = "images") -> dict:
    """Per-channel max abs error over the pixels where ok is true, relative to
    the channel's largest |oracle| value over those pixels; also the 99.9th
    percentile of the elementwise relative error (floored at 1e-6 of the
    channel's largest value).  Raises ParityCoverageError if ok selects no
    pixel or fewer than floor of them."""
    ok = np.asarray(ok, bool)
    P = int(sum(c.width * c.height for c in cams))
    assert ok.size == P, (ok.size, P)
    require_coverage(ok, floor, label)
    out, p999 = {}, {}
    chans = dict(zip("rgb", _channel_planes(_np(gpu["rgb"]), cams)))
    chans_o = dict(zip("rgb", _channel_planes(np.asarray(orc.rgb, np.float64), cams)))
    chans["depth"], chans_o["depth"] = _np(gpu["depth"]), np.asarray(orc.depth, np.float64)
    chans["sil"], chans_o["sil"] = _np(gpu["sil"]), np.asarray(orc.sil, np.float64)
    for name in ("r", "g", "b", "depth", "sil"):
        g, o = chans[name][ok], chans_o[name][ok]
        scale = max(float(np.abs(o).max()), 1e-30)
        d = np.abs(g - o)
        out[name] = float(d.max() / scale)
        p999[name] = float(np.percentile(d / np.maximum(np.abs(o), 1e-6 * scale), 99.9))
    out["p99.9_elem"] = max(p999.values())
    return out


def grad_errors(gpu: dict, orc_grads: dict, keys=None, elem: dict = None) -> dict:
    """||g - o||_inf / ||o||_inf per parameter group.  If `elem` is a dict, it
    receives per group the largest elementwise relative error over the
    entries whose |oracle| exceeds 1e-3 of the group's largest."""
    names = {"means": "g_means", "quats": "g_quats", "log_scales": "g_log_scales",
             "opacity_logits": "g_opacity_logits", "rgb": "g_rgb", "dq_t": "dq_t", "dt": "dt", "dq_c": "dq_c",
             "dc": "dc"}
    out = {}
    # a group whose oracle gradient is rounding noise (e.g. quaternions of
    # isotropic Gaussians, exactly zero in theory) is measured against the
    # largest gradient of all groups instead of against itself
    scale = max(float(np.abs(v).max()) for k, v in orc_grads.items() if k in names)
    assert scale > 0.0, "every oracle gradient is zero: nothing would be compared"
    for k, gk in names.items():
        if keys is not None and k not in keys:
            continue
        if gpu.get(gk) is None:
            continue
        g = _np(gpu[gk]).reshape(orc_grads[k].shape)
        o = orc_grads[k]
        top = float(np.abs(o).max())
        den = max(top, 1e-9 * scale, 1e-300)
        out[k] = float(np.abs(g - o).max() / den)
        if elem is not None:
            big = np.abs(o) > 1e-3 * top
            elem[k] = float((np.abs(g - o)[big] / np.abs(o)[big]).max()) if top > 1e-9 * scale and big.any() else 0.0
    return out
