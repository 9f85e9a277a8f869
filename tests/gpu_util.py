"""Helpers shared by the GPU parity tests: move seeded scenes to the device,
build oracle targets, and measure errors the way the parity bar states them
(images: max abs error over non-ambiguous pixels / max |oracle| per channel;
gradients: ||gpu - oracle||_inf / ||oracle||_inf per parameter group)."""
from __future__ import annotations

import numpy as np
import torch

import oracle

IMG_TOL = 1e-5
GRAD_TOL = 1e-4
# residual-sign decisions are flagged within this relative margin (a few
# times the FP32 error of an accumulated image value near 1)
RES_MARGIN = 4e-6


def dev_params(g, device="cuda"):
    from paper_2408_05635_amd.raster import GaussianParams
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)  # noqa: E731
    return GaussianParams(t(g.means), t(g.quats), t(g.log_scales), t(g.opacity_logits).reshape(-1), t(g.rgb))


def dev_poses(views, device="cuda"):
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
    return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device))
            for k, v in d.items()}


def image_errors(gpu: dict, orc, cams, ok: np.ndarray) -> dict:
    """Per-channel relative max error over pixels where ok is true."""
    P = int(sum(c.width * c.height for c in cams))
    out = {}
    rgb_g = gpu["rgb"].double().cpu().numpy()
    offs = 0
    chans = {"r": [], "g": [], "b": []}
    chans_o = {"r": [], "g": [], "b": []}
    okc = []
    for c in cams:
        p = c.width * c.height
        for k, name in enumerate("rgb"):
            chans[name].append(rgb_g[3 * offs + k * p: 3 * offs + (k + 1) * p])
            chans_o[name].append(orc.rgb[3 * offs + k * p: 3 * offs + (k + 1) * p])
        okc.append(ok[offs:offs + p])
        offs += p
    okc = np.concatenate(okc)
    for name in "rgb":
        g = np.concatenate(chans[name])
        o = np.concatenate(chans_o[name])
        out[name] = float(np.abs(g - o)[okc].max(initial=0.0) / max(np.abs(o).max(), 1e-30))
    for name, o in (("depth", orc.depth), ("sil", orc.sil)):
        g = gpu[name].double().cpu().numpy()
        assert g.size == P
        out[name] = float(np.abs(g - o)[ok].max(initial=0.0) / max(np.abs(o).max(), 1e-30))
    return out


def grad_errors(gpu: dict, orc_grads: dict, keys=None) -> dict:
    names = {"means": "g_means", "quats": "g_quats", "log_scales": "g_log_scales",
             "opacity_logits": "g_opacity_logits", "rgb": "g_rgb", "dq_t": "dq_t", "dt": "dt", "dq_c": "dq_c",
             "dc": "dc"}
    out = {}
    # a group whose oracle gradient is rounding noise (e.g. quaternions of
    # isotropic Gaussians, exactly zero in theory) is measured against the
    # largest gradient of all groups instead of against itself
    scale = max(float(np.abs(v).max()) for k, v in orc_grads.items() if k in names)
    for k, gk in names.items():
        if keys is not None and k not in keys:
            continue
        if gpu.get(gk) is None:
            continue
        g = gpu[gk].double().cpu().numpy().reshape(orc_grads[k].shape)
        o = orc_grads[k]
        den = max(float(np.abs(o).max()), 1e-9 * scale, 1e-300)
        out[k] = float(np.abs(g - o).max() / den)
    return out
