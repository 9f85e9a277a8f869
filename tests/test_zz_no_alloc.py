"""The allocation-free entry point (gsr_render_loss_grad_noalloc) against the
fused entry point with a caller workspace (gsr_render_loss_grad): the same
kernels on the device's static scratch, two calls in a row, the second on a
smaller input, each compared with the workspace call on the same inputs."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2408_05635_amd import scenes
from gpu_util import GRAD_TOL, dev_params, dev_poses, oracle_targets, to_dev

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 128 << 20


def _opts(w):
    from paper_2408_05635_amd.raster import RenderOptions
    return RenderOptions(**w.weights)


def _compare(a: dict, b: dict, label: str):
    for k in ("rgb", "depth", "sil", "loss", "loss_total"):
        assert torch.equal(a[k], b[k]), (label, k)
    for k in ("g_means", "g_quats", "g_log_scales", "g_opacity_logits", "g_rgb", "dq_t", "dt", "dq_c", "dc"):
        x, y = a[k].double(), b[k].double()
        err = float((x - y).abs().max() / max(float(y.abs().max()), 1e-30))
        assert err <= GRAD_TOL, (label, k, err)
        assert torch.isfinite(x).all(), (label, k)


def test_noalloc_matches_the_workspace_call_twice():
    from paper_2408_05635_amd import raster
    rast = raster.Rasterizer(0)
    ref = raster.Rasterizer(0)
    for label, w in (("config2 view, 100k", scenes.config2(n_views=1, n=100_000)), ("config1", scenes.config1())):
        g = dev_params(w.gaussians)
        q, t = dev_poses(w.views)
        cams = w.views.cams
        tg = to_dev(oracle_targets(w))
        V, P = len(cams), sum(c.width * c.height for c in cams)
        out = rast.alloc_outputs(g, V, P, _opts(w))
        for v in out.values():
            v.fill_(float("nan"))   # every output must be written by the call
        print(f"[noalloc] {label}: n={w.gaussians.n} views={V}", flush=True)
        used = rast.render_loss_grad_noalloc(g, q, t, cams, tg, out, _opts(w))
        torch.cuda.synchronize()
        assert used.ptr and used.bytes == SCRATCH_BYTES and used.pair_capacity > 0
        assert rast.check_overflow(used) is False
        _, k_used, _ = rast.read_counters(used)
        want = ref.render_loss_grad(g, q, t, cams, tg, _opts(w))
        torch.cuda.synchronize()
        assert ref.last_counters[1] == k_used <= used.pair_capacity
        _compare(out, want, label)


def test_noalloc_rejects_calls_beyond_the_scratch():
    from paper_2408_05635_amd import _abi, raster
    rast = raster.Rasterizer(0)
    lib = _abi.load()
    V = 16
    cams = (_abi.Camera * V)(*[_abi.Camera(1200, 680, 600.0, 600.0, 599.5, 339.5) for _ in range(V)])
    q = torch.zeros(V, 4, device="cuda")
    t = torch.zeros(V, 3, device="cuda")
    views = _abi.Views(V, cams, C.c_void_p(q.data_ptr()), C.c_void_p(t.data_ptr()))
    gs = _abi.Gaussians(3_000_000, None, None, None, None, None)
    o = _abi.Options(0.5, 1.0, 1.0, 0.0, 0.2, 0.3, -1.0, 16, 16, 0)
    tg = _abi.Targets(None, None, None, None, None)
    st = lib.gsr_render_loss_grad_noalloc(rast._ctx, C.byref(gs), C.byref(views), C.byref(o), C.byref(tg),
                                          _abi.Images(None, None, None), None, None, None, None, None)
    assert st == _abi.GSR_ENOMEM
    assert b"static scratch" in lib.gsr_last_error(rast._ctx)
    o.flags = _abi.GSR_SYNC
    gs.n = 10
    st = lib.gsr_render_loss_grad_noalloc(rast._ctx, C.byref(gs), C.byref(views), C.byref(o), C.byref(tg),
                                          _abi.Images(None, None, None), None, None, None, None, None)
    assert st == _abi.GSR_EINVAL
