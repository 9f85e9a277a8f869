"""Torch-facing interface of the HIP rasteriser.

torch provides device memory and the stream; every step of the path
(projection, binning, sorting, compositing, loss, backward) runs in
libgsr.so.  There is no CPU or PyTorch fallback: if the library is missing
the import-time load fails loudly.

Conventions (the C ABI's, include/gsr.h): Gaussian parameters are raw
(means [N,3], quats [N,4] wxyz, log_scales [N,3] or [N,1], opacity_logits
[N], rgb [N,3]); poses are world-to-camera quats [V,4] (wxyz) and trans
[V,3]; images of several views are concatenated, RGB planar per view.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

from . import _abi

_ABI = _abi.load()

# the tile shapes gsr_autotune tries (the order of the sizing calls does not matter)
TUNE_TILES = ((8, 8), (8, 16), (16, 8), (16, 16), (32, 16), (16, 32), (32, 32))


@dataclass
class RenderOptions:
    """Loss weights and rasteriser settings (the ABI's gsr_options)."""
    w_rgb: float = 0.5
    w_depth: float = 1.0
    w_sil: float = 1.0
    w_prior: float = 0.0
    z_near: float = 0.2
    blur2d: float = 0.3
    sil_mask_thresh: float = -1.0
    tile: Tuple[int, int] = (16, 16)
    gauss_grads: bool = True
    pose_grads: bool = True
    count_work: bool = False
    pixel_hash: bool = False   # forwards write the decision hash that pixel_state reports
    # the pose translation tensor holds the camera centre C (X_c = R(q)(X - C)); the
    # autograd functions then return dL/dq at fixed C and dL/dC (decoupled update)
    pose_centre: bool = False
    # the library waits after its binning and raises GsrError(GSR_ECAPACITY) on overflow
    sync: bool = False
    # gradients bit-reproducible run to run (fixed-order sums instead of float atomics)
    deterministic: bool = False


@dataclass
class GaussianParams:
    means: torch.Tensor
    quats: torch.Tensor
    log_scales: torch.Tensor
    opacity_logits: torch.Tensor
    rgb: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def isotropic(self) -> bool:
        return self.log_scales.dim() == 2 and self.log_scales.shape[1] == 1

    def tensors(self):
        return (self.means, self.quats, self.log_scales, self.opacity_logits, self.rgb)


@dataclass
class PoseAdam:
    """Step sizes of the decoupled pose update (quaternion, camera centre in metres)."""
    lr_rot: float = 2e-3
    lr_pos: float = 2e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self) -> _abi.PoseAdam:
        return _abi.PoseAdam(self.lr_rot, self.lr_pos, self.beta1, self.beta2, self.eps)


@dataclass
class MapAdam:
    """Step sizes of the map update, one per raw parameter array."""
    lr_means: float = 1e-4
    lr_quats: float = 1e-3
    lr_log_scales: float = 1e-3
    lr_opacity: float = 5e-2
    lr_rgb: float = 2.5e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    def c(self) -> _abi.MapAdam:
        return _abi.MapAdam(self.lr_means, self.lr_quats, self.lr_log_scales, self.lr_opacity, self.lr_rgb,
                            self.beta1, self.beta2, self.eps)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_f32(name: str, t: torch.Tensor, shape, device):
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on {device} (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _loss_ptr(out: dict):
    """Device pointer of the loss buffer of `out`: the library writes V + 1
    float64 values there (per view, then the total)."""
    loss = out["loss"]
    V = int(loss.numel())
    if loss.dtype != torch.float64 or not loss.is_cuda:
        raise TypeError("loss must be a float64 device tensor")
    if loss.untyped_storage().nbytes() < (loss.storage_offset() + V + 1) * 8:
        raise ValueError("the loss buffer needs V + 1 entries (per view, then the total): use alloc_outputs")
    return _ptr(loss)


def _stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class _SizeOnly:
    """A camera of which only the resolution matters (tuning-cache shapes)."""
    width: int
    height: int
    fx: float = 1.0
    fy: float = 1.0
    cx: float = 0.0
    cy: float = 0.0


def total_pixels(cams: Sequence) -> int:
    return int(sum(c.width * c.height for c in cams))


class Rasterizer:
    """Owns a library context and a reusable workspace on one GPU.

    The pair capacity (number of (Gaussian, tile) pairs the workspace holds)
    grows automatically when a checked call overflows it.
    """

    def __init__(self, device=None, pair_capacity: int = 1 << 20):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        self.device = dev
        h = C.c_void_p()
        st = _ABI.gsr_create(C.byref(h), dev.index)
        _abi.check(st, None)
        self._ctx = h
        self.pair_capacity = int(pair_capacity)
        self._ws: Optional[torch.Tensor] = None
        self.last_counters = (0, 0, 0)
        self.tuning: List[dict] = []   # tile choices of autotune()/set_tile(), for save_tuning()

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                _ABI.gsr_destroy(self._ctx)
                self._ctx = None
        except Exception:
            pass

    # ------------------------------------------------------------------ marshalling
    def _views(self, cams, quat, trans):
        V = len(cams)
        arr = (_abi.Camera * V)()
        for k, c in enumerate(cams):
            arr[k] = _abi.Camera(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy))
        _check_f32("pose quat", quat, (V, 4), self.device)
        _check_f32("pose trans", trans, (V, 3), self.device)
        return _abi.Views(V, arr, _ptr(quat), _ptr(trans)), arr

    def _gauss(self, g: GaussianParams):
        n = g.n
        _check_f32("means", g.means, (n, 3), self.device)
        _check_f32("quats", g.quats, (n, 4), self.device)
        _check_f32("log_scales", g.log_scales, (n, 1) if g.isotropic else (n, 3), self.device)
        _check_f32("opacity_logits", g.opacity_logits, (n,), self.device)
        _check_f32("rgb", g.rgb, (n, 3), self.device)
        return _abi.Gaussians(n, *[_ptr(t) for t in g.tensors()])

    @staticmethod
    def _opts(o: RenderOptions, iso: bool, gauss_grads=None, pose_grads=None):
        flags = 0
        if iso:
            flags |= _abi.GSR_ISOTROPIC
        if not (o.gauss_grads if gauss_grads is None else gauss_grads):
            flags |= _abi.GSR_NO_GAUSS_GRADS
        if not (o.pose_grads if pose_grads is None else pose_grads):
            flags |= _abi.GSR_NO_POSE_GRADS
        if o.count_work:
            flags |= _abi.GSR_COUNT_WORK
        if o.pixel_hash:
            flags |= _abi.GSR_PIXEL_HASH
        if o.pose_centre:
            flags |= _abi.GSR_POSE_CENTRE
        if o.sync:
            flags |= _abi.GSR_SYNC
        if o.deterministic:
            flags |= _abi.GSR_DETERMINISTIC
        return _abi.Options(o.w_rgb, o.w_depth, o.w_sil, o.w_prior, o.z_near, o.blur2d, o.sil_mask_thresh,
                            int(o.tile[0]), int(o.tile[1]), flags)

    def workspace_bytes(self, n: int, views, opts, capacity: int) -> int:
        out = C.c_size_t()
        _abi.check(_ABI.gsr_workspace_size(self._ctx, n, C.byref(views), C.byref(opts), capacity, C.byref(out)),
                   self._ctx)
        return int(out.value)

    def new_workspace(self, n: int, views, opts, capacity: int) -> Tuple[torch.Tensor, _abi.Workspace]:
        nbytes = self.workspace_bytes(n, views, opts, capacity)
        buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return buf, _abi.Workspace(buf.data_ptr(), nbytes, capacity)

    def _shared_ws(self, n: int, views, opts) -> _abi.Workspace:
        nbytes = self.workspace_bytes(n, views, opts, self.pair_capacity)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return _abi.Workspace(self._ws.data_ptr(), self._ws.numel(), self.pair_capacity)

    def plan(self, g: GaussianParams, quat, trans, cams, opts: RenderOptions = RenderOptions()) -> int:
        """(Gaussian, tile) pairs the call with these inputs needs (runs the
        binning and synchronises); grows the pair capacity to hold them."""
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic)
        ws = self._shared_ws(g.n, views, o)
        k = C.c_int64()
        st = _ABI.gsr_plan(self._ctx, C.byref(gs), C.byref(views), C.byref(o), ws, C.byref(k), _stream_ptr())
        if st == _abi.GSR_ECAPACITY:
            self._grow(int(k.value))
        else:
            _abi.check(st, self._ctx)
        return int(k.value)

    def check_overflow(self, ws: Optional[_abi.Workspace] = None) -> bool:
        """True if the last call (or loop iteration) on ws overflowed its pair
        capacity (synchronises)."""
        ws = self.shared_workspace() if ws is None else ws
        o = C.c_int32()
        st = _ABI.gsr_check_overflow(self._ctx, ws, _stream_ptr(), C.byref(o))
        if st != _abi.GSR_ECAPACITY:
            _abi.check(st, self._ctx)
        return bool(o.value)

    def read_counters(self, ws: _abi.Workspace) -> Tuple[int, int, int]:
        m, k, o = C.c_int64(), C.c_int64(), C.c_int32()
        _abi.check(_ABI.gsr_read_counters(self._ctx, ws, _stream_ptr(), C.byref(m), C.byref(k), C.byref(o)),
                   self._ctx)
        self.last_counters = (int(m.value), int(k.value), int(o.value))
        return self.last_counters

    def read_work(self, ws: Optional[_abi.Workspace] = None) -> dict:
        """Work counters of the last GSR_COUNT_WORK call (synchronises)."""
        if ws is None:
            ws = _abi.Workspace(self._ws.data_ptr(), self._ws.numel(), self.pair_capacity)
        arr = (C.c_int64 * 6)()
        _abi.check(_ABI.gsr_read_work(self._ctx, ws, _stream_ptr(), arr), self._ctx)
        return dict(eval_fwd=arr[0], contrib_fwd=arr[1], eval_bwd=arr[2], contrib_bwd=arr[3], reduce_bwd=arr[4],
                    work_items=arr[5])

    def set_timing(self, on: bool) -> None:
        _abi.check(_ABI.gsr_set_timing(self._ctx, int(bool(on))), self._ctx)

    def read_timing(self) -> dict:
        """{stage: (total ms, launches)} since the last read (waits for the events)."""
        ms = (C.c_double * 4)()
        cnt = (C.c_int64 * 4)()
        _abi.check(_ABI.gsr_read_timing(self._ctx, ms, cnt), self._ctx)
        return {name: (ms[k], cnt[k]) for k, name in enumerate(_abi.STAGES)}

    def shared_workspace(self) -> Optional[_abi.Workspace]:
        if self._ws is None:
            return None
        return _abi.Workspace(self._ws.data_ptr(), self._ws.numel(), self.pair_capacity)

    def _grow(self, needed: int) -> None:
        self.pair_capacity = max(int(needed * 1.25) + 1024, self.pair_capacity)

    # ------------------------------------------------------------------ calls
    def _fused_args(self, g: GaussianParams, quat, trans, cams, targets: dict, opts: RenderOptions, out: dict):
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic)
        P = total_pixels(cams)
        for k in ("rgb", "depth", "sil", "prior", "weight"):
            t = targets.get(k)
            if t is not None:
                _check_f32(f"target {k}", t, (3 * P,) if k == "rgb" else (P,), self.device)
        tg = _abi.Targets(_ptr(targets["rgb"]), _ptr(targets["depth"]), _ptr(targets.get("sil")),
                          _ptr(targets.get("prior")), _ptr(targets.get("weight")))
        imgs = _abi.Images(_ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["sil"]))
        gg = _abi.GaussGrads(*[_ptr(out.get(k)) for k in ("g_means", "g_quats", "g_log_scales", "g_opacity_logits",
                                                            "g_rgb")])
        pg = _abi.PoseGrads(*[_ptr(out.get(k)) for k in ("dq_t", "dt", "dq_c", "dc")])
        return dict(views=views, keep=keep, gs=gs, o=o, tg=tg, imgs=imgs, gg=gg, pg=pg)

    def autotune(self, g: GaussianParams, quat, trans, cams, targets: dict, opts: RenderOptions = RenderOptions(),
                 reps: int = 5, out: Optional[dict] = None) -> Tuple[Tuple[int, int], float]:
        """Time every tile size on these inputs and keep the fastest for this
        shape (later calls with opts.tile == (0, 0) use it).  The workspace is
        first sized for the tile that needs the most pairs."""
        V = len(cams)
        P = total_pixels(cams)
        if out is None:
            out = self.alloc_outputs(g, V, P, opts)
        for tile in TUNE_TILES:
            self.render_loss_grad(g, quat, trans, cams, targets, RenderOptions(**{**opts.__dict__, "tile": tile}),
                                  check=True, out=out)
        a = self._fused_args(g, quat, trans, cams, targets, opts, out)
        ws = self._shared_ws(g.n, a["views"], self._opts(RenderOptions(**{**opts.__dict__, "tile": (8, 8)}),
                                                          g.isotropic))
        best = (C.c_int32 * 2)()
        ms = C.c_double()
        _abi.check(_ABI.gsr_autotune(self._ctx, C.byref(a["gs"]), C.byref(a["views"]), C.byref(a["o"]),
                                     C.byref(a["tg"]), ws, a["imgs"], _loss_ptr(out), C.byref(a["gg"]),
                                     C.byref(a["pg"]), int(reps), best, C.byref(ms), _stream_ptr()), self._ctx)
        tile = (int(best[0]), int(best[1]))
        self._remember(g.n, cams, tile, g.isotropic, opts.gauss_grads, opts.pose_grads, float(ms.value))
        return tile, float(ms.value)

    def _remember(self, n, cams, tile, isotropic, gauss_grads, pose_grads, ms=None):
        e = dict(n=int(n), sizes=[[int(c.width), int(c.height)] for c in cams], tile=list(tile),
                 isotropic=bool(isotropic), gauss_grads=bool(gauss_grads), pose_grads=bool(pose_grads))
        self.tuning = [x for x in self.tuning if {**x, "tile": None, "ms": None} != {**e, "tile": None, "ms": None}]
        if ms is not None:
            e["ms"] = ms
        self.tuning.append(e)

    def save_tuning(self, path: str) -> None:
        """Writes the tile choices made in this process (autotune, set_tile)
        as JSON, for load_tuning() in a later one."""
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump({"tiles": self.tuning}, fh, indent=1)
        os.replace(tmp, path)

    def load_tuning(self, path: str) -> int:
        """Applies the tile choices of a save_tuning() file through gsr_set_tile
        (calls with tile (0, 0) then use them); returns how many it applied."""
        with open(path) as fh:
            entries = json.load(fh)["tiles"]
        for e in entries:
            cams = [_SizeOnly(w, h) for w, h in e["sizes"]]
            self.set_tile(e["n"], cams, tuple(e["tile"]), e["isotropic"], e["gauss_grads"], e["pose_grads"])
        return len(entries)

    def set_tile(self, n: int, cams, tile: Tuple[int, int], isotropic=False, gauss_grads=True, pose_grads=True):
        """Record a tile choice for a shape (e.g. loaded from a tuning cache):
        the Gaussian count's power-of-two class, the views' resolutions and
        the gradient and isotropy flags form the shape."""
        V = len(cams)
        arr = (_abi.Camera * V)(*[_abi.Camera(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx),
                                              float(c.cy)) for c in cams])
        views = _abi.Views(V, arr, None, None)
        flags = (_abi.GSR_ISOTROPIC if isotropic else 0) | (0 if gauss_grads else _abi.GSR_NO_GAUSS_GRADS) | \
            (0 if pose_grads else _abi.GSR_NO_POSE_GRADS)
        _abi.check(_ABI.gsr_set_tile(self._ctx, n, C.byref(views), flags, int(tile[0]), int(tile[1])), self._ctx)
        self._remember(n, cams, tile, isotropic, gauss_grads, pose_grads)

    def capture_graph(self, g: GaussianParams, quat, trans, cams, targets: dict,
                      opts: RenderOptions = RenderOptions(), out: Optional[dict] = None):
        """Capture one fused call into a HIP graph; returns (graph id, out).
        Every tensor passed (and the workspace) must stay alive and in place
        while the graph is used."""
        V = len(cams)
        P = total_pixels(cams)
        if out is None:
            out = self.alloc_outputs(g, V, P, opts)
        self.render_loss_grad(g, quat, trans, cams, targets, opts, check=True, out=out)   # size the capacity
        a = self._fused_args(g, quat, trans, cams, targets, opts, out)
        ws = self._shared_ws(g.n, a["views"], a["o"])
        gid = C.c_int32()
        _abi.check(_ABI.gsr_graph_capture(self._ctx, C.byref(a["gs"]), C.byref(a["views"]), C.byref(a["o"]),
                                          C.byref(a["tg"]), ws, a["imgs"], _loss_ptr(out), C.byref(a["gg"]),
                                          C.byref(a["pg"]), _stream_ptr(), C.byref(gid)), self._ctx)
        self._graph_refs = getattr(self, "_graph_refs", {})
        self._graph_refs[gid.value] = (a, out, self._ws)
        return gid.value, out

    def launch_graph(self, graph_id: int) -> None:
        _abi.check(_ABI.gsr_graph_launch(self._ctx, int(graph_id), _stream_ptr()), self._ctx)

    def destroy_graph(self, graph_id: int) -> None:
        _abi.check(_ABI.gsr_graph_destroy(self._ctx, int(graph_id)), self._ctx)
        getattr(self, "_graph_refs", {}).pop(graph_id, None)

    def render_loss_grad(self, g: GaussianParams, quat: torch.Tensor, trans: torch.Tensor, cams: Sequence,
                         targets: dict, opts: RenderOptions = RenderOptions(), check: bool = True,
                         out: Optional[dict] = None):
        """Forward + fused loss + backward.  Returns a dict with rgb, depth, sil,
        loss [V] (float64) and the gradients (None where switched off).
        With check=True the call synchronises once to verify the pair
        capacity (and re-runs after growing it if needed); pass check=False
        for capture in a graph or for timing loops, and verify afterwards."""
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic)
        P = total_pixels(cams)
        V = len(cams)
        if out is None:
            out = self.alloc_outputs(g, V, P, opts)
        tg = _abi.Targets(_ptr(targets["rgb"]), _ptr(targets["depth"]), _ptr(targets.get("sil")),
                          _ptr(targets.get("prior")), _ptr(targets.get("weight")))
        for k in ("rgb", "depth", "sil", "prior", "weight"):
            t = targets.get(k)
            if t is not None:
                _check_f32(f"target {k}", t, (3 * P,) if k == "rgb" else (P,), self.device)
        while True:
            ws = self._shared_ws(g.n, views, o)
            imgs = _abi.Images(_ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["sil"]))
            gg = _abi.GaussGrads(*[_ptr(out.get(k)) for k in ("g_means", "g_quats", "g_log_scales",
                                                                "g_opacity_logits", "g_rgb")])
            pg = _abi.PoseGrads(*[_ptr(out.get(k)) for k in ("dq_t", "dt", "dq_c", "dc")])
            st = _ABI.gsr_render_loss_grad(self._ctx, C.byref(gs), C.byref(views), C.byref(o), C.byref(tg), ws,
                                           imgs, _loss_ptr(out), C.byref(gg), C.byref(pg), _stream_ptr())
            _abi.check(st, self._ctx)
            if not check:
                break
            _, k, ovf = self.read_counters(ws)
            if not ovf:
                break
            self._grow(k)
        return out

    def render_loss_grad_noalloc(self, g: GaussianParams, quat: torch.Tensor, trans: torch.Tensor, cams: Sequence,
                                 targets: dict, out: dict, opts: RenderOptions = RenderOptions()) -> _abi.Workspace:
        """gsr_render_loss_grad_noalloc: the fused call on the device's static
        scratch (the library allocates nothing; `out` comes from
        alloc_outputs).  Returns the workspace the call used, for
        check_overflow() and read_counters()."""
        a = self._fused_args(g, quat, trans, cams, targets, opts, out)
        used = _abi.Workspace()
        _abi.check(_ABI.gsr_render_loss_grad_noalloc(self._ctx, C.byref(a["gs"]), C.byref(a["views"]),
                                                     C.byref(a["o"]), C.byref(a["tg"]), a["imgs"], _loss_ptr(out),
                                                     C.byref(a["gg"]), C.byref(a["pg"]), _stream_ptr(),
                                                     C.byref(used)), self._ctx)
        return used

    def alloc_outputs(self, g: GaussianParams, V: int, P: int, opts: RenderOptions) -> dict:
        """Output tensors of a fused call.  The library writes V + 1 losses (per
        view, then their total): `loss` is the per-view view [V] of that
        buffer and `loss_total` its last entry."""
        dev = self.device
        e = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)  # noqa: E731
        lbuf = torch.empty(V + 1, dtype=torch.float64, device=dev)
        out = dict(rgb=e(3 * P), depth=e(P), sil=e(P), loss=lbuf[:V], loss_total=lbuf[V])
        n = g.n
        if opts.gauss_grads:
            out.update(g_means=e(n, 3), g_quats=e(n, 4), g_log_scales=e(*g.log_scales.shape),
                       g_opacity_logits=e(n), g_rgb=e(n, 3))
        if opts.pose_grads:
            out.update(dq_t=e(V, 4), dt=e(V, 3), dq_c=e(V, 4), dc=e(V, 3))
        return out

    def forward(self, g: GaussianParams, quat, trans, cams, opts: RenderOptions = RenderOptions(),
                ws_pair: Optional[Tuple[torch.Tensor, _abi.Workspace]] = None, check: bool = True):
        """Render only.  Returns (rgb, depth, sil, (ws_tensor, ws)): the
        workspace holds the state that backward() needs."""
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic)
        P = total_pixels(cams)
        rgb = torch.empty(3 * P, dtype=torch.float32, device=self.device)
        depth = torch.empty(P, dtype=torch.float32, device=self.device)
        sil = torch.empty(P, dtype=torch.float32, device=self.device)
        while True:
            if ws_pair is None:
                ws_pair = self.new_workspace(g.n, views, o, self.pair_capacity)
            imgs = _abi.Images(_ptr(rgb), _ptr(depth), _ptr(sil))
            _abi.check(_ABI.gsr_forward(self._ctx, C.byref(gs), C.byref(views), C.byref(o), ws_pair[1], imgs,
                                        _stream_ptr()), self._ctx)
            if not check:
                break
            _, k, ovf = self.read_counters(ws_pair[1])
            if not ovf:
                break
            self._grow(k)
            ws_pair = None
        return rgb, depth, sil, ws_pair

    def backward(self, g: GaussianParams, quat, trans, cams, opts: RenderOptions, ws_pair, images,
                 g_rgb=None, g_depth=None, g_sil=None, gauss_grads: bool = True, pose_grads: bool = True):
        """Backward of forward(): upstream image gradients -> parameter and pose gradients."""
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic, gauss_grads, pose_grads)
        P = total_pixels(cams)
        V = len(cams)
        for name, t, shp in (("g_rgb", g_rgb, (3 * P,)), ("g_depth", g_depth, (P,)), ("g_sil", g_sil, (P,))):
            if t is not None:
                _check_f32(name, t, shp, self.device)
        dev = self.device
        e = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)  # noqa: E731
        gr = {}
        if gauss_grads:
            gr = dict(means=e(g.n, 3), quats=e(g.n, 4), log_scales=e(*g.log_scales.shape),
                      opacity_logits=e(g.n), rgb=e(g.n, 3))
        pr = {}
        if pose_grads:
            pr = dict(dq_t=e(V, 4), dt=e(V, 3), dq_c=e(V, 4), dc=e(V, 3))
        gg = _abi.GaussGrads(*[_ptr(gr.get(k)) for k in ("means", "quats", "log_scales", "opacity_logits", "rgb")])
        pg = _abi.PoseGrads(*[_ptr(pr.get(k)) for k in ("dq_t", "dt", "dq_c", "dc")])
        imgs = _abi.Images(*[_ptr(t) for t in images])
        _abi.check(_ABI.gsr_backward(self._ctx, C.byref(gs), C.byref(views), C.byref(o), ws_pair[1], imgs,
                                     _ptr(g_rgb), _ptr(g_depth), _ptr(g_sil), C.byref(gg), C.byref(pg),
                                     _stream_ptr()), self._ctx)
        return gr, pr

    def debug_binning(self, g: GaussianParams, quat, trans, cams, opts: RenderOptions, ws: _abi.Workspace):
        """Copies the binning state of the last call on ws (for bit-exact tests)."""
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic)
        M, K, ovf = self.read_counters(ws)
        tw, th = opts.tile
        T = sum(((c.width + tw - 1) // tw) * ((c.height + th - 1) // th) for c in cams)
        dev = self.device
        gid = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
        xy = torch.empty(max(M, 1), 2, dtype=torch.float32, device=dev)
        rad = torch.empty(max(M, 1), dtype=torch.float32, device=dev)
        z = torch.empty(max(M, 1), dtype=torch.float32, device=dev)
        ranges = torch.empty(max(T, 1), 2, dtype=torch.int32, device=dev)
        pairs = torch.empty(max(K, 1), dtype=torch.int32, device=dev)
        _abi.check(_ABI.gsr_debug_binning(self._ctx, C.byref(gs), C.byref(views), C.byref(o), ws, M, T, K,
                                          _ptr(gid), _ptr(xy), _ptr(rad), _ptr(z), _ptr(ranges), _ptr(pairs),
                                          _stream_ptr()), self._ctx)
        torch.cuda.current_stream().synchronize()
        return dict(M=M, K=K, overflow=ovf, gid=gid[:M].cpu(), xy=xy[:M].cpu(), radius=rad[:M].cpu(),
                    z=z[:M].cpu(), ranges=ranges[:T].cpu(), pairs=pairs[:K].cpu())

    def pixel_state(self, g: GaussianParams, quat, trans, cams, opts: RenderOptions,
                    ws: Optional[_abi.Workspace] = None) -> dict:
        """Per-pixel final transmittance, last contributor and decision hash
        left by the last call on ws (default: the shared workspace)."""
        views, keep = self._views(cams, quat, trans)
        gs = self._gauss(g)
        o = self._opts(opts, g.isotropic)
        ws = self.shared_workspace() if ws is None else ws
        P = total_pixels(cams)
        dev = self.device
        t_final = torch.empty(P, dtype=torch.float32, device=dev)
        n_last = torch.empty(P, dtype=torch.int32, device=dev)
        hsh = torch.empty(P, dtype=torch.int32, device=dev)
        _abi.check(_ABI.gsr_debug_pixel_state(self._ctx, C.byref(gs), C.byref(views), C.byref(o), ws, _ptr(t_final),
                                              _ptr(n_last), _ptr(hsh), _stream_ptr()), self._ctx)
        return dict(t_final=t_final, n_last=n_last, hash=hsh)

    # ------------------------------------------------------------------ optimisation steps
    def pose_opt_init(self, quat: torch.Tensor, trans: torch.Tensor) -> torch.Tensor:
        """Optimiser state [V, GSR_POSE_STATE_DOUBLES] (float64) for the poses."""
        V = int(quat.shape[0])
        _check_f32("pose quat", quat, (V, 4), self.device)
        _check_f32("pose trans", trans, (V, 3), self.device)
        state = torch.empty(V, _abi.GSR_POSE_STATE_DOUBLES, dtype=torch.float64, device=self.device)
        _abi.check(_ABI.gsr_pose_opt_init(self._ctx, V, _ptr(quat), _ptr(trans), _ptr(state), _stream_ptr()),
                   self._ctx)
        return state

    def pose_opt_step(self, state: torch.Tensor, dq_c: torch.Tensor, dc: torch.Tensor, quat: torch.Tensor,
                      trans: torch.Tensor, hp: PoseAdam = PoseAdam()) -> None:
        """One decoupled step; rewrites quat and trans in place."""
        V = int(quat.shape[0])
        for name, t, shp in (("dq_c", dq_c, (V, 4)), ("dc", dc, (V, 3)), ("pose quat", quat, (V, 4)),
                             ("pose trans", trans, (V, 3))):
            _check_f32(name, t, shp, self.device)
        hpc = hp.c()
        _abi.check(_ABI.gsr_pose_opt_step(self._ctx, V, _ptr(dq_c), _ptr(dc), C.byref(hpc), _ptr(state), _ptr(quat),
                                          _ptr(trans), _stream_ptr()), self._ctx)

    def _track_args(self, g, quat, trans, cams, targets, opts, hp, state, iters, out, hist):
        a = self._fused_args(g, quat, trans, cams, targets, opts, out)
        ws = self._shared_ws(g.n, a["views"], self._opts(opts, g.isotropic, gauss_grads=False))
        hpc = hp.c()
        args = [self._ctx, C.byref(a["gs"]), a["views"].cams, len(cams), _ptr(quat), _ptr(trans), C.byref(a["o"]),
                C.byref(a["tg"]), ws, a["imgs"], _loss_ptr(out), C.byref(a["pg"]), C.byref(hpc), _ptr(state),
                int(iters), _ptr(hist), _stream_ptr()]
        return args, (a, hpc, ws)

    def track(self, g: GaussianParams, quat: torch.Tensor, trans: torch.Tensor, cams: Sequence, targets: dict,
              opts: RenderOptions = RenderOptions(), hp: PoseAdam = PoseAdam(), iters: int = 40,
              state: Optional[torch.Tensor] = None, capture: bool = False, out: Optional[dict] = None):
        """The tracking loop on the device: `iters` x (render + loss + pose
        gradients, decoupled Adam step).  quat/trans are updated in place.
        Returns dict(loss_hist [iters, V] float64, state, out, graph (id or None)).
        Eagerly, the pair capacity is checked after the loop and the loop is
        re-run from its start if any iteration overflowed it; with capture=True
        the loop is captured (not run) and the caller checks read_counters after
        replays."""
        V = len(cams)
        P = total_pixels(cams)
        opts = RenderOptions(**{**opts.__dict__, "gauss_grads": False, "pose_grads": True})
        if out is None:
            out = self.alloc_outputs(g, V, P, opts)
        if state is None:
            state = self.pose_opt_init(quat, trans)
        hist = torch.zeros(max(iters, 1), V, dtype=torch.float64, device=self.device)
        self.render_loss_grad(g, quat, trans, cams, targets, opts, check=True, out=out)   # size the capacity
        if capture:
            args, keep = self._track_args(g, quat, trans, cams, targets, opts, hp, state, iters, out, hist)
            gid = C.c_int32()
            _abi.check(_ABI.gsr_track_capture(*args, C.byref(gid)), self._ctx)
            self._graph_refs = getattr(self, "_graph_refs", {})
            self._graph_refs[gid.value] = (keep, out, hist, state, self._ws)
            return dict(loss_hist=hist[:iters], state=state, out=out, graph=gid.value)
        q0, t0, s0 = quat.clone(), trans.clone(), state.clone()
        while True:
            args, keep = self._track_args(g, quat, trans, cams, targets, opts, hp, state, iters, out, hist)
            _abi.check(_ABI.gsr_track(*args), self._ctx)
            _, k, ovf = self.read_counters(keep[2])
            if not ovf:
                break
            self._grow(k)
            quat.copy_(q0)
            trans.copy_(t0)
            state.copy_(s0)
        return dict(loss_hist=hist[:iters], state=state, out=out, graph=None)

    def map_opt_init(self, g: GaussianParams) -> torch.Tensor:
        """Zeroed mapping optimiser state (bytes) for g."""
        nbytes = int(_ABI.gsr_map_state_size(g.n, int(g.isotropic)))
        state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _abi.check(_ABI.gsr_map_opt_init(self._ctx, g.n, int(g.isotropic), _ptr(state), _stream_ptr()), self._ctx)
        return state

    def map_opt_step(self, g: GaussianParams, grads: dict, state: torch.Tensor, hp: MapAdam = MapAdam()) -> None:
        """One Adam step over g's arrays in place; grads holds g_means, g_quats,
        g_log_scales, g_opacity_logits, g_rgb (as returned by the backward)."""
        self._gauss(g)
        keys = ("means", "quats", "log_scales", "opacity_logits", "rgb")
        for k in keys:
            _check_f32("g_" + k, grads["g_" + k], tuple(getattr(g, k).shape), self.device)
        rw = _abi.GaussiansRW(g.n, *[_ptr(getattr(g, k)) for k in keys])
        gg = _abi.GaussGrads(*[_ptr(grads["g_" + k]) for k in keys])
        hpc = hp.c()
        _abi.check(_ABI.gsr_map_opt_step(self._ctx, rw, C.byref(gg), int(g.isotropic), C.byref(hpc), _ptr(state),
                                         _stream_ptr()), self._ctx)

    def map_iterate(self, g: GaussianParams, quat: torch.Tensor, trans: torch.Tensor, cams: Sequence,
                    targets: dict, opts: RenderOptions = RenderOptions(), hp: MapAdam = MapAdam(), iters: int = 10,
                    state: Optional[torch.Tensor] = None, capture: bool = False, out: Optional[dict] = None):
        """The mapping loop on the device: `iters` x (render + loss + Gaussian
        gradients over the views, Adam step of the map); g's arrays are updated
        in place.  Returns dict(loss_hist [iters, V] float64, state, out, graph).
        Eagerly, the pair capacity is checked after the loop and the loop re-run
        from its start if any iteration overflowed it; with capture=True the loop
        is captured (not run)."""
        V = len(cams)
        P = total_pixels(cams)
        opts = RenderOptions(**{**opts.__dict__, "gauss_grads": True, "pose_grads": False})
        if out is None:
            out = self.alloc_outputs(g, V, P, opts)
        if state is None:
            state = self.map_opt_init(g)
        hist = torch.zeros(max(iters, 1), V, dtype=torch.float64, device=self.device)
        self.render_loss_grad(g, quat, trans, cams, targets, opts, check=True, out=out)   # size the capacity

        def args():
            a = self._fused_args(g, quat, trans, cams, targets, opts, out)
            ws = self._shared_ws(g.n, a["views"], a["o"])
            hpc = hp.c()
            rw = _abi.GaussiansRW(g.n, *[_ptr(t) for t in g.tensors()])
            return [self._ctx, rw, C.byref(a["views"]), C.byref(a["o"]), C.byref(a["tg"]), ws, a["imgs"],
                    _loss_ptr(out), C.byref(a["gg"]), C.byref(hpc), _ptr(state), int(iters), _ptr(hist),
                    _stream_ptr()], (a, hpc, ws, rw)

        if capture:
            al, keep = args()
            gid = C.c_int32()
            _abi.check(_ABI.gsr_map_capture(*al, C.byref(gid)), self._ctx)
            self._graph_refs = getattr(self, "_graph_refs", {})
            self._graph_refs[gid.value] = (keep, out, hist, state, self._ws)
            return dict(loss_hist=hist[:iters], state=state, out=out, graph=gid.value)
        saved = [t.clone() for t in g.tensors()] + [state.clone()]
        while True:
            al, keep = args()
            _abi.check(_ABI.gsr_map_iterate(*al), self._ctx)
            _, k, ovf = self.read_counters(keep[2])
            if not ovf:
                break
            self._grow(k)
            for t, s0 in zip(list(g.tensors()) + [state], saved):
                t.copy_(s0)
        return dict(loss_hist=hist[:iters], state=state, out=out, graph=None)

    def densify(self, cam, quat: torch.Tensor, trans: torch.Tensor, rgb: torch.Tensor, depth: torch.Tensor,
                sil: Optional[torch.Tensor], out: GaussianParams, offset: int, sil_thresh: float = 0.5,
                n_new: Optional[torch.Tensor] = None) -> torch.Tensor:
        """New Gaussians from one RGB-D frame written into rows offset.. of
        `out` (its row count is the capacity).  Returns the device count
        (int64 [1]) of qualifying pixels, written or not."""
        P = int(cam.width) * int(cam.height)
        _check_f32("quat", quat, (4,), self.device)
        _check_f32("trans", trans, (3,), self.device)
        _check_f32("rgb", rgb, (3 * P,), self.device)
        _check_f32("depth", depth, (P,), self.device)
        if sil is not None:
            _check_f32("sil", sil, (P,), self.device)
        self._gauss(out)
        if n_new is None:
            n_new = torch.zeros(1, dtype=torch.int64, device=self.device)
        wb = int(_ABI.gsr_densify_work_size(int(cam.width), int(cam.height)))
        work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        camc = _abi.Camera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                           float(cam.cy))
        rw = _abi.GaussiansRW(out.n, *[_ptr(t) for t in out.tensors()])
        _abi.check(_ABI.gsr_densify(self._ctx, camc, _ptr(quat), _ptr(trans), _ptr(rgb), _ptr(depth), _ptr(sil),
                                    float(sil_thresh), rw, int(out.isotropic), int(offset), int(out.n), _ptr(n_new),
                                    _ptr(work), wb, _stream_ptr()), self._ctx)
        self._densify_keep = work
        return n_new

    def selftest(self) -> int:
        d = torch.empty(1, dtype=torch.int32, device=self.device)
        _abi.check(_ABI.gsr_selftest(self._ctx, _ptr(d), _stream_ptr()), self._ctx)
        return int(d.item())


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
def _pose_grads(pr: dict, opts: RenderOptions):
    """The gradients of the pose tensors as passed: (dL/dq at fixed t, dL/dt),
    or with opts.pose_centre, where the translation tensor is the camera centre,
    (dL/dq at fixed C, dL/dC)."""
    if opts.pose_centre:
        return pr.get("dq_c"), pr.get("dc")
    return pr.get("dq_t"), pr.get("dt")


class _RenderFn(torch.autograd.Function):
    """Images as a differentiable function of the Gaussians and the poses.
    The workspace holding the forward state travels in ctx."""

    @staticmethod
    def forward(ctx, means, quats, log_scales, opacity_logits, rgb, pose_q, pose_t, rast, cams, opts, check):
        g = GaussianParams(means.detach(), quats.detach(), log_scales.detach(), opacity_logits.detach(),
                           rgb.detach())
        img, depth, sil, ws_pair = rast.forward(g, pose_q.detach(), pose_t.detach(), cams, opts, check=check)
        ctx.rast, ctx.cams, ctx.opts, ctx.ws_pair = rast, cams, opts, ws_pair
        ctx.save_for_backward(means, quats, log_scales, opacity_logits, rgb, pose_q, pose_t, img, depth, sil)
        return img, depth, sil

    @staticmethod
    def backward(ctx, g_img, g_depth, g_sil):
        means, quats, log_scales, opacity_logits, rgb, pose_q, pose_t, img, depth, sil = ctx.saved_tensors
        g = GaussianParams(means, quats, log_scales, opacity_logits, rgb)
        need_g = any(ctx.needs_input_grad[:5])
        need_p = any(ctx.needs_input_grad[5:7])
        cont = lambda t: None if t is None else t.contiguous()  # noqa: E731
        gr, pr = ctx.rast.backward(g, pose_q, pose_t, ctx.cams, ctx.opts, ctx.ws_pair, (img, depth, sil),
                                   cont(g_img), cont(g_depth), cont(g_sil), gauss_grads=need_g, pose_grads=need_p)
        ctx.ws_pair = None
        gq, gt = _pose_grads(pr, ctx.opts)
        return (gr.get("means"), gr.get("quats"), gr.get("log_scales"), gr.get("opacity_logits"), gr.get("rgb"),
                gq, gt, None, None, None, None)


def render(rast: Rasterizer, g: GaussianParams, pose_q: torch.Tensor, pose_t: torch.Tensor, cams: Sequence,
           opts: RenderOptions = RenderOptions(), check: bool = True):
    """(rgb [3*sumP], depth [sumP], sil [sumP]) with autograd to every input
    tensor.  With opts.pose_centre, pose_t is the camera centre C and its
    gradient dL/dC (the pose_q gradient is then taken at fixed C).  check=False
    skips the host synchronisation that verifies the pair capacity (for
    timing loops and graph capture; verify with rast.check_overflow())."""
    return _RenderFn.apply(g.means, g.quats, g.log_scales, g.opacity_logits, g.rgb, pose_q, pose_t, rast,
                           list(cams), opts, check)


class _RenderLossFn(torch.autograd.Function):
    """The fused loss: the library computes the loss (per view and their FP64
    total) and, in the same kernels, all its gradients; backward scales them
    by the upstream scalar."""

    @staticmethod
    def forward(ctx, means, quats, log_scales, opacity_logits, rgb, pose_q, pose_t, rast, cams, targets, opts, check):
        g = GaussianParams(means.detach(), quats.detach(), log_scales.detach(), opacity_logits.detach(),
                           rgb.detach())
        o = RenderOptions(**{**opts.__dict__})
        o.gauss_grads = any(ctx.needs_input_grad[:5])
        o.pose_grads = any(ctx.needs_input_grad[5:7])
        out = rast.render_loss_grad(g, pose_q.detach(), pose_t.detach(), cams, targets, o, check=check)
        ctx.out, ctx.opts = out, o
        return out["loss_total"]

    @staticmethod
    def backward(ctx, gl):
        out = ctx.out
        s = lambda t: None if t is None else t * gl.to(t.dtype)  # noqa: E731
        gq, gt = _pose_grads(out, ctx.opts)
        return (s(out.get("g_means")), s(out.get("g_quats")), s(out.get("g_log_scales")),
                s(out.get("g_opacity_logits")), s(out.get("g_rgb")), s(gq), s(gt), None, None, None, None, None)


def render_loss(rast: Rasterizer, g: GaussianParams, pose_q, pose_t, cams, targets: dict,
                opts: RenderOptions = RenderOptions(), check: bool = True):
    """The combined objective (sum over the views of the per-view losses, as
    the library's FP64 total: a float64 scalar), differentiable.  With
    opts.pose_centre, pose_t is the camera centre C (see render()).
    check=False skips the host synchronisation of the pair-capacity check."""
    return _RenderLossFn.apply(g.means, g.quats, g.log_scales, g.opacity_logits, g.rgb, pose_q, pose_t, rast,
                               list(cams), targets, opts, check)
