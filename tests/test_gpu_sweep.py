"""A seeded sweep of small calls against the oracle: every case draws its
scene, its views (one to three, ragged sizes, each its own pose), the tile
shape and the options (isotropic Gaussians, deterministic or atomic backward,
the silhouette tracking mask, the loss weights), so that combinations no
targeted test picks out get compared too.  The bar and the coverage floors
are those of the targeted parity tests."""
import numpy as np
import pytest

from paper_2408_05635_amd import scenes
from gpu_util import oracle_targets
from test_gpu_parity import _fused_parity, rast  # noqa: F401  (rast: the module fixture)

pytestmark = pytest.mark.gpu

TILES = [(8, 8), (8, 16), (16, 8), (16, 16), (32, 16), (16, 32), (32, 32)]


def _case(seed: int):
    rng = np.random.default_rng(7000 + seed)
    iso = bool(rng.integers(0, 3) == 0)
    base = scenes.tiny_scene(40 + seed, n=int(rng.integers(20, 80)), isotropic=iso, spread=0.6)
    V = int(rng.integers(1, 4))
    cams, qs, ts = [], [], []
    for v in range(V):
        W, H = int(rng.integers(9, 72)), int(rng.integers(7, 56))
        f = 1.1 * max(W, H)
        cams.append(scenes.Camera(W, H, f, f, (W - 1) / 2.0, (H - 1) / 2.0))
        q, t = scenes.perturb_pose(np.array([1.0, 0.0, 0.0, 0.0]), np.zeros(3), 4.0 * v, 0.05 * v,
                                   np.random.default_rng(7100 + 10 * seed + v), np.random.default_rng(7200 + 10 * seed + v))
        qs.append(q)
        ts.append(t)
    target = scenes.Views(cams, np.stack(qs).astype(np.float32), np.stack(ts).astype(np.float32))
    views = scenes._perturbed_views(target, 7300 + seed, 7400 + seed)
    weights = dict(w_rgb=float(rng.choice([0.5, 1.0])), w_depth=float(rng.choice([0.0, 1.0])),
                   w_sil=float(rng.choice([0.0, 1.0])), w_prior=0.0)
    w = scenes.Workload(f"sweep{seed}", base.gaussians, views, target, weights=weights)
    opts = dict(deterministic=bool(rng.integers(0, 2)))
    if rng.integers(0, 4) == 0:
        opts["sil_mask_thresh"] = 0.5
    tile = TILES[int(rng.integers(0, len(TILES)))]
    return w, tile, opts


@pytest.mark.parametrize("seed", range(16))
def test_sweep_case_matches_oracle(rast, seed):
    w, tile, opts = _case(seed)
    label = (f"sweep{seed} views={[(c.width, c.height) for c in w.views.cams]} tile={tile} "
             f"iso={w.gaussians.log_scales.shape[1] == 1} weights={w.weights} {opts}")
    print(label, flush=True)
    _fused_parity(rast, w, oracle_targets(w), label, tile=tile, **opts)
