"""The parity helpers refuse a comparison that covers no pixel, or fewer than
its floor, so a GPU parity test cannot pass by comparing nothing (CPU only:
the helpers are fed host arrays)."""
import numpy as np
import pytest

from gpu_util import ParityCoverageError, grad_errors, image_errors, require_coverage


class _Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


class _Res:
    pass


def _images(P, rng):
    r = _Res()
    r.rgb = rng.uniform(0.1, 1.0, 3 * P)
    r.depth = rng.uniform(0.5, 3.0, P)
    r.sil = rng.uniform(0.1, 1.0, P)
    return r


def test_require_coverage_floors():
    m = np.zeros(100, bool)
    with pytest.raises(ParityCoverageError):
        require_coverage(m, 0.0, "empty")
    m[:89] = True
    with pytest.raises(ParityCoverageError):
        require_coverage(m, 0.9, "89%")
    m[89] = True
    assert require_coverage(m, 0.9, "90%") == 90


def test_image_errors_refuses_an_all_masked_comparison():
    rng = np.random.default_rng(0)
    cams = [_Cam(8, 4), _Cam(4, 2)]
    P = 40
    o = _images(P, rng)
    g = {"rgb": o.rgb.copy(), "depth": o.depth.copy(), "sil": o.sil.copy()}
    with pytest.raises(ParityCoverageError):
        image_errors(g, o, cams, np.zeros(P, bool))
    with pytest.raises(ParityCoverageError):
        image_errors(g, o, cams, np.arange(P) < 10, floor=0.5)


def test_image_errors_measure_on_the_selected_pixels_only():
    rng = np.random.default_rng(1)
    cams = [_Cam(8, 4), _Cam(4, 2)]
    P = 40
    o = _images(P, rng)
    g = {"rgb": o.rgb.copy(), "depth": o.depth.copy(), "sil": o.sil.copy()}
    # a large error on pixel 5 of view 1's green plane (planar per view)
    idx = 3 * 32 + 8 + 5
    g["rgb"][idx] += 0.5
    ok = np.ones(P, bool)
    e = image_errors(g, o, cams, ok)
    scale = max(o.rgb[3 * 32 + 8: 3 * 32 + 16].max(), o.rgb[32:64].max())
    assert e["g"] == pytest.approx(0.5 / scale) and e["r"] == 0 and e["depth"] == 0
    ok[32 + 5] = False       # that pixel masked: no error left
    assert image_errors(g, o, cams, ok)["g"] == 0.0


def test_grad_errors_refuse_all_zero_oracle_gradients():
    with pytest.raises(AssertionError):
        grad_errors({"g_means": np.zeros((3, 3))}, {"means": np.zeros((3, 3))})
    elem = {}
    o = {"means": np.array([[1.0, 1e-2, 1e-5]])}
    e = grad_errors({"g_means": np.array([[1.0, 1.1e-2, 2e-5]])}, o, elem=elem)
    assert e["means"] == pytest.approx(1e-3)
    assert elem["means"] == pytest.approx(0.1)    # the 1e-5 entry is below 1e-3 of the max: not counted
