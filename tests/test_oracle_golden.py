"""The oracle against its committed regression record (tests/golden/oracle_tiny.json,
written by tests/golden/make_golden.py from the oracle alone): a change of the
oracle's arithmetic shows up here and has to be made on purpose."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2408_05635_amd import scenes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_tiny.json")
REL = 1e-12   # summation order across the oracle's threads moves only the last bits


def _close(a, b, label, floor=1e-300):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    assert a.shape == b.shape, (label, a.shape, b.shape)
    scale = max(float(np.abs(b).max()), floor)
    err = float(np.abs(a - b).max()) / scale
    assert err <= REL, f"{label}: {err:.3e} relative to its largest value"


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: f"seed{c['seed']}")
def test_oracle_matches_its_regression_record(case):
    w = scenes.tiny_scene(case["seed"], isotropic=case["isotropic"])
    tgt = oracle.run(w.gaussians, w.target_views)
    targets = oracle.Targets(rgb=tgt.rgb, depth=tgt.depth, sil=tgt.sil)
    r = oracle.run(w.gaussians, w.views, oracle.Options(**w.weights), targets, want_grads=True)
    s = case["stride"]
    for name in ("rgb", "depth", "sil"):
        _close(getattr(r, name)[::s], case[name], name)
    _close(r.loss, case["loss"], "loss")
    assert set(r.grads) == set(case["grads"])
    # a group that is rounding noise (the quaternions of isotropic Gaussians,
    # zero in theory) is measured against the largest gradient of all groups
    top = max(float(np.abs(np.asarray(v)).max()) for v in case["grads"].values())
    for k, v in r.grads.items():
        _close(np.asarray(v).reshape(-1), case["grads"][k], f"grad {k}", floor=1e-4 * top)
