"""Writes tests/golden/oracle_tiny.json: the FP64 oracle's outputs on two seeded
tiny scenes (one anisotropic, one isotropic) -- images at every fifth pixel,
the per-view loss and every gradient -- as a regression record of the oracle.

It calls only `oracle` and the seeded scene generators (which hold no method
arithmetic).  The record pins the oracle to its own committed behaviour, not to
the paper: the paper prints no worked example, and the oracle's pins against
closed forms, brute force and finite differences live in test_oracle_pins.py.
A change of the oracle's arithmetic that moves these numbers is deliberate and
regenerates the file with this script.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2408_05635_amd import scenes  # noqa: E402

CASES = [dict(seed=5, isotropic=False), dict(seed=6, isotropic=True)]
STRIDE = 5


def case_outputs(seed: int, isotropic: bool) -> dict:
    w = scenes.tiny_scene(seed, isotropic=isotropic)
    tgt = oracle.run(w.gaussians, w.target_views)
    targets = oracle.Targets(rgb=tgt.rgb, depth=tgt.depth, sil=tgt.sil)
    opts = oracle.Options(**{k: v for k, v in w.weights.items()})
    r = oracle.run(w.gaussians, w.views, opts, targets, want_grads=True)
    return dict(
        seed=seed, isotropic=isotropic, stride=STRIDE,
        rgb=r.rgb[::STRIDE].tolist(), depth=r.depth[::STRIDE].tolist(), sil=r.sil[::STRIDE].tolist(),
        loss=r.loss.tolist(),
        grads={k: np.asarray(v).reshape(-1).tolist() for k, v in r.grads.items()},
    )


def main():
    out = dict(
        what="FP64 oracle outputs on seeded tiny scenes (regression record of the oracle)",
        written_by="tests/golden/make_golden.py",
        cases=[case_outputs(**c) for c in CASES],
    )
    path = os.path.join(HERE, "oracle_tiny.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
