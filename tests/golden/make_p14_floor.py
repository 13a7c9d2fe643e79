"""Writes p14_floor.json: the perturbation-twin floor of the 64x32x16
workload (one solid box, one tree block), computed by the oracle alone.

Two twins of a 100-step oracle run from the initial state:

* "perturbed": the initial velocity, k and omega are each multiplied by
  (1 + 2^-24 r), r uniform in [-1, 1] (seeded), the size of one FP32
  rounding of the state.  Its distance from the run measures how much the
  flow itself amplifies (or damps) such a difference.
* "fp32_storage": the state is rounded to FP32 after every step (FP64
  arithmetic, FP32 storage).  Its distance is the part of an FP32 result's
  error that storing the state in FP32 alone causes.

The relative L2 distance per field group after n steps is recorded.

    python tests/golden/make_p14_floor.py      (about 20 s)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from uf_layouts import preset, preset_porosity  # noqa: E402
from oracle import OracleGrid  # noqa: E402

CHECKPOINTS = (1, 10, 50, 100)
SEED = 24


def groups(st):
    return {"vel": np.concatenate([st[f].ravel() for f in "uvw"]), "p": st["p"].ravel(),
            "k": st["k"].ravel(), "omega": st["omega"].ravel()}


def _dist(a, b):
    ga, gb = groups(a.state()), groups(b.state())
    return {k: float(np.linalg.norm(gb[k] - ga[k]) / np.linalg.norm(ga[k])) for k in ga}


def twin_floor(steps=CHECKPOINTS, seed=SEED):
    """{"perturbed": {n: {group: distance}}, "fp32_storage": {...}}."""
    p = preset("C0")
    phi, cfg = preset_porosity(p)
    cfg = dict(cfg, dtype="f64")
    a, b, c = OracleGrid(cfg), OracleGrid(cfg), OracleGrid(cfg)
    for g in (a, b, c):
        g.set_porosity(phi)
    rng = np.random.default_rng(seed)
    for f in ("u", "v", "w", "k", "omega"):
        x = b.get_field(f)
        b.set_field(f, x * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, size=x.shape)))

    def round32(g):
        for f in ("u", "v", "w", "p", "k", "omega", "nut"):
            g.set_field(f, g.get_field(f).astype(np.float32).astype(np.float64))

    round32(c)
    out = {"perturbed": {}, "fp32_storage": {}}
    for n in range(1, max(steps) + 1):
        a.step(1)
        b.step(1)
        c.step(1)
        round32(c)
        if n in steps:
            out["perturbed"][str(n)] = _dist(a, b)
            out["fp32_storage"][str(n)] = _dist(a, c)
    return out


def main():
    res = {"what": "relative L2 distance between the oracle (64x32x16 workload, FP64, direct pressure solve) "
                   "and two twins: 'perturbed' starts from the initial velocity, k and omega times "
                   "(1 + 2^-24 r), r uniform in [-1, 1] (seed %d); 'fp32_storage' rounds its state to FP32 "
                   "after every step" % SEED,
           "after_steps": twin_floor()}
    with open(os.path.join(HERE, "p14_floor.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["after_steps"]))


if __name__ == "__main__":
    main()
