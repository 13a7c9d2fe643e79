"""P14: the FP32 floor of the 64x32x16 workload, from oracle twins.

tests/golden/make_p14_floor.py (oracle only) wrote p14_floor.json; this test
recomputes it, so the stored floor always belongs to the oracle as it is,
and checks what it says about the parity bar: the flow damps an initial
FP32-sized perturbation instead of amplifying it, and FP32 storage alone
stays well below the 1e-4 bar after 100 steps.  The GPU's 100-step parity
test reports its own distance beside these figures.
"""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


@pytest.mark.slow
def test_p14_twin_floor_reproduces_and_sits_below_the_bar():
    sys.path.insert(0, GOLD)
    try:
        import make_p14_floor as M
    finally:
        sys.path.remove(GOLD)
    stored = json.load(open(os.path.join(GOLD, "p14_floor.json")))["after_steps"]
    now = M.twin_floor()
    for kind in ("perturbed", "fp32_storage"):
        for n, grp in stored[kind].items():
            for k, v in grp.items():
                assert abs(now[kind][n][k] - v) <= 1e-2 * v, (kind, n, k, now[kind][n][k], v)
    pert, store = now["perturbed"], now["fp32_storage"]
    # the perturbation is seen after one step (about one FP32 rounding) ...
    assert 2.0 ** -24 / 4 < pert["1"]["vel"] < 2.0 ** -24 * 4
    # ... and the flow damps it: no chaotic growth over 100 steps
    for k in pert["100"]:
        assert pert["100"][k] < pert["1"][k], k
    # FP32 storage alone stays far below the 1e-4 bar after 100 steps
    for k, v in store["100"].items():
        assert v < 1e-6, (k, v)
