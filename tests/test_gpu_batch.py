"""Several grids advanced together (uf_step_batch) compute exactly what each
computes alone with uf_step: the batch only interleaves the enqueueing, so
the states must agree bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from uf_layouts import preset, preset_porosity
from helpers import random_small_config, random_porosity

import paper_2204_01117_amd as U


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(cfg, phi, own_stream):
    g = U.Grid(cfg, stream=torch.cuda.Stream() if own_stream else None)
    g.set_porosity(torch.as_tensor(phi))
    return g


def test_batch_equals_single_grid_steps():
    cases = []
    for seed, dt in ((1, "f32"), (2, "f64"), (5, "f32"), (7, "f64"), (9, "f32")):
        cfg = random_small_config(seed, dtype=dt)
        cases.append((cfg, random_porosity(seed, (cfg["nx"], cfg["ny"], cfg["nz"]))))
    batched = [make(c, p, True) for c, p in cases]
    single = [make(c, p, False) for c, p in cases]
    sb = U.step_batch(batched, 6)
    for g, s in zip(single, sb):
        ss = g.step(6)
        assert ss["cg_iters_total"] == s["cg_iters_total"]
        assert ss["cg_iters_max"] == s["cg_iters_max"]
    for gb, gs in zip(batched, single):
        sa, sb_ = gb.state(), gs.state()
        for f in sa:
            assert torch.equal(sa[f], sb_[f]), f
    # a second call continues from where the first stopped
    U.step_batch(batched, 2)
    for g in single:
        g.step(2)
    for gb, gs in zip(batched, single):
        assert torch.equal(gb.get_field("p"), gs.get_field("p"))
    for g in batched + single:
        g.close()


def test_batch_rejects_bad_lists():
    cfg = random_small_config(3, dtype="f32")
    g = U.Grid(cfg)
    with pytest.raises(U.UFError) as e:
        U.step_batch([g, g], 1)
    assert e.value.name == "UF_EINVAL"
    with pytest.raises(U.UFError) as e:
        U.step_batch([], 1)
    assert e.value.name == "UF_EINVAL"
    g.close()


def test_batch_of_uneven_city_cases():
    """Four of the sixteen wind-direction cases (uneven grids, each on its own
    stream) for three steps: each equals the same case stepped alone."""
    p = preset("C3")
    cases = [preset_porosity(p, case=c) for c in (0, 5, 10, 15)]
    log("shapes", [(c["nx"], c["ny"], c["nz"]) for _, c in cases])
    batched = [make(c, phi, True) for phi, c in cases]
    st = U.step_batch(batched, 3)
    assert all(s["converged"] for s in st)
    for (phi, c), gb in zip(cases, batched):
        gs = make(c, phi, False)
        gs.step(3)
        assert torch.equal(gb.get_field("u"), gs.get_field("u"))
        assert torch.equal(gb.get_field("p"), gs.get_field("p"))
        gs.close()
    for g in batched:
        g.close()
