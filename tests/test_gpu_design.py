"""Smoothed object porosity (uf_smooth_porosity) against the oracle, and
the design-parameter map on it."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from uf_layouts import preset, random_city
from oracle.smooth import smooth_porosity as oracle_smooth

import paper_2204_01117_amd as U


def objects(seed, n, h):
    boxes, cyls, _ = random_city(*n, *h, seed, 6, 5, footprint=(6.0, 14.0), height=(4.0, 14.0), tree_r=(2.0, 4.0),
                                 tree_h=(3.0, 8.0))
    b = [(*x.x, *x.y, *x.z, x.phi) for x in boxes]
    b.append((5.1, 9.3, 3.3, 8.8, 3.7, 9.9, 0.2))   # a lifted box
    c = [(x.cx, x.cy, x.r, *x.z, x.phi) for x in cyls]
    return b, c


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_smooth_porosity_matches_oracle(seed, dtype):
    n, h = (24, 20, 10), (2.0, 1.5, 2.0)
    b, c = objects(seed, n, h)
    for width in (0.3, 1.0, 3.0):
        got = U.smooth_porosity(n, h, b, c, width, dtype=dtype).double().cpu().numpy()
        ref = oracle_smooth(n, h, b, c, width)
        if dtype == "f64":
            assert np.allclose(got, ref, rtol=0, atol=1e-14)
        else:
            assert np.allclose(got, ref, rtol=0, atol=1.2e-7)
        assert (got < 0.999).sum() > 50


def test_smooth_porosity_rejects_bad_input():
    n, h = (4, 4, 4), (1.0, 1.0, 1.0)
    for b, c, w in (([(0, 1, 0, 1, 0, 1, 1.5)], [], 1.0), ([], [(1, 1, -1, 0, 2, 0.5)], 1.0),
                    ([(0, 1, 0, 1, 0, float("nan"), 0.0)], [], 1.0), ([], [], 0.0)):
        with pytest.raises(U.UFError) as e:
            U.smooth_porosity(n, h, b, c, w)
        assert e.value.name == "UF_EINVAL"
    assert torch.equal(U.smooth_porosity(n, h, [], [], 1.0), torch.ones(4, 4, 4, device="cuda"))


def test_design_map_moves_objects_continuously():
    p = preset("C4")
    cfg, lay = p["config"], p["layout"]
    n, h = (cfg["nx"], cfg["ny"], cfg["nz"]), (cfg["dx"], cfg["dy"], cfg["dz"])
    boxes, cyls, _ = random_city(*n, *h, lay["seed"], lay["n_boxes"], lay["n_trees"])
    d = U.BoxDesign(n, h, [(*x.x, *x.y, *x.z, x.phi) for x in boxes], [(x.cx, x.cy, x.r, *x.z, x.phi) for x in cyls],
                    width=h[0] / 2, dtype="f64")
    assert d.nparams == 64
    t0 = d.initial()
    phi0 = d.porosity(t0).cpu().numpy()
    b, c = d.objects(t0)
    assert np.allclose(phi0, oracle_smooth(n, h, b, c, h[0] / 2), rtol=0, atol=1e-13)
    # a 0.1 m shift of one building changes the field a little, continuously
    t1 = t0.copy()
    t1[1] += 0.1
    phi1 = d.porosity(t1).cpu().numpy()
    diff = np.abs(phi1 - phi0)
    assert 0 < diff.max() < 0.1
    t2 = t0.copy()
    t2[1] += 0.05
    mid = d.porosity(t2).cpu().numpy()
    assert np.abs(mid - phi0).max() < diff.max()


def _many_objects(seed, n, h, nb, nc):
    rng = np.random.default_rng(seed)
    ext = [n[a] * h[a] for a in range(3)]
    boxes = []
    for _ in range(nb):
        x0, y0 = rng.uniform(0, 0.8 * ext[0]), rng.uniform(0, 0.8 * ext[1])
        boxes.append([x0, x0 + rng.uniform(2, 0.3 * ext[0]), y0, y0 + rng.uniform(2, 0.3 * ext[1]),
                      0.0, rng.uniform(2, 0.7 * ext[2]), rng.uniform(0.0, 0.8)])
    cyls = [[rng.uniform(0, ext[0]), rng.uniform(0, ext[1]), rng.uniform(1, 0.2 * min(ext[:2])), 0.0,
             rng.uniform(2, 0.6 * ext[2]), rng.uniform(0.2, 0.8)] for _ in range(nc)]
    return np.array(boxes).reshape(-1, 7), np.array(cyls).reshape(-1, 6)


@pytest.mark.parametrize("nb,nc", [(6, 5), (700, 324)])
def test_smooth_porosity_grad_is_the_same_bits_every_run(nb, nc):
    """The design-porosity gradient sums its per-cell terms in a fixed
    order: repeated calls (and repeated calls of the allocation-free
    variant) give the same bits, up to the object limit."""
    n, h = (48, 40, 24), (2.0, 2.0, 1.5)
    boxes, cyls = _many_objects(11, n, h, nb, nc)
    gen = torch.Generator().manual_seed(5)
    phibar = torch.randn(n, dtype=torch.float64, generator=gen).to("cuda:0")
    for noalloc in (False, True):
        runs = [U.smooth_porosity_grad(n, h, boxes, cyls, 1.0, phibar, noalloc=noalloc) for _ in range(3)]
        for gb, gc in runs[1:]:
            assert np.array_equal(gb, runs[0][0]) and np.array_equal(gc, runs[0][1])
        assert np.count_nonzero(runs[0][0]) > 0
