"""uf_smooth_porosity_grad_noalloc (the allocation-free variant of the
design-porosity gradient) against uf_smooth_porosity_grad, through the C
ABI: two calls in a row, the second on a smaller grid with fewer objects,
then one with the most objects the variant takes (its partial rows then
fill the fixed scratch: fewer blocks than the allocating entry point)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2204_01117_amd as U


def _objects(seed, n, h, nb, nc):
    rng = np.random.default_rng(seed)
    ext = [n[a] * h[a] for a in range(3)]
    boxes = []
    for _ in range(nb):
        x0, y0 = rng.uniform(0, 0.8 * ext[0]), rng.uniform(0, 0.8 * ext[1])
        z0 = 0.0 if rng.random() < 0.7 else rng.uniform(0, 0.3 * ext[2])
        boxes.append([x0, x0 + rng.uniform(2, 0.3 * ext[0]), y0, y0 + rng.uniform(2, 0.3 * ext[1]),
                      z0, z0 + rng.uniform(2, 0.7 * ext[2]), rng.choice([0.0, rng.uniform(0.2, 0.8)])])
    cyls = []
    for _ in range(nc):
        z0 = 0.0 if rng.random() < 0.7 else rng.uniform(0, 0.3 * ext[2])
        cyls.append([rng.uniform(0, ext[0]), rng.uniform(0, ext[1]), rng.uniform(1, 0.2 * min(ext[:2])),
                     z0, z0 + rng.uniform(2, 0.6 * ext[2]), rng.uniform(0.2, 0.8)])
    return np.array(boxes).reshape(-1, 7), np.array(cyls).reshape(-1, 6)


def _compare(seed, n, h, nb, nc):
    boxes, cyls = _objects(seed, n, h, nb, nc)
    width = 0.5 * h[0]
    gen = torch.Generator().manual_seed(seed)
    phibar = torch.randn(n, dtype=torch.float64, generator=gen).to("cuda:0")
    rb, rc = U.smooth_porosity_grad(n, h, boxes, cyls, width, phibar)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    gb, gc = U.smooth_porosity_grad(n, h, boxes, cyls, width, phibar, noalloc=True)
    assert torch.cuda.memory_allocated() == before
    ref = np.concatenate([rb.ravel(), rc.ravel()])
    got = np.concatenate([gb.ravel(), gc.ravel()])
    assert got.shape == ref.shape and np.isfinite(got).all()
    # FP64 sums of the same per-cell terms in another grouping: a few
    # roundings of the largest partial sums
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    print("noalloc gradient", n, nb, nc, "max rel deviation %.2e" % err, flush=True)
    assert err <= 1e-12, err
    assert np.count_nonzero(ref) > 0


def test_noalloc_gradient_matches_the_allocating_call_twice():
    _compare(1, (48, 40, 24), (2.0, 2.0, 1.5), 24, 30)
    _compare(2, (17, 13, 9), (1.0, 1.2, 0.8), 3, 2)          # smaller: stale scratch must not leak in


def test_noalloc_gradient_at_the_object_limit():
    _compare(3, (64, 64, 32), (2.0, 2.0, 2.0), 700, 1024 - 700)


def test_noalloc_rejects_more_objects_than_its_scratch():
    n, h = (8, 8, 8), (1.0, 1.0, 1.0)
    boxes, cyls = _objects(4, n, h, 1000, 25)
    phibar = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(U.UFError) as e:
        U.smooth_porosity_grad(n, h, boxes, cyls, 0.5, phibar, noalloc=True)
    assert "UF_EINVAL" in str(e.value) and "UF_NOALLOC_MAX_OBJECTS" in str(e.value)
