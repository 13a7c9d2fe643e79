"""A grid's results do not depend on what its device memory held before it
was handed out: the same grid built in memory whose every byte (and 64 KiB
on each side of every allocation) is 0xFF -- a NaN in either precision --
steps to the same bits as one built in zeroed memory.  A kernel that reads
an element no one wrote, or past an array's end, turns NaN there."""
import ctypes
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from helpers import random_small_config, random_porosity
from uf_layouts import default_config, random_city, porosity_field

import paper_2204_01117_amd as U
from paper_2204_01117_amd import _lib as L

GUARD = 64 * 1024


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class FilledMemory:
    """uf_config alloc/free callbacks handing out torch byte tensors filled
    with one byte value, each with a guard of the same value on both sides."""

    def __init__(self, byte, stream):
        self.byte, self.stream, self.live = byte, stream, {}
        self.fns = (L.ALLOC_FN(self._alloc), L.FREE_FN(self._free))

    def _alloc(self, nbytes, ctx):
        with torch.cuda.stream(self.stream):
            t = torch.full((int(nbytes) + 2 * GUARD,), self.byte, dtype=torch.uint8, device="cuda:0")
        self.stream.synchronize()
        p = t.data_ptr() + GUARD
        self.live[p] = t
        return p

    def _free(self, ptr, ctx):
        self.live.pop(ptr, None)


def _cases():
    out = []
    for seed, dt in ((5, "f32"), (2, "f64"), (9, "f32"), (13, "f64")):
        cfg = random_small_config(seed, dtype=dt)
        out.append((cfg, random_porosity(seed, (cfg["nx"], cfg["ny"], cfg["nz"]))))
    nx, ny, nz, h = 64, 48, 64, 2.0
    cfg = default_config(nx, ny, nz, h, dt=0.09, u_ref=6.0, z_ref=10.0, dtype="f32", cg_maxit=2000,
                         cg_tol=1e-6, wind_dir_deg=30.0)
    boxes, cyls, _ = random_city(nx, ny, nz, h, h, h, seed=77, n_boxes=6, n_trees=10)
    out.append((cfg, porosity_field(nx, ny, nz, h, h, h, boxes, cyls)))
    return out


@pytest.mark.parametrize("which", range(5))
def test_results_do_not_depend_on_fresh_memory(which):
    cfg, phi = _cases()[which]
    log("case", which, (cfg["nx"], cfg["ny"], cfg["nz"]), cfg["dtype"])
    grids, mems = [], []
    for byte in (0x00, 0xFF):
        s = torch.cuda.Stream()
        m = FilledMemory(byte, s)
        g = U.Grid(cfg, stream=s, allocator=m.fns)
        g.set_porosity(torch.as_tensor(phi))
        grids.append(g)
        mems.append(m)
    st = [g.step(4) for g in grids]
    log("iters", [s["cg_iters_total"] for s in st], [s["status"] if "status" in s else "" for s in st])
    assert st[0]["cg_iters_total"] == st[1]["cg_iters_total"]
    a, b = grids[0].state(), grids[1].state()
    for f in a:
        assert torch.equal(a[f], b[f]), f
    for g in grids:
        g.close()
