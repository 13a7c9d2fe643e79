"""Boundary items of the C ABI on the GPU: the allocator hook, the
end-of-call diagnostics in uf_step_stats and the non-finite flag that the
drag and k-omega stages raise."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from uf_layouts import default_config, preset, preset_porosity, perturbed_state
from uf_layouts.configs import BC_INLET, BC_OUTLET, BC_SLIP, INFLOW_UNIFORM, TURB_OFF
from oracle import OracleGrid
from helpers import to_np, random_small_config, random_porosity

import paper_2204_01117_amd as U


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_torch_allocator_and_hipmalloc_give_identical_steps():
    p = preset("C0")
    phi, cfg = preset_porosity(p)
    cfg = dict(cfg, dtype="f32")
    before = torch.cuda.memory_allocated()
    a = U.Grid(cfg, torch_memory=True)
    grown = torch.cuda.memory_allocated() - before
    b = U.Grid(cfg, torch_memory=False)
    # 21 padded fields of (nx+3)(ny+3)(nz+3) floats at least come from torch
    assert grown >= 21 * 67 * 35 * 19 * 4, grown
    for g in (a, b):
        g.set_porosity(torch.as_tensor(phi))
        g.step(5)
        g.adjoint_step([g.get_field(f) for f in g.adjoint_fields()],
                       [torch.zeros_like(g.get_field(f)) for f in g.adjoint_fields()])
    sa, sb = a.state(), b.state()
    for f in sa:
        assert torch.equal(sa[f], sb[f]), f
    # the compared copies are the test's own tensors: release them before
    # counting what the grids leave behind
    del sa, sb
    a.close()
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + 1024


def _state_diag(cfg, st):
    """max |div u|, max dt sum |u_c| / h and the capped fraction of nu_t of
    the stored face and cell arrays exactly as they are (no boundary value
    re-imposed), in FP64 with the grid's spacing, time step and cap in its
    own dtype (the values the library holds)."""
    cast = np.float32 if cfg["dtype"] == "f32" else np.float64
    h = [float(cast(cfg[a])) for a in ("dx", "dy", "dz")]
    dt = float(cast(cfg["dt"]))
    u, v, w = st["u"], st["v"], st["w"]
    div = np.diff(u, axis=0) / h[0] + np.diff(v, axis=1) / h[1] + np.diff(w, axis=2) / h[2]
    cen = [0.5 * np.abs(u[1:] + u[:-1]), 0.5 * np.abs(v[:, 1:] + v[:, :-1]), 0.5 * np.abs(w[:, :, 1:] + w[:, :, :-1])]
    cfl = dt * (cen[0] / h[0] + cen[1] / h[1] + cen[2] / h[2])
    og = OracleGrid(dict(cfg, dtype="f64"), solver="none")
    cap = float(cast(og.g.nu_max() - cfg["nu"]))
    clip = float((st["nut"] >= cap).mean()) if cfg["turb_model"] else 0.0
    return float(np.abs(div).max()), float(cfl.max()), clip, cap


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_step_stats_diagnostics_match_the_state(dtype):
    cfg = random_small_config(8, dtype=dtype, cg_tol=1e-13 if dtype == "f64" else 1e-7, cg_maxit=5000)
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    phi = random_porosity(8, n)
    g = U.Grid(cfg)
    g.set_porosity(torch.as_tensor(phi))
    og = OracleGrid(dict(cfg, dtype="f64"), solver="none")
    st0 = perturbed_state(og.state(), seed=8)
    st0["nut"] = np.where(np.arange(np.prod(n)).reshape(n) % 3 == 0, 1e3, st0["nut"])   # some capped cells
    g.set_state({f: torch.as_tensor(v) for f, v in st0.items()})
    s = g.step(1)
    out = {f: to_np(v) for f, v in g.state().items()}
    mdiv, mcfl, clip, cap = _state_diag(cfg, out)
    log(dtype, "stats", {k: s[k] for k in ("max_div", "max_cfl", "nut_clip_frac")}, "oracle", mdiv, mcfl, clip)
    # both sides evaluate the same FP32 (or FP64) values in FP64: only the
    # order of the three additions may differ
    tol = 1e-12
    assert abs(s["max_cfl"] - mcfl) <= tol * mcfl
    assert abs(s["max_div"] - mdiv) <= max(tol * mdiv, 1e-14 * mcfl / cfg["dt"])
    assert abs(s["nut_clip_frac"] - clip) <= 1.0 / np.prod(n)
    # after a projection the divergence is at the solver's tolerance
    assert s["max_div"] * cfg["dt"] < (1e-9 if dtype == "f64" else 1e-3)
    g.close()


def test_step_stats_clip_fraction_zero_without_turbulence():
    cfg = random_small_config(9, dtype="f64", turb_model=TURB_OFF)
    g = U.Grid(cfg)
    s = g.step(2)
    assert s["nut_clip_frac"] == 0.0 and s["max_cfl"] > 0
    g.close()


def _flag_case(stages):
    cfg = default_config(10, 6, 5, 1.0, dt=0.1, inflow_kind=INFLOW_UNIFORM, u_ref=2.0, dtype="f32",
                         stages=stages, bc=[BC_INLET, BC_OUTLET, BC_SLIP, BC_SLIP, BC_SLIP, BC_SLIP])
    return U.Grid(cfg)


def test_drag_stage_raises_the_nonfinite_flag():
    g = _flag_case(4)                      # drag only: no solve sees the value
    clean = {f: to_np(g.get_field(f)) for f in "uvw"}
    u = clean["u"].copy()
    u[4, 2, 2] = np.inf
    g.set_field("u", u)
    st = g.step(1, allow=(5,))
    assert st["status"] == "UF_ENONFINITE" and st["nonfinite"] == 1
    # sticky until the state is overwritten
    assert g.step(1, allow=(5,))["status"] == "UF_ENONFINITE"
    # the drag spread the value into neighbouring faces of every component:
    # a clean state clears the flag
    for f in "uvw":
        g.set_field(f, clean[f])
    st = g.step(1)
    assert st["status"] == "UF_OK" and st["nonfinite"] == 0
    g.close()


def test_komega_stage_raises_the_nonfinite_flag():
    g = _flag_case(16)                     # k-omega only
    k = to_np(g.get_field("k"))
    k[5, 3, 1] = np.nan
    g.set_field("k", k)
    st = g.step(1, allow=(5,))
    assert st["status"] == "UF_ENONFINITE" and st["nonfinite"] == 1
    g.close()
    # without stats the last step's flag is reported by the next call
    g = _flag_case(16 | 8 | 4)
    k = to_np(g.get_field("k"))
    k[5, 3, 1] = np.nan
    g.set_field("k", k)
    assert g.step(1, stats=False)["status"] == "UF_OK"
    assert g.step(1, stats=False, allow=(5,))["status"] == "UF_ENONFINITE"
    g.close()
