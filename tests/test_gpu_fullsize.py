"""Parity of the HIP path with the oracle at full size and at the edges of the
method's regime, every input drawn on the host from the oracle's initial
state plus a seeded smooth perturbation (uf_layouts.perturbed_state); no
input of the oracle comes from the GPU.

* one complete 256x256x64 step, element by element, FP32 (the benchmark's
  launch configuration) and FP64;
* 100 free-running steps on a 64x48x64 city, a grid that takes the
  full-size launch paths (64-cell columns in the CG kernels, three multigrid
  levels above the single-workgroup tail), reported beside the P14 floor;
* the 512x512x128 step stage by stage: the projection over the whole grid,
  the local stages (advection, diffusion, drag; k-omega) on windows whose
  artificial sides are kept away from the compared cells;
* CFL 1 (a pure shift) and CFL 0.97 through the C ABI;
* an active MacCormack clamp and an active eddy-viscosity cap;
* a case of the sixteen-case workload stepped by uf_step_batch.
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from uf_layouts import default_config, preset, preset_porosity, perturbed_state, random_city, porosity_field
from uf_layouts.configs import (BC_INLET, BC_OUTLET, BC_SLIP, INFLOW_UNIFORM, PC_MG, STAGE_ADVECT)
from oracle import OracleGrid, Geometry, resolve_bc
from helpers import rel, to_np, state_errors, random_small_config, random_porosity

import paper_2204_01117_amd as U

HERE = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_grid(cfg, phi=None, state=None, stream=None):
    g = U.Grid(cfg, stream=stream)
    if phi is not None:
        g.set_porosity(torch.as_tensor(phi))
    if state is not None:
        g.set_state({f: torch.as_tensor(v) for f, v in state.items()})
    return g


def np_state(g):
    return {f: to_np(v) for f, v in g.state().items()}


def assert_close(errs, tol, fields=("vel", "p", "k", "omega"), what=""):
    bad = {f: e for f, e in errs.items() if f in fields and not e <= tol}
    assert not bad, "%s errors above %.1e: %s (all: %s)" % (what, tol, bad, errs)


def column_initial_state(cfg):
    """The oracle's initial state of a whole grid from a 4x4 window of it: the
    initial state carries the inflow of each height on every face and k,
    omega and nu_t that depend on the height only, so it is the window's
    interior columns repeated over x and y."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    win = OracleGrid(dict(cfg, nx=4, ny=4, bc=resolve_bc(cfg)), solver="none")
    st = win.state()
    out = {}
    for f, v in st.items():
        col = v[1, 1, :]
        ext = {"u": (nx + 1, ny, nz), "v": (nx, ny + 1, nz), "w": (nx, ny, nz + 1)}.get(f, (nx, ny, nz))
        out[f] = np.broadcast_to(col[None, None, :], ext).copy()
    return out


# ------------------------------------------------ one full 256x256x64 step ---
@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype,cg_tol,tol", [("f32", 1e-6, 1e-5), ("f64", 1e-13, 1e-10)])
def test_c1_one_complete_step_elementwise(dtype, cg_tol, tol):
    p = preset("C1")
    phi, cfg = preset_porosity(p)
    cfg = dict(cfg, dtype=dtype, cg_tol=cg_tol, cg_maxit=2000)
    og = OracleGrid(dict(cfg, dtype="f64"))         # exact (fast-diagonalisation) pressure solve
    og.set_porosity(phi)
    st0 = perturbed_state(og.state(), seed=1)
    for f, v in st0.items():
        og.set_field(f, v)
    # the column shortcut used at 512x512x128 reproduces the oracle's own initial state
    og0 = OracleGrid(dict(cfg, dtype="f64"), solver="none")
    cols = column_initial_state(cfg)
    for f, v in og0.state().items():
        assert np.array_equal(cols[f], v), f
    g = gpu_grid(cfg, phi, st0)
    log("C1 %s: stepping" % dtype)
    og.step(1)
    st = g.step(1)
    assert st["converged"] == 1, st
    errs = state_errors(np_state(g), og.state())
    log("C1 one step", dtype, "cg", st["cg_iters"], errs)
    assert_close(errs, tol, what="C1 %s step" % dtype)
    # nu_t is not one of the compared groups: where the limiter is active
    # (98% of the cells here) it is k / (C |S|), and |S| is a difference of
    # face velocities -- 0.04 to 0.07 1/s in most of those cells against
    # |u| / h of about 6 1/s, so nu_t carries the velocity's relative error
    # (a few 1e-7 here, set by the solve's tolerance) about a hundredfold
    assert_close(errs, tol if dtype == "f64" else 1e-4, fields=("nut",), what="C1 %s nu_t" % dtype)
    g.close()


# ------------------------------------- 100 steps on the full-size launch paths
@pytest.mark.timeout(300)
def test_hundred_steps_on_full_size_launch_paths():
    nx, ny, nz, h = 64, 48, 64, 2.0
    cfg = default_config(nx, ny, nz, h, dt=0.09, u_ref=6.0, z_ref=10.0, precond=PC_MG, cg_maxit=2000)
    boxes, cyls, _ = random_city(nx, ny, nz, h, h, h, seed=77, n_boxes=6, n_trees=10)
    phi = porosity_field(nx, ny, nz, h, h, h, boxes, cyls)
    og = OracleGrid(dict(cfg, dtype="f64"))
    og.set_porosity(phi)
    # multigrid levels 64x48x64, 32x24x32, 16x12x16 above the single-workgroup
    # tail (8x6x8 and below: the first level of at most 1024 cells)
    g32 = gpu_grid(dict(cfg, dtype="f32", cg_tol=1e-6), phi)
    g64 = gpu_grid(dict(cfg, dtype="f64", cg_tol=1e-13), phi)
    for blk in range(10):
        og.step(10)
        for g in (g32, g64):
            st = g.step(10)
            assert st["converged"] == 1, st
        log("block", blk, "done")
    so = og.state()
    e32 = state_errors(np_state(g32), so)
    e64 = state_errors(np_state(g64), so)
    floor = json.load(open(os.path.join(HERE, "golden", "p14_floor.json")))["after_steps"]
    log("64x48x64, 100 steps: FP32", e32, "FP64", e64,
        "| 64x32x16 P14 after 100 steps: perturbed", floor["perturbed"]["100"],
        "FP32 storage", floor["fp32_storage"]["100"])
    assert_close(e32, 1e-4, what="FP32 100 steps")
    assert_close(e64, 1e-10, what="FP64 100 steps")
    g32.close()
    g64.close()


# ------------------------------------------- 512x512x128, stage by stage ---
@pytest.fixture(scope="module")
def c2_case():
    p = preset("C2")
    phi, cfg = preset_porosity(p)
    cfg = dict(cfg, cg_maxit=2000)
    st = perturbed_state(column_initial_state(cfg), seed=2)
    return phi, cfg, st


def _window(cfg, phi, st, i0, i1, j0, j1):
    """An oracle grid over cells [i0, i1) x [j0, j1) x all of z: the domain's
    own side kinds where the window reaches the domain side, outlets on the
    artificial sides (whose cells are not compared)."""
    nx, ny = cfg["nx"], cfg["ny"]
    bc = resolve_bc(cfg)
    wbc = [bc[0] if i0 == 0 else BC_OUTLET, bc[1] if i1 == nx else BC_OUTLET,
           bc[2] if j0 == 0 else BC_OUTLET, bc[3] if j1 == ny else BC_OUTLET, bc[4], bc[5]]
    wcfg = dict(cfg, nx=i1 - i0, ny=j1 - j0, bc=wbc, dtype="f64")
    og = OracleGrid(wcfg, solver="none")
    og.set_porosity(phi[i0:i1, j0:j1])
    sl = {"u": (slice(i0, i1 + 1), slice(j0, j1)), "v": (slice(i0, i1), slice(j0, j1 + 1))}
    for f, v in st.items():
        og.set_field(f, v[sl.get(f, (slice(i0, i1), slice(j0, j1)))])
    return og


def _window_compare(out, og, i0, i1, j0, j1, nx, ny, m, fields):
    """Relative L2 error over the window's cells at least m cells from an
    artificial side, per field."""
    a0 = m if i0 > 0 else 0
    a1 = (i1 - i0) - m if i1 < nx else i1 - i0
    b0 = m if j0 > 0 else 0
    b1 = (j1 - j0) - m if j1 < ny else j1 - j0
    errs = {}
    for f in fields:
        ref = og.get_field(f)
        gpu = out[f][i0:i1 + (f == "u"), j0:j1 + (f == "v")]
        errs[f] = rel(gpu[a0:a1 + (f == "u" and i1 == nx), b0:b1 + (f == "v" and j1 == ny)],
                      ref[a0:a1 + (f == "u" and i1 == nx), b0:b1 + (f == "v" and j1 == ny)])
    return errs


WINDOWS = [(0, 40, 0, 40), (236, 276, 300, 340), (472, 512, 472, 512), (0, 40, 472, 512)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("stages,fields", [(7, ("u", "v", "w")), (16, ("k", "omega", "nut"))])
def test_c2_local_stages_on_windows(c2_case, stages, fields):
    phi, cfg, st = c2_case
    nx, ny = cfg["nx"], cfg["ny"]
    g = gpu_grid(dict(cfg, stages=stages), phi, st)
    g.step(1)
    out = np_state(g)
    g.close()
    for (i0, i1, j0, j1) in WINDOWS:
        og = _window(dict(cfg, stages=stages), phi, st, i0, i1, j0, j1)
        og.step(1)
        errs = _window_compare(out, og, i0, i1, j0, j1, nx, ny, 6, fields)
        log("C2 stages", stages, "window", (i0, i1, j0, j1), errs)
        assert max(errs.values()) <= 1e-5, errs


@pytest.mark.timeout(300)
def test_c2_projection_whole_grid(c2_case):
    phi, cfg, st = c2_case
    g = gpu_grid(dict(cfg, stages=8), phi, st)
    s = g.step(1)
    assert s["converged"] == 1, s
    out = np_state(g)
    g.close()
    og = OracleGrid(dict(cfg, stages=8, dtype="f64"), solver="fastdiag")
    for f, v in st.items():
        og.set_field(f, v)
    og.step(1)
    ref = og.state()
    errs = state_errors(out, ref)
    log("C2 projection: cg", s["cg_iters"], errs)
    assert errs["vel"] <= 1e-5 and errs["p"] <= 1e-5, errs
    # a preconditioner broken but still positive definite would converge too,
    # only slowly: from the perturbed state's warm start this takes about 10
    assert s["cg_iters"] <= 25, s


@pytest.mark.timeout(300)
def test_c2_multigrid_marching_kernels_are_a_symmetric_operator(c2_case):
    """At 512x512x128 level 0 of the multigrid cycle runs the marching
    kernels (the update-free restriction march of a stand-alone application,
    the prolongation/smoothing march; chunks of 16 coarse and 32 fine planes):
    in FP64 the preconditioner they form is symmetric (y.Mx = x.My to 1e-12)
    and positive, and applying it twice gives the same bits.  A restriction
    that is not the transpose of the prolongation, a dropped halo entry or a
    misplaced plane breaks the symmetry."""
    _, cfg, _ = c2_case
    g = gpu_grid(dict(cfg, dtype="f64", precond=PC_MG))
    rng = np.random.default_rng(11)
    x = torch.tensor(rng.normal(size=g.n))
    y = torch.tensor(rng.normal(size=g.n))
    mx, my = to_np(g.apply_operator(1, x)), to_np(g.apply_operator(1, y))
    xn, yn = x.numpy(), y.numpy()
    a, b = float((yn * mx).sum()), float((xn * my).sum())
    xmx, ymy = float((xn * mx).sum()), float((yn * my).sum())
    log("C2 multigrid: y.Mx", a, "x.My", b, "x.Mx", xmx)
    assert xmx > 0 and ymy > 0
    assert abs(a - b) <= 1e-12 * np.sqrt(xmx * ymy)
    assert np.array_equal(mx, to_np(g.apply_operator(1, x)))
    g.close()


# ------------------------------------------------------ CFL at and near 1 ---
def _shift_cfg(nx, U0, dt, dx, dtype):
    return default_config(nx, 4, 3, dx, dt=dt, inflow_kind=INFLOW_UNIFORM, u_ref=U0, nu=0.0,
                          stages=STAGE_ADVECT, dtype=dtype,
                          bc=[BC_INLET, BC_OUTLET, BC_OUTLET, BC_OUTLET, BC_SLIP, BC_SLIP])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_integer_cfl_is_a_pure_shift_gpu(dtype):
    nx, U0, dt, dx = 16, 2.0, 1.0, 2.0           # CFL exactly 1
    f = np.random.default_rng(3).normal(size=nx)
    g = gpu_grid(_shift_cfg(nx, U0, dt, dx, dtype))
    g.set_field("v", np.repeat(np.repeat(f[:, None, None], 5, axis=1), 3, axis=2))
    g.step(4)
    out = to_np(g.get_field("v"))[:, 1:-1, :]
    for i in range(5, nx - 1):
        assert np.abs(out[i] - f[i - 4]).max() <= (1e-13 if dtype == "f64" else 1e-6)
    assert np.abs(to_np(g.get_field("u")) - U0).max() <= 1e-6
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_cfl_near_one_full_step(dtype):
    cfg = random_small_config(21, dtype=dtype, precond=PC_MG, cg_tol=1e-13 if dtype == "f64" else 1e-7,
                              cg_maxit=5000)
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    phi = random_porosity(21, n)
    og = OracleGrid(dict(cfg, dtype="f64"))
    og.set_porosity(phi)
    st = perturbed_state(og.state(), seed=21, rel_velocity=0.4)
    h = (cfg["dx"], cfg["dy"], cfg["dz"])
    cfl = max(np.abs(st[f]).max() * cfg["dt"] / h[c] for c, f in enumerate("uvw"))
    cfg = dict(cfg, dt=cfg["dt"] * 0.97 / cfl)       # largest one-axis CFL 0.97
    og = OracleGrid(dict(cfg, dtype="f64"))
    og.set_porosity(phi)
    for f, v in st.items():
        og.set_field(f, v)
    g = gpu_grid(cfg, phi, st)
    og.step(1)
    s = g.step(1)
    assert s["converged"] == 1
    errs = state_errors(np_state(g), og.state())
    log("CFL 0.97", dtype, errs)
    assert_close(errs, 1e-11 if dtype == "f64" else 1e-5, what="CFL 0.97")
    g.close()


# ------------------------------------------ active clamp, active nu_t cap ---
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_maccormack_clamp_active_gpu(dtype):
    """The random 1-D profile of the oracle's clamp pin: several faces are
    clamped; GPU = oracle face by face."""
    nx, U0, dt, dx = 24, 1.0, 0.4, 1.0
    f = np.random.default_rng(11).normal(size=nx)
    v = np.repeat(np.repeat(f[:, None, None], 5, axis=1), 3, axis=2)
    cfg = _shift_cfg(nx, U0, dt, dx, dtype)
    og = OracleGrid(dict(cfg, dtype="f64"))
    og.set_field("v", v)
    g = gpu_grid(cfg)
    g.set_field("v", v)
    og.step(1)
    g.step(1)
    ref, out = og.get_field("v"), to_np(g.get_field("v"))
    assert np.abs(out - ref).max() <= (1e-13 if dtype == "f64" else 3e-6)
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_nut_cap_active_gpu(dtype):
    """k / omega far above the explicit-diffusion bound in a large share of
    the cells (the rest stay below it, so both branches of the clip run):
    the capped eddy viscosity drives the diffusion of the next step.  Two
    steps, each from the oracle's state (per-step parity); the second has
    the cap active from the start and its pressure falls fourteenfold."""
    cfg = random_small_config(33, dtype=dtype, precond=PC_MG, cg_tol=1e-13 if dtype == "f64" else 1e-7,
                              cg_maxit=5000, nu=0.01)
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    phi = random_porosity(33, n)
    og = OracleGrid(dict(cfg, dtype="f64"))
    og.set_porosity(phi)
    st = og.state()
    st["k"] = st["k"] * 50.0
    st["omega"] = st["omega"] * 1e-3
    cap = og.g.nu_max() - 0.01
    st["nut"] = np.full(n, cap)
    for f, v in st.items():
        og.set_field(f, v)
    g = gpu_grid(cfg, phi)
    for step in range(2):
        g.set_state({f: torch.as_tensor(v) for f, v in og.state().items()})
        og.step(1)
        s = g.step(1)
        assert s["converged"] == 1
        so = og.state()
        frac = float((so["nut"] >= cap * (1 - 1e-12)).mean())
        errs = state_errors(np_state(g), so)
        log("step %d: nu_t cap active in %.2f of the cells" % (step + 1, frac), dtype, errs)
        assert 0.2 < frac < 0.9, frac          # 0.26 after the first step, 0.43 after the second
        assert_close(errs, 1e-11 if dtype == "f64" else 1e-5, fields=("vel", "p", "k", "omega", "nut"),
                     what="capped nu_t, step %d" % (step + 1))
    g.close()


# ------------------------------------------ a batched case against the oracle
@pytest.mark.timeout(300)
def test_batched_case_matches_oracle():
    """The smallest of the sixteen uneven cases and two ragged small grids
    stepped together by uf_step_batch, each from a seeded state; every one
    against the oracle after one step."""
    p = preset("C3")
    cases = []
    for c in range(16):
        phi, cfg = preset_porosity(p, case=c)
        if (cfg["nx"], cfg["ny"], cfg["nz"]) == (128, 128, 48):
            cases.append((phi, dict(cfg, cg_tol=1e-6, cg_maxit=2000)))
            break
    assert cases
    for seed in (41, 42):
        cfg = random_small_config(seed, dtype="f32", cg_tol=1e-7, cg_maxit=5000)
        cases.append((random_porosity(seed, (cfg["nx"], cfg["ny"], cfg["nz"])), cfg))
    grids, oracles = [], []
    for q, (phi, cfg) in enumerate(cases):
        og = OracleGrid(dict(cfg, dtype="f64"))
        og.set_porosity(phi)
        st = perturbed_state(og.state(), seed=50 + q)
        for f, v in st.items():
            og.set_field(f, v)
        oracles.append(og)
        grids.append(gpu_grid(cfg, phi, st, stream=torch.cuda.Stream()))
    stats = U.step_batch(grids, 1)
    assert all(s["converged"] for s in stats), stats
    for g, og, (phi, cfg) in zip(grids, oracles, cases):
        og.step(1)
        errs = state_errors(np_state(g), og.state())
        log("batched case", (cfg["nx"], cfg["ny"], cfg["nz"]), errs)
        assert_close(errs, 1e-5, what="batched case")
        g.close()
