"""The target-region objective (Sec. 4) and the forward-difference optimiser
on the GPU, through the C ABI, against the oracle.

The objective sums cell speeds in FP64 on both sides, so the GPU value must
equal the oracle's on the same state to 1e-12 relative in both precisions
(only the order of the FP64 additions differs)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from uf_layouts import default_config, preset, preset_porosity
from oracle import OracleGrid, region_objective, plane_objective, field_objective, fd_gradient
from helpers import to_np, random_small_config, random_porosity

import paper_2204_01117_amd as U
from paper_2204_01117_amd import optimize as O

OBJ_TOL = 1e-12


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def random_regions(rng, n, count):
    out = []
    for _ in range(count):
        box = []
        for a in range(3):
            lo = int(rng.integers(0, n[a]))
            hi = int(rng.integers(lo + 1, n[a] + 1))
            box.append((lo, hi))
        out.append(tuple(box))
    return out


def oracle_J(g, regions, ut):
    s = {f: to_np(g.get_field(f)) for f in "uvw"}
    return region_objective(s["u"], s["v"], s["w"], regions, ut)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_objective_matches_oracle_on_random_state(seed, dtype):
    cfg = random_small_config(seed, dtype=dtype)
    log("case", seed, dtype, cfg["nx"], cfg["ny"], cfg["nz"])
    g = U.Grid(cfg)
    rng = np.random.default_rng(seed + 50)
    for f in "uvw":
        g.set_field(f, torch.as_tensor(rng.normal(size=g.extent(f))))
    nx, ny, nz = g.n
    regions = random_regions(rng, g.n, 5)
    regions += [((0, nx), (0, ny), (0, nz)),                          # whole grid
                ((nx - 1, nx), (ny - 1, ny), (nz - 1, nz)),           # last cell: top/east/north faces
                ((0, 1), (0, 1), (0, 1))]
    for ut in (0.55, 0.0):
        J = g.objective(regions, ut)
        ref = oracle_J(g, regions, ut)
        assert abs(J - ref) <= OBJ_TOL * abs(ref), (J, ref)
    g.close()


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_field_objective_matches_oracle(seed, dtype):
    cfg = random_small_config(seed + 40, dtype=dtype)
    g = U.Grid(cfg)
    rng = np.random.default_rng(seed + 7)
    for f in "uvw":
        g.set_field(f, torch.as_tensor(rng.normal(size=g.extent(f))))
    nx, ny, nz = g.n
    ut = rng.normal(size=(3, nx, ny, nz))
    if dtype == "f32":
        ut = ut.astype(np.float32).astype(np.float64)   # the GPU holds it in the grid's dtype
    regions = random_regions(rng, g.n, 4) + [((0, nx), (0, ny), (0, nz)), ((nx - 1, nx), (ny - 1, ny), (nz - 1, nz))]
    J = g.field_objective(regions, torch.as_tensor(ut))
    s = {f: to_np(g.get_field(f)) for f in "uvw"}
    ref = field_objective(s["u"], s["v"], s["w"], ut, regions)
    assert abs(J - ref) <= OBJ_TOL * abs(ref), (J, ref)
    # the desired flow equal to the current one scores 0 (bit for bit in FP64)
    if dtype == "f64":
        cc = np.stack([(s["u"][:-1] + s["u"][1:]) / 2, (s["v"][:, :-1] + s["v"][:, 1:]) / 2,
                       (s["w"][:, :, :-1] + s["w"][:, :, 1:]) / 2])
        assert g.field_objective(regions, torch.as_tensor(cc)) == 0.0
    g.close()


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_plane_objective_matches_oracle(seed, dtype):
    cfg = random_small_config(seed + 20, dtype=dtype)
    g = U.Grid(cfg)
    rng = np.random.default_rng(seed)
    for f in "uvw":
        g.set_field(f, torch.as_tensor(rng.normal(size=g.extent(f)) * (0.3 if seed == 1 else 1.0)))
    phi = random_porosity(seed, g.n)
    g.set_porosity(torch.as_tensor(phi))
    h = (cfg["dx"], cfg["dy"], cfg["dz"])
    s = {f: to_np(g.get_field(f)) for f in ("u", "v", "w", "phi")}
    for zp in (0.5 * h[2], 1.5, 0.37 * g.n[2] * h[2], (g.n[2] - 0.5) * h[2]):
        if not 0.5 * h[2] <= zp <= (g.n[2] - 0.5) * h[2]:
            continue
        J = g.plane_objective(zp)
        ref = plane_objective(s["u"], s["v"], s["w"], s["phi"], h, zp)
        assert abs(J - ref) <= OBJ_TOL * abs(ref), (zp, J, ref)
    with pytest.raises(U.UFError):
        g.plane_objective(0.49 * h[2])
    with pytest.raises(U.UFError):
        g.plane_objective(1.5, w_penalty=-1.0)
    g.close()


def test_objective_rejects_bad_specs_before_work():
    cfg = random_small_config(3, dtype="f32")
    g = U.Grid(cfg)
    nx, ny, nz = g.n
    ok = ((0, nx), (0, ny), (0, nz))
    bad = [[((0, nx + 1), (0, ny), (0, nz))], [((-1, 1), (0, ny), (0, nz))],
           [((2, 2), (0, ny), (0, nz))], [((0, nx), (0, ny), (3, 1))], [],
           [ok] * 65]
    for regions in bad:
        with pytest.raises(U.UFError) as e:
            g.objective(regions, 0.55)
        assert e.value.name == "UF_EINVAL", regions
    with pytest.raises(U.UFError) as e:
        g.objective([ok], float("nan"))
    assert e.value.name == "UF_EINVAL"
    # a bad plane is refused before its gradient buffer is touched
    import ctypes
    from paper_2204_01117_amd import _lib
    J = ctypes.c_double()
    ext = [g.extent(f) for f in ("u", "v", "w")]
    buf = torch.zeros(sum(e[0] * e[1] * e[2] for e in ext), dtype=g.dtype, device="cuda")
    pspec = _lib.make_plane_spec(0.1 * cfg["dz"])
    rc = U.uf_objective(g.handle, ctypes.byref(pspec), ctypes.byref(J), ctypes.c_void_p(buf.data_ptr()))
    assert U.STATUS[rc] == "UF_EINVAL"
    assert not buf.any()
    # 64 regions is the maximum and works
    assert g.objective([ok] * 64, 0.55) >= 0.0
    g.close()


def test_objective_full_size_after_steps():
    """256x256x64 with the preset city, six near-ground target regions (the
    paper's Nurnberg study scores six), after a few steps."""
    p = preset("C1")
    phi, cfg = preset_porosity(p)
    g = U.Grid(cfg)
    g.set_porosity(torch.as_tensor(phi))
    g.step(5)
    rng = np.random.default_rng(11)
    regions = []
    for _ in range(6):
        i0, j0 = int(rng.integers(0, 224)), int(rng.integers(0, 224))
        regions.append(((i0, i0 + 32), (j0, j0 + 32), (0, 2)))
    regions.append(((0, 256), (0, 256), (0, 64)))
    J = g.objective(regions, 0.55)
    ref = oracle_J(g, regions, 0.55)
    log("C1 objective", J, ref)
    assert abs(J - ref) <= OBJ_TOL * abs(ref)
    s = {f: to_np(g.get_field(f)) for f in ("u", "v", "w", "phi")}
    Jp = g.plane_objective(1.5)
    refp = plane_objective(s["u"], s["v"], s["w"], s["phi"], (2.0, 2.0, 2.0), 1.5)
    log("C1 plane objective", Jp, refp)
    assert abs(Jp - refp) <= OBJ_TOL * abs(refp)
    g.close()


# ------------------------------------------------ forward-difference descent --
BLOCKS = (((4, 7), (3, 9), (0, 5)), ((4, 7), (0, 3), (0, 3)))
TARGETS = [((8, 12), (3, 9), (0, 3)), ((8, 12), (0, 3), (0, 3))]


def _tiny_cfg():
    # pressure solved to 1e-13 so that ten steps stay within FP64 parity of
    # the oracle's direct solve
    return default_config(16, 12, 8, 2.0, dtype="f64", dt=0.05, u_ref=3.0, z_ref=6.0, cg_tol=1e-13)


def _phi_of(theta):
    phi = np.ones((16, 12, 8))
    for t, ((a, b), (c, d), (e, f)) in zip(theta, BLOCKS):
        phi[a:b, c:d, e:f] = min(max(float(t), 0.0), 1.0)
    return phi


def _oracle_sim(theta, nsteps, ut):
    o = OracleGrid(_tiny_cfg())
    o.set_porosity(_phi_of(theta))
    o.step(nsteps)
    s = o.state()
    return region_objective(s["u"], s["v"], s["w"], TARGETS, ut)


def test_forward_difference_descent_matches_oracle_and_descends():
    """Two porosity parameters of blocks upstream of two target regions;
    N + 1 = 3 GPU simulations of 10 steps per iteration.  Objective and
    gradient agree with forward differences over oracle simulations, and
    the descent lowers the objective."""
    nsteps, ut, eps, lam = 10, 1.0, 0.1, 0.05
    g = U.Grid(_tiny_cfg())
    J = O.SimulationObjective(g, _phi_of, TARGETS, ut, nsteps)
    theta0 = np.array([0.5, 0.7])
    theta, hist = O.gradient_descent(J, theta0, eps=eps, lam=lam, iters=2, lower=0.0, upper=1.0)
    assert J.calls == 6
    j0_ref, g0_ref = fd_gradient(lambda t: _oracle_sim(t, nsteps, ut), theta0, eps)
    log("J0", hist[0][1], j0_ref, "grad", hist[0][2], g0_ref)
    assert abs(hist[0][1] - j0_ref) <= 1e-10 * abs(j0_ref)
    assert np.allclose(hist[0][2], g0_ref, rtol=1e-8, atol=1e-9)
    assert np.allclose(hist[1][0], np.clip(theta0 - lam * hist[0][2], 0, 1), rtol=0, atol=0)
    J_end = J(theta)
    log("J history", [h[1] for h in hist], J_end)
    assert hist[1][1] < hist[0][1] and J_end < hist[1][1]
    g.close()


def test_batched_forward_differences_equal_sequential_ones():
    """The N + 1 simulations of one gradient run together (uf_step_batch)
    and give the same objective values, bit for bit, as one after another."""
    nsteps, ut = 6, 1.0
    g = U.Grid(_tiny_cfg())
    J = O.SimulationObjective(g, _phi_of, TARGETS, ut, nsteps)
    theta = np.array([0.45, 0.8])
    pts = [theta, theta + [0.1, 0.0], theta + [0.0, 0.1]]
    seq = [J(p) for p in pts]
    bat = J.many(pts)
    assert seq == bat
    j0, grad = O.forward_difference_gradient(J, theta, 0.1)
    assert j0 == seq[0]
    assert np.array_equal(grad, (np.array(seq[1:]) - seq[0]) / 0.1)
    g.close()
