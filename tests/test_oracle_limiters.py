"""Pins of the oracle's limiters, floors and side-kind resolution.

Each expected value here is worked out by hand from the definition the
oracle follows, in scalar arithmetic that shares nothing with the oracle's
array code:

* the MacCormack clamp (Selle et al.'s limiter, cited for the advection in
  Sec. 2/3): in one dimension with a uniform carrier velocity the forward
  trace, the reverse trace and the correction are two-point interpolations
  that a test can write out, and the clamp keeps the corrected value inside
  the range of the samples the forward trace read;
* the eddy-viscosity cap of Sec. 3, restated as the von Neumann bound of
  explicit 3-D diffusion, nu_t <= 1/(2 dt (dx^-2 + dy^-2 + dz^-2)) - nu;
* the floors k >= k_min and omega >= omega_min of the k-omega update;
* the automatic side kinds: an inlet where the wind enters the domain, an
  outlet elsewhere on the vertical sides, a no-slip ground and a slip sky.
"""
import math

import numpy as np
import pytest

from uf_layouts import default_config
from uf_layouts.configs import (BC_AUTO, BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP, INFLOW_UNIFORM,
                                STAGE_ADVECT)
from oracle import OracleGrid, Geometry, resolve_bc
from oracle import step as S
from oracle import bc as B

I, O, W, SL = BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP


# ------------------------------------------------------ MacCormack clamp ----
def _carrier_cfg(nx, U, dt, dx):
    """Uniform carrier u = U along +x, advection only, outlets on the y sides
    (so a field that is constant in y stays constant in y)."""
    return default_config(nx, 4, 3, dx, dt=dt, inflow_kind=INFLOW_UNIFORM, u_ref=U, nu=0.0,
                          stages=STAGE_ADVECT, bc=[I, O, O, O, SL, SL])


def _maccormack_1d(f, c, clamp="forward"):
    """One MacCormack step of the profile f on a uniform carrier of CFL c in
    (0, 1), written out point by point.

    forward trace from x_i lands at i - c:   qh_i = c f[i-1] + (1 - c) f[i]
    reverse trace from x_i lands at i + c:   qc_i = (1 - c) qh_i + c qh_{i+1}
    corrected value:                         q_i  = qh_i + (f[i] - qc_i) / 2
    clamp "forward": into [min, max] of f[i-1], f[i] (the forward samples);
    "reverse": into the range of qh_i, qh_{i+1}; None: no clamp.
    Returns values for i = 1 .. len(f) - 2 (index i - 1) and the unclamped ones."""
    n = len(f)
    qh = [None] * n
    for i in range(1, n):
        qh[i] = c * f[i - 1] + (1.0 - c) * f[i]
    out, raw = [], []
    for i in range(1, n - 1):
        qc = (1.0 - c) * qh[i] + c * qh[i + 1]
        q = qh[i] + 0.5 * (f[i] - qc)
        raw.append(q)
        if clamp == "forward":
            lo, hi = min(f[i - 1], f[i]), max(f[i - 1], f[i])
        elif clamp == "reverse":
            lo, hi = min(qh[i], qh[i + 1]), max(qh[i], qh[i + 1])
        else:
            lo, hi = -math.inf, math.inf
        out.append(min(max(q, lo), hi))
    return np.array(out), np.array(raw)


def test_maccormack_clamp_to_forward_samples_random_profile():
    nx, U, dt, dx = 24, 1.0, 0.4, 1.0          # CFL 0.4
    c = U * dt / dx
    f = np.random.default_rng(11).normal(size=nx)
    og = OracleGrid(_carrier_cfg(nx, U, dt, dx))
    og.set_field("v", np.repeat(np.repeat(f[:, None, None], 5, axis=1), 3, axis=2))
    og.step(1)
    out = og.get_field("v")
    expect, raw = _maccormack_1d(list(f), c, "forward")
    rev, _ = _maccormack_1d(list(f), c, "reverse")
    # faces 1 .. nx-2 map to expect[0 ..]; stay two faces away from the inlet
    # ghost and the outlet's zero-gradient ghost
    sel = slice(2, nx - 3)
    got = out[sel]
    exp = expect[1:nx - 4]
    assert np.abs(got - exp[:, None, None]).max() < 1e-13
    # the clamp is active on several faces and changes the value there ...
    clamped = np.abs(raw[1:nx - 4] - exp) > 1e-3
    assert clamped.sum() >= 3, clamped.sum()
    # ... and clamping to the reverse trace's samples would differ
    assert np.abs(rev[1:nx - 4] - exp).max() > 1e-3


@pytest.mark.parametrize("up", [True, False])
def test_maccormack_clamp_at_a_step(up):
    """A unit step (up or down) at face s: in front of it the correction
    over- or undershoots by c (1 - c) / 2 and the clamp takes it back to the
    flat side exactly; at the step itself the value is 1 - c/2 - c^2/2
    (up) or c/2 + c^2/2 (down), inside the range, unclamped."""
    nx, U, dt, dx, s = 20, 1.0, 0.35, 1.0, 10
    c = U * dt / dx
    f = np.where(np.arange(nx) >= s, 1.0, 0.0) if up else np.where(np.arange(nx) >= s, 0.0, 1.0)
    og = OracleGrid(_carrier_cfg(nx, U, dt, dx))
    og.set_field("v", np.repeat(np.repeat(f[:, None, None], 5, axis=1), 3, axis=2))
    og.step(1)
    out = og.get_field("v")
    flat = 0.0 if up else 1.0
    # unclamped, face s-1 would be flat -/+ c (1 - c)/2
    assert abs(out[s - 1] - flat).max() < 1e-15
    at_step = 1.0 - c / 2 - c * c / 2 if up else c / 2 + c * c / 2
    assert abs(out[s] - at_step).max() < 1e-13
    assert abs(out[s + 2] - (1.0 - flat)).max() < 1e-15


def test_trilinear_range_is_the_eight_corner_samples():
    """The clamp range comes from the eight samples of the interpolation
    cell: brute force over random positions of a random 3-D array, including
    positions past the padded extent (clamped to it)."""
    rng = np.random.default_rng(5)
    Qp = rng.normal(size=(7, 6, 5))
    pos = [rng.uniform(-2.5, n - 0.5, size=200) for n in (5, 4, 3)]
    val, lo, hi = S.trilinear(Qp, *pos)
    for q in range(200):
        idx, frac = [], []
        for a, n in enumerate(Qp.shape):
            x = min(max(pos[a][q], -1.0), n - 2.0)     # unpadded index range of the padded array
            i0 = min(math.floor(x), n - 3)
            idx.append(i0 + 1)
            frac.append(x - i0)
        corners = [Qp[idx[0] + a, idx[1] + b, idx[2] + d] for a in (0, 1) for b in (0, 1) for d in (0, 1)]
        assert lo[q] == min(corners) and hi[q] == max(corners)
        w = 0.0
        for a in (0, 1):
            for b in (0, 1):
                for d in (0, 1):
                    wt = ((frac[0] if a else 1 - frac[0]) * (frac[1] if b else 1 - frac[1]) *
                          (frac[2] if d else 1 - frac[2]))
                    w += wt * Qp[idx[0] + a, idx[1] + b, idx[2] + d]
        assert abs(val[q] - w) < 1e-13


# ------------------------------------------------------ eddy-viscosity cap ----
def _uniform_faces(g, U):
    Q = []
    for c in range(3):
        q = np.zeros(g.face_pshape(c))
        if c == 0:
            q[...] = U
        Q.append(q)
    return Q


def test_nut_cap_is_the_explicit_diffusion_bound():
    """k / omega far above the bound: nu_t, the k diffusion and the new nu_t
    all use 1/(2 dt (dx^-2 + dy^-2 + dz^-2)) - nu, evaluated here with the
    grid's own numbers (anisotropic cells, nu large enough to matter)."""
    dx, dy, dz, dt, nu = 1.0, 0.8, 1.3, 0.1, 0.01
    cfg = default_config(10, 6, 6, dx, dy=dy, dz=dz, dt=dt, nu=nu, inflow_kind=INFLOW_UNIFORM, u_ref=2.0,
                         bc=[I, O, SL, SL, SL, SL])
    g = Geometry(cfg)
    cap = 1.0 / (2 * 0.1 * (1.0 / 1.0 + 1.0 / 0.64 + 1.0 / 1.69)) - 0.01
    assert abs(cap - 1.5751800) < 1e-6
    x = (np.arange(12) - 0.5) * dx
    a, b2 = 40.0, 0.3
    kprof = a + b2 * x * x                       # L_x k = 2 b2 exactly
    Kp = np.broadcast_to(kprof[:, None, None], g.cell_pshape()).copy()
    w0 = 1e-3                                     # k / omega = 4e4 >> cap
    Wp = np.full(g.cell_pshape(), w0)
    K2, W2, N2 = S.turbulence(g, _uniform_faces(g, 2.0), Kp, Wp, cfg)
    xi, k = x[1:-1], kprof[1:-1]
    upwind = b2 * (2 * xi - dx)                   # (k_i - k_{i-1}) / dx
    k_exp = k + dt * (-2.0 * upwind - 0.09 * k * w0 + (nu + 0.6 * cap) * 2 * b2)
    w_exp = w0 + dt * (-0.0708 * w0 * w0)
    got = K2[2:-2, 2, 2]
    assert np.allclose(got, k_exp[1:-1], rtol=1e-13)
    assert np.allclose(W2[2:-2, 2, 2], w_exp, rtol=1e-13)
    # the new eddy viscosity sits at the cap too (k_new / omega_new >> cap)
    assert np.all(np.abs(B.win(N2, g.n) - cap) <= 1e-14 * cap)
    # and the diffusion of the momentum reads it through the face mean
    NUTp = g.apply_scalar_bc(N2.copy())
    assert np.allclose(S.face_mean_of_cells(g, NUTp, 0), cap, rtol=1e-14)


def test_nut_cap_zero_when_nu_reaches_the_bound():
    """With nu at the stability bound the cap is 0: no eddy viscosity at all."""
    dx, dt = 1.0, 0.1
    bound = 1.0 / (2 * dt * 3.0 / dx ** 2)
    cfg = default_config(6, 4, 4, dx, dt=dt, nu=bound, inflow_kind=INFLOW_UNIFORM, u_ref=1.0,
                         bc=[I, O, SL, SL, SL, SL])
    g = Geometry(cfg)
    Kp = np.full(g.cell_pshape(), 2.0)
    Wp = np.full(g.cell_pshape(), 0.5)
    _, _, N2 = S.turbulence(g, _uniform_faces(g, 1.0), Kp, Wp, cfg)
    assert np.abs(N2).max() <= 1e-15


# ------------------------------------------------------ k and omega floors ----
def test_k_and_omega_floors():
    """dt C_mu omega > 1 drives k negative and dt beta omega > 1 drives omega
    negative in one explicit step (uniform fields, no strain): both end at
    their floors exactly, and nu_t = k_min / omega_min."""
    dt = 0.5
    cfg = default_config(8, 4, 4, 1.0, dt=dt, inflow_kind=INFLOW_UNIFORM, u_ref=1.0,
                         k_min=2e-6, omega_min=3e-4, bc=[I, O, SL, SL, SL, SL])
    g = Geometry(cfg)
    w0 = 40.0                                      # dt C_mu w0 = 1.8, dt beta w0 = 1.416
    assert dt * 0.09 * w0 > 1 and dt * 0.0708 * w0 > 1
    Kp = np.full(g.cell_pshape(), 0.7)
    Wp = np.full(g.cell_pshape(), w0)
    K2, W2, N2 = S.turbulence(g, _uniform_faces(g, 1.0), Kp, Wp, cfg)
    assert np.all(B.win(K2, g.n) == 2e-6)
    assert np.all(B.win(W2, g.n) == 3e-4)
    assert np.allclose(B.win(N2, g.n), 2e-6 / 3e-4, rtol=1e-14)
    # one floor only: a milder omega keeps k above its floor
    Wp[...] = 5.0                                  # dt C_mu 5 = 0.225, dt beta 5 = 0.177
    K3, W3, _ = S.turbulence(g, _uniform_faces(g, 1.0), Kp, Wp, cfg)
    assert np.allclose(B.win(K3, g.n), 0.7 * (1 - dt * 0.09 * 5.0), rtol=1e-14)
    assert np.allclose(B.win(W3, g.n), 5.0 - dt * 0.0708 * 25.0, rtol=1e-14)


# ------------------------------------------------------ automatic side kinds --
@pytest.mark.parametrize("deg,expect", [
    (0.0, [I, O, O, O, W, SL]),          # wind +x enters through -x
    (90.0, [O, O, I, O, W, SL]),         # +y: through -y; cos 90 deg ~ 6e-17 is tangential
    (180.0, [O, I, O, O, W, SL]),        # -x: through +x; sin 180 deg ~ 1e-16 is tangential
    (225.0, [O, I, O, I, W, SL]),        # (-1, -1)/sqrt 2: through +x and +y
    (270.0, [O, O, O, I, W, SL]),        # -y: through +y
    (30.0, [I, O, I, O, W, SL]),
    (-90.0, [O, O, O, I, W, SL]),
])
def test_resolve_bc_auto(deg, expect):
    cfg = default_config(8, 6, 4, 1.0, wind_dir_deg=deg)
    assert resolve_bc(cfg) == expect


def test_resolve_bc_explicit_kinds_override_and_tolerance():
    cfg = default_config(8, 6, 4, 1.0, wind_dir_deg=45.0, bc=[O, BC_AUTO, W, BC_AUTO, SL, BC_AUTO])
    assert resolve_bc(cfg) == [O, O, W, O, SL, SL]
    # a wind a hair off tangential (inward component 1e-9 > 1e-12) enters
    deg = math.degrees(math.acos(1e-9))           # cos = 1e-9: +x component just positive
    assert resolve_bc(default_config(8, 6, 4, 1.0, wind_dir_deg=deg))[0] == I
    deg = math.degrees(math.acos(1e-13))          # below the 1e-12 tolerance: tangential
    assert resolve_bc(default_config(8, 6, 4, 1.0, wind_dir_deg=deg))[0] == O
