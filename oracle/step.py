"""The stages of one time step, in float64 (oracle).

The paper integrates the terms of the RANS momentum equation one by one
(time splitting, Sec. 3 "Discretization and Numerical Integration") and
solves the turbulence model after the projection.  The order used is

    advection -> diffusion -> porosity drag -> projection -> k-omega

Every function takes and returns padded arrays (see ``bc``); boundary rules
are re-imposed on each intermediate field.
"""
import numpy as np

from .bc import (C_MU, ALPHA, BETA, SIGMA, SIGMA_STAR, C_LIM, win, unit)


# ---------------------------------------------------------------------------
# S1: velocity vector at a face
# ---------------------------------------------------------------------------
def face_velocity(g, Q, c):
    """Velocity vector at every face of component c (interior extent).

    The face's own component is stored there; each other component c' is the
    mean of its four nearest faces: offsets {-1, 0} along axis c and {0, +1}
    along axis c' (the staggered MAC arrangement, Sec. 3)."""
    ext = g.face_ext(c)
    out = [None, None, None]
    out[c] = win(Q[c], ext).copy()
    for cp in range(3):
        if cp == c:
            continue
        acc = np.zeros(ext)
        for a in (-1, 0):
            for b in (0, 1):
                off = [0, 0, 0]
                off[c] = a
                off[cp] = b
                acc += win(Q[cp], ext, off)
        out[cp] = 0.25 * acc
    return out


# ---------------------------------------------------------------------------
# S2: MacCormack semi-Lagrangian advection (Selle et al., cited in Sec. 2/3)
# ---------------------------------------------------------------------------
def trilinear(Qp, fi, fj, fk):
    """Trilinear interpolation of padded array Qp at continuous (unpadded)
    indices.  Positions are clamped to the padded extent.  Returns the value
    and the min and max of the eight samples used."""
    corner = []
    for f, n in zip((fi, fj, fk), Qp.shape):
        f = np.clip(f, -1.0, n - 2.0)
        i0 = np.minimum(np.floor(f), n - 3.0)
        corner.append((i0.astype(np.int64) + 1, f - i0))
    (i0, ti), (j0, tj), (k0, tk) = corner
    s = {}
    for a in (0, 1):
        for b in (0, 1):
            for cc in (0, 1):
                s[a, b, cc] = Qp[i0 + a, j0 + b, k0 + cc]
    c00 = s[0, 0, 0] + ti * (s[1, 0, 0] - s[0, 0, 0])
    c10 = s[0, 1, 0] + ti * (s[1, 1, 0] - s[0, 1, 0])
    c01 = s[0, 0, 1] + ti * (s[1, 0, 1] - s[0, 0, 1])
    c11 = s[0, 1, 1] + ti * (s[1, 1, 1] - s[0, 1, 1])
    c0 = c00 + tj * (c10 - c00)
    c1 = c01 + tj * (c11 - c01)
    val = c0 + tk * (c1 - c0)
    allv = np.stack(list(s.values()))
    return val, allv.min(axis=0), allv.max(axis=0)


def advect(g, Q):
    """MacCormack advection of u, v, w by the old velocity field.

    For every face f and component q: forward trace x* = x_f - dt V_f and
    q^ = I_q(x*); the intermediate field q^ gets the boundary rules; reverse
    trace x** = x_f + dt V_f and qv = I_{q^}(x**); corrected value
    q~ = q^ + (q - qv)/2 clamped to the range of the eight samples used for
    q^ (Selle's limiter).  All components read the old field."""
    dt = g.dt
    out = []
    for c in range(3):
        ext = g.face_ext(c)
        V = face_velocity(g, Q, c)
        I, J, K = np.meshgrid(np.arange(ext[0]), np.arange(ext[1]), np.arange(ext[2]),
                              indexing="ij")
        d = [V[a] * dt / g.h[a] for a in range(3)]
        qhat, qmin, qmax = trilinear(Q[c], I - d[0], J - d[1], K - d[2])
        Qhat = Q[c].copy()
        win(Qhat, ext)[...] = qhat
        g.apply_face_bc(Qhat, c)
        qchk, _, _ = trilinear(Qhat, I + d[0], J + d[1], K + d[2])
        q = win(Q[c], ext)
        qt = np.clip(qhat + 0.5 * (q - qchk), qmin, qmax)
        Qt = Q[c].copy()
        win(Qt, ext)[...] = qt
        out.append(g.apply_face_bc(Qt, c))
    return out


# ---------------------------------------------------------------------------
# S3: explicit viscous diffusion, (nu + nu_t) Laplacian u  (eq. RANS momentum)
# ---------------------------------------------------------------------------
def laplacian(Qp, ext, h):
    """7-point Laplacian of padded array Qp over the interior range ``ext``."""
    q = win(Qp, ext)
    lap = np.zeros(ext)
    for a in range(3):
        lap += (win(Qp, ext, unit(a, 1)) - 2.0 * q + win(Qp, ext, unit(a, -1))) / h[a] ** 2
    return lap


def face_mean_of_cells(g, Cp, c):
    """Mean of the two cells adjacent to each face of component c (padded
    cell array with zero-gradient ghosts, so boundary faces take the single
    interior cell)."""
    ext = g.face_ext(c)
    return 0.5 * (win(Cp, ext, unit(c, -1)) + win(Cp, ext))


def diffuse(g, Q, NUTp, nu):
    """u_bar = u + dt (nu + nu_t,f) L_h u, with nu_t,f the face mean of the
    (limited) cell eddy viscosity.  Explicit Euler, as the paper's viscosity
    limiter presumes."""
    out = []
    for c in range(3):
        ext = g.face_ext(c)
        nuf = nu + face_mean_of_cells(g, NUTp, c)
        new = Q[c].copy()
        win(new, ext)[...] = win(Q[c], ext) + g.dt * nuf * laplacian(Q[c], ext, g.h)
        out.append(g.apply_face_bc(new, c))
    return out


# ---------------------------------------------------------------------------
# S4: porosity drag, forward Euler with the non-negativity clamp (Sec. 3)
# ---------------------------------------------------------------------------
def drag_coefficient(cfg, phi):
    """Cell drag coefficient C_d a ((1 - phi)/(phi + e))^b (the drag law of
    Sec. 3 with LAD replaced by the porosity term of its footnote)."""
    return cfg["Cd"] * cfg["a"] * ((1.0 - phi) / (phi + cfg["e"])) ** cfg["b"]


def drag(g, Q, Cp):
    """u* = max(0, 1 - dt c_f |V_f|) u for every component, where c_f is the
    mean drag coefficient of the two cells next to the face and V_f the
    velocity vector at the face.  All components read the same field."""
    out = []
    for c in range(3):
        ext = g.face_ext(c)
        V = face_velocity(g, Q, c)
        speed = np.sqrt(V[0] ** 2 + V[1] ** 2 + V[2] ** 2)
        cf = face_mean_of_cells(g, Cp, c)
        fac = np.maximum(0.0, 1.0 - g.dt * cf * speed)
        new = Q[c].copy()
        win(new, ext)[...] = fac * win(Q[c], ext)
        out.append(g.apply_face_bc(new, c))
    return out


# ---------------------------------------------------------------------------
# S5: pressure projection (Sec. 3)
# ---------------------------------------------------------------------------
def divergence(g, Q):
    """Discrete divergence at cell centres from the six face values."""
    ext = g.n
    div = np.zeros(ext)
    for c in range(3):
        div += (win(Q[c], ext, unit(c, 1)) - win(Q[c], ext)) / g.h[c]
    return div


def project(g, Q, p, rho):
    """u^{n+1} = u* - (dt/rho) grad p on the solved faces; outlet faces see
    the zero ghost pressure beyond the boundary."""
    Pp = np.zeros(g.cell_pshape())
    win(Pp, g.n)[...] = p
    out = []
    for c in range(3):
        ext = g.face_ext(c)
        grad = (win(Pp, ext) - win(Pp, ext, unit(c, -1))) / g.h[c]
        new = Q[c].copy()
        win(new, ext)[...] = win(Q[c], ext) - g.dt / rho * grad
        out.append(g.apply_face_bc(new, c))
    return out


# ---------------------------------------------------------------------------
# S6: k-omega turbulence model (Sec. 3), solved after the projection
# ---------------------------------------------------------------------------
def strain_rate(g, Q):
    """Mean strain rate S = (grad u + grad u^T)/2 at cell centres.

    Normal derivatives come from the two faces of the cell; cross
    derivatives are central differences of cell-centred velocities (face
    means), with ghost faces supplying the values beyond the domain.
    Returns (|S|^2 = S_ij S_ij, cell-centred velocity components)."""
    n = g.n
    # cell-centred component c over the cell range extended by one ghost cell
    # on the two axes other than c
    cen = []
    for c in range(3):
        ext = [n[0] + 2, n[1] + 2, n[2] + 2]
        ext[c] = n[c]
        off = [-1, -1, -1]
        off[c] = 0
        a = win(Q[c], ext, off)
        o2 = list(off)
        o2[c] = 1
        b = win(Q[c], ext, o2)
        cen.append(0.5 * (a + b))          # index [i', j', k'] with +1 on the non-c axes
    G = np.zeros((3, 3) + n)               # G[c, d] = d u_c / d x_d
    for c in range(3):
        G[c, c] = (win(Q[c], n, unit(c, 1)) - win(Q[c], n)) / g.h[c]
        for d in range(3):
            if d == c:
                continue
            sl_p = [slice(None)] * 3
            sl_m = [slice(None)] * 3
            for a in range(3):
                if a == c:
                    continue
                if a == d:
                    sl_p[a] = slice(2, 2 + n[a])
                    sl_m[a] = slice(0, n[a])
                else:
                    sl_p[a] = slice(1, 1 + n[a])
                    sl_m[a] = slice(1, 1 + n[a])
            G[c, d] = (cen[c][tuple(sl_p)] - cen[c][tuple(sl_m)]) / (2.0 * g.h[d])
    S2 = np.zeros(n)
    for c in range(3):
        for d in range(3):
            S2 += (0.5 * (G[c, d] + G[d, c])) ** 2
    ucell = []
    for c in range(3):
        sl = [slice(1, 1 + n[a]) for a in range(3)]
        sl[c] = slice(None)
        ucell.append(cen[c][tuple(sl)])
    return S2, ucell


def omega_limit(S2):
    """Strain-rate bound of the omega limiter (Wilcox 2006, cited in Sec. 3):
    C_lim * |S| / sqrt(C_mu / 2) with |S| = sqrt(S_ij S_ij).  The printed
    formula drops the square root; this restates Wilcox's limiter."""
    return C_LIM * np.sqrt(S2) / np.sqrt(C_MU / 2.0)


def upwind_advection(g, ucell, Qp):
    """First-order upwind (u . grad) q at cell centres."""
    n = g.n
    q = win(Qp, n)
    adv = np.zeros(n)
    for d in range(3):
        qm = win(Qp, n, unit(d, -1))
        qp = win(Qp, n, unit(d, 1))
        ud = ucell[d]
        adv += (np.maximum(ud, 0.0) * (q - qm) + np.minimum(ud, 0.0) * (qp - q)) / g.h[d]
    return adv


def turbulence(g, Q, Kp, Wp, cfg):
    """One forward-Euler step of the k-omega model on the projected velocity.

    nu_t = k / omega~, omega~ = max(omega, omega_limit(S)), clipped to
    [0, nu_max - nu] (the paper's viscosity limiter); upwind advection,
    central Laplacian, P_k = 2 nu_t |S|^2, dissipation C_mu k omega and
    beta omega^2, omega production 2 alpha |S|^2.  Floors k_min, omega_min.
    Returns (K, W, NUT) padded, NUT being the eddy viscosity for the next
    step computed from the new k and omega."""
    n = g.n
    nu = float(cfg["nu"])
    cap = g.nu_max() - nu
    S2, ucell = strain_rate(g, Q)
    lim = omega_limit(S2)
    k = win(Kp, n)
    w = win(Wp, n)
    nut = np.minimum(np.maximum(k / np.maximum(w, lim), 0.0), cap)
    adv_k = upwind_advection(g, ucell, Kp)
    adv_w = upwind_advection(g, ucell, Wp)
    lap_k = laplacian(Kp, n, g.h)
    lap_w = laplacian(Wp, n, g.h)
    k_new = k + g.dt * (-adv_k + 2.0 * nut * S2 - C_MU * k * w + (nu + SIGMA_STAR * nut) * lap_k)
    w_new = w + g.dt * (-adv_w + 2.0 * ALPHA * S2 - BETA * w * w + (nu + SIGMA * nut) * lap_w)
    k_new = np.maximum(k_new, float(cfg["k_min"]))
    w_new = np.maximum(w_new, float(cfg["omega_min"]))
    nut_new = np.minimum(np.maximum(k_new / np.maximum(w_new, lim), 0.0), cap)
    k_in, w_in = g.turb_inlet()
    K2 = np.zeros(g.cell_pshape())
    W2 = np.zeros(g.cell_pshape())
    N2 = np.zeros(g.cell_pshape())
    win(K2, n)[...] = k_new
    win(W2, n)[...] = w_new
    win(N2, n)[...] = nut_new
    g.apply_scalar_bc(K2, k_in)
    g.apply_scalar_bc(W2, w_in)
    g.apply_scalar_bc(N2)
    return K2, W2, N2


def eddy_viscosity(g, Q, Kp, Wp, cfg):
    """nu_t from k, omega and the strain rate of Q (used for the initial
    state): clip(k / max(omega, omega_limit), 0, nu_max - nu)."""
    S2, _ = strain_rate(g, Q)
    cap = g.nu_max() - float(cfg["nu"])
    n = g.n
    nut = np.minimum(np.maximum(win(Kp, n) / np.maximum(win(Wp, n), omega_limit(S2)), 0.0), cap)
    N2 = np.zeros(g.cell_pshape())
    win(N2, n)[...] = nut
    return g.apply_scalar_bc(N2)
