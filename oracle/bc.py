"""Grid geometry, boundary kinds, inflow profile and ghost-layer rules (oracle).

Storage convention of the oracle: every field lives in a NumPy array with one
ghost layer on each side of each axis.

* u (x-faces) has interior extent (nx+1, ny, nz), v (y-faces) (nx, ny+1, nz),
  w (z-faces) (nx, ny, nz+1); cell fields (nx, ny, nz).  The padded array adds
  one layer on both ends of every axis, so element (i, j, k) of the unpadded
  range sits at [i+1, j+1, k+1].
* Face (i, j, k) of component c lies at position index (i, j, k) shifted by
  +1/2 on the two axes other than c: u(i,j,k) is at (i dx, (j+1/2) dy,
  (k+1/2) dz).  Cell (i,j,k) is centred at ((i+1/2) dx, (j+1/2) dy, (k+1/2) dz).

Boundary behaviour (Sec. 3, "Porosity Model vs. Solid-wall Boundary
Conditions"): Dirichlet velocity at the inlet, zero normal derivative at the
outlet, no-slip at solid walls, zero pressure in outlet ghost cells and zero
normal pressure derivative elsewhere.  The paper leaves the ghost treatment
open; the reading used here (both for the oracle and for the HIP path) is:

========  =======================  ===============  ============  ==========
kind      normal boundary face     tangential ghost  k, omega      pressure
========  =======================  ===============  ============  ==========
INLET     fixed: inflow normal     inflow value      inlet k, w    Neumann
OUTLET    unknown (solved)         = interior        = interior    ghost = 0
WALL      fixed: 0                 = -interior       = interior    Neumann
SLIP      fixed: 0                 = interior        = interior    Neumann
========  =======================  ===============  ============  ==========

The ghost face *beyond* a boundary normal face copies the boundary face.
Ghost layers are filled axis by axis, x first, then y, then z, each pass
covering the full padded extent of the other axes; edge and corner ghosts
thereby compose the rules of the sides they touch.
"""
import math

import numpy as np

INLET, OUTLET, WALL, SLIP = 0, 1, 2, 3
AUTO = -1

# k-omega model coefficients, Table 1 of the paper.
C_MU, ALPHA, BETA, SIGMA, SIGMA_STAR, C_LIM = 0.09, 0.52, 0.0708, 0.5, 0.6, 7.0 / 8.0


def resolve_bc(cfg):
    """Resolve AUTO side kinds: a vertical side is an inlet when the wind
    blows into the domain through it (inward normal . wind direction > 1e-12),
    an outlet otherwise; the ground is a no-slip wall and the sky a slip
    surface (Sec. 5.1 puts the outflow on the sides the wind leaves through)."""
    th = math.radians(cfg["wind_dir_deg"])
    wx, wy = math.cos(th), math.sin(th)
    inward = [(1.0, 0.0), (-1.0, 0.0), (0.0, 1.0), (0.0, -1.0)]
    out = []
    for s, kind in enumerate(cfg["bc"]):
        if kind != AUTO:
            out.append(int(kind))
        elif s < 4:
            nx_, ny_ = inward[s]
            out.append(INLET if nx_ * wx + ny_ * wy > 1e-12 else OUTLET)
        else:
            out.append(WALL if s == 4 else SLIP)
    return out


class Geometry:
    """Grid sizes, boundary kinds and inflow of one configuration."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.n = (int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"]))
        self.h = (float(cfg["dx"]), float(cfg["dy"]), float(cfg["dz"]))
        self.dt = float(cfg["dt"])
        self.bc = resolve_bc(cfg)
        th = math.radians(cfg["wind_dir_deg"])
        self.dir = (math.cos(th), math.sin(th), 0.0)
        nx, ny, nz = self.n
        self.ncell = nx * ny * nz

    # ----- extents ---------------------------------------------------------
    def face_ext(self, c):
        e = list(self.n)
        e[c] += 1
        return tuple(e)

    def face_pshape(self, c):
        return tuple(x + 2 for x in self.face_ext(c))

    def cell_pshape(self):
        return tuple(x + 2 for x in self.n)

    # ----- inflow (Sec. 5.1: log-law profile) -------------------------------
    def inflow_speed(self, k):
        """Inflow speed at the height (k+1/2) dz of vertical cell index k
        (an integer array, may include the ghost indices -1 and nz).

        Log-law u(z) = (u*/kappa) ln(z/z0) with the friction speed fixed by
        the reference speed at z_ref, u* = U_ref kappa / ln(z_ref/z0); zero at
        and below the roughness length."""
        cfg = self.cfg
        k = np.asarray(k)
        kind = cfg["inflow_kind"]
        if kind == 0:
            return np.full(k.shape, float(cfg["u_ref"]))
        if kind == 1:
            kap, z0 = float(cfg["karman"]), float(cfg["z0"])
            ustar = float(cfg["u_ref"]) * kap / math.log(float(cfg["z_ref"]) / z0)
            z = (k + 0.5) * self.h[2]
            out = np.zeros(k.shape)
            m = z > z0
            out[m] = ustar / kap * np.log(z[m] / z0)
            return out
        if kind == 2:
            prof = np.asarray(cfg["inflow_profile"], dtype=np.float64)
            return prof[np.clip(k, 0, self.n[2] - 1)]
        raise ValueError("bad inflow kind")

    def inflow_component(self, c, k):
        """Velocity component c of the inflow at vertical index k."""
        if c == 2:
            return np.zeros(np.shape(k))
        return self.inflow_speed(k) * self.dir[c]

    def turb_inlet(self):
        """Inlet k and omega (Sec. 3): k = 1.5 (I U_ref)^2,
        omega = C_mu^(-1/4) k^(1/2) / L.  L defaults to 0.1 x domain height."""
        cfg = self.cfg
        I, U = float(cfg["turb_I"]), float(cfg["u_ref"])
        L = float(cfg["turb_L"]) if cfg["turb_L"] > 0 else 0.1 * self.n[2] * self.h[2]
        k_in = 1.5 * (I * U) ** 2
        w_in = math.sqrt(k_in) / (C_MU ** 0.25 * L)
        return k_in, w_in

    def nu_max(self):
        """Largest total viscosity for which explicit 3-D diffusion is stable
        (von Neumann): nu dt (dx^-2 + dy^-2 + dz^-2) <= 1/2.  The paper derives
        its eddy-viscosity limiter from this analysis (Sec. 3, "Discretization
        and Numerical Integration"); its printed formula is dimensionally
        garbled, so the bound is restated here."""
        dx, dy, dz = self.h
        return 1.0 / (2.0 * self.dt * (dx ** -2 + dy ** -2 + dz ** -2))

    # ----- boundary application --------------------------------------------
    def apply_face_bc(self, Q, c):
        """Impose the boundary rules on padded face array Q of component c:
        Dirichlet normal faces first, then ghosts x -> y -> z (in place)."""
        ext = self.face_ext(c)
        # Dirichlet boundary normal faces (both ends of axis c)
        for end, side in ((0, 2 * c), (1, 2 * c + 1)):
            kind = self.bc[side]
            if kind == OUTLET:
                continue
            idx = [slice(None)] * 3
            idx[c] = 1 if end == 0 else ext[c]
            if kind == INLET and c != 2:
                kp = np.arange(Q.shape[2]) - 1
                Q[tuple(idx)] = self.inflow_component(c, kp)[None, :]
            else:
                Q[tuple(idx)] = 0.0
        # ghosts, one axis after the other
        for ax in range(3):
            for end in (0, 1):
                side = 2 * ax + end
                g = [slice(None)] * 3
                a = [slice(None)] * 3
                g[ax] = 0 if end == 0 else -1
                a[ax] = 1 if end == 0 else -2
                g, a = tuple(g), tuple(a)
                if ax == c:
                    Q[g] = Q[a]                 # beyond a normal face: copy
                    continue
                kind = self.bc[side]
                if kind == INLET:
                    # inflow depends on height only (vertical padded index)
                    if ax == 2:
                        kk = -1 if end == 0 else Q.shape[2] - 2
                        Q[g] = self.inflow_component(c, np.array(kk))
                    else:
                        kp = np.arange(Q.shape[2]) - 1
                        Q[g] = self.inflow_component(c, kp)[None, :]
                elif kind == WALL:
                    Q[g] = -Q[a]
                else:                            # OUTLET, SLIP
                    Q[g] = Q[a]
        return Q

    def apply_scalar_bc(self, Q, inlet_value=None):
        """Ghosts of a padded cell field: the inlet value on INLET sides when
        ``inlet_value`` is given, a copy of the interior neighbour otherwise
        (zero normal gradient).  Filled x -> y -> z."""
        for ax in range(3):
            for end in (0, 1):
                side = 2 * ax + end
                g = [slice(None)] * 3
                a = [slice(None)] * 3
                g[ax] = 0 if end == 0 else -1
                a[ax] = 1 if end == 0 else -2
                if inlet_value is not None and self.bc[side] == INLET:
                    Q[tuple(g)] = inlet_value
                else:
                    Q[tuple(g)] = Q[tuple(a)]
        return Q

    def unknown_face_mask(self, c):
        """Boolean mask over the interior extent of component c: True where
        the face is solved for (everything but non-outlet boundary normals)."""
        m = np.ones(self.face_ext(c), dtype=bool)
        idx = [slice(None)] * 3
        if self.bc[2 * c] != OUTLET:
            idx[c] = 0
            m[tuple(idx)] = False
        if self.bc[2 * c + 1] != OUTLET:
            idx[c] = -1
            m[tuple(idx)] = False
        return m


def win(Q, ext, off=(0, 0, 0)):
    """View of padded array Q over an unpadded index range [0, ext) shifted by off."""
    return Q[1 + off[0]:1 + off[0] + ext[0],
             1 + off[1]:1 + off[1] + ext[1],
             1 + off[2]:1 + off[2] + ext[2]]


def unit(d, s=1):
    o = [0, 0, 0]
    o[d] = s
    return tuple(o)
