"""OracleGrid: the oracle's mirror of the library calls (create_grid,
set_porosity, set_field/get_field, step), all in float64 on the CPU.

Initial state (the paper does not state one): every face carries the inflow
profile of its height, k and omega their inlet values, p = 0, and nu_t is
computed from them.
"""
import numpy as np

from .bc import Geometry, win
from . import step as S
from .pressure import PressureSolver

FIELDS = ("u", "v", "w", "p", "k", "omega", "nut", "phi")

ADVECT, DIFFUSE, DRAG, PROJECT, TURB = 1, 2, 4, 8, 16


class OracleGrid:
    def __init__(self, cfg, solver="auto", solver_tol=1e-12):
        self.cfg = dict(cfg)
        g = self.g = Geometry(self.cfg)
        if g.nu_max() - float(cfg["nu"]) < 0:
            raise ValueError("nu exceeds the explicit-diffusion stability bound")
        if 1 not in g.bc:
            raise ValueError("at least one outlet side is required")
        self.pressure = PressureSolver(g, method=solver, tol=solver_tol)
        self.turb_on = int(cfg["turb_model"]) != 0
        # porosity 1 everywhere until set
        self.phi = np.ones(g.n)
        self.C = np.zeros(g.cell_pshape())
        self.Q = []
        for c in range(3):
            Qc = np.zeros(g.face_pshape(c))
            ext = g.face_ext(c)
            kk = np.arange(ext[2])
            win(Qc, ext)[...] = g.inflow_component(c, kk)[None, None, :]
            self.Q.append(g.apply_face_bc(Qc, c))
        self.p = np.zeros(g.n)
        k_in, w_in = g.turb_inlet()
        self.K = g.apply_scalar_bc(np.full(g.cell_pshape(), k_in), k_in)
        self.W = g.apply_scalar_bc(np.full(g.cell_pshape(), w_in), w_in)
        self._refresh_nut()
        self.last_stats = {}

    def _refresh_nut(self):
        if self.turb_on:
            self.NUT = S.eddy_viscosity(self.g, self.Q, self.K, self.W, self.cfg)
        else:
            self.NUT = np.zeros(self.g.cell_pshape())

    # ----- inputs ----------------------------------------------------------
    def set_porosity(self, phi):
        phi = np.asarray(phi, dtype=np.float64).reshape(self.g.n)
        if not np.all(np.isfinite(phi)) or phi.min() < 0.0 or phi.max() > 1.0:
            raise ValueError("porosity must be finite and in [0, 1]")
        self.phi = phi.copy()
        C = np.zeros(self.g.cell_pshape())
        win(C, self.g.n)[...] = S.drag_coefficient(self.cfg, phi)
        self.C = self.g.apply_scalar_bc(C)

    def set_field(self, name, arr):
        g = self.g
        arr = np.asarray(arr, dtype=np.float64)
        if name in ("u", "v", "w"):
            c = "uvw".index(name)
            ext = g.face_ext(c)
            win(self.Q[c], ext)[...] = arr.reshape(ext)
            g.apply_face_bc(self.Q[c], c)
        elif name == "p":
            self.p = arr.reshape(g.n).copy()
        elif name in ("k", "omega"):
            k_in, w_in = g.turb_inlet()
            P, v = (self.K, k_in) if name == "k" else (self.W, w_in)
            win(P, g.n)[...] = arr.reshape(g.n)
            g.apply_scalar_bc(P, v)
        elif name == "nut":
            win(self.NUT, g.n)[...] = arr.reshape(g.n)
            g.apply_scalar_bc(self.NUT)
        elif name == "phi":
            self.set_porosity(arr)
        else:
            raise KeyError(name)

    def get_field(self, name):
        g = self.g
        if name in ("u", "v", "w"):
            c = "uvw".index(name)
            return win(self.Q[c], g.face_ext(c)).copy()
        if name == "p":
            return self.p.copy()
        if name == "k":
            return win(self.K, g.n).copy()
        if name == "omega":
            return win(self.W, g.n).copy()
        if name == "nut":
            return win(self.NUT, g.n).copy()
        if name == "phi":
            return self.phi.copy()
        raise KeyError(name)

    def state(self):
        return {f: self.get_field(f) for f in FIELDS if f != "phi"}

    # ----- time stepping -----------------------------------------------------
    def step(self, nsteps=1):
        """Advance ``nsteps`` steps; returns the stats of the last one."""
        for _ in range(nsteps):
            self.last_stats = self._one_step()
        return self.last_stats

    def _one_step(self):
        g, cfg = self.g, self.cfg
        st = int(cfg["stages"])
        rho, nu = float(cfg["rho"]), float(cfg["nu"])
        Q = self.Q
        stats = dict(cg_iters=0, max_div=0.0)
        if st & ADVECT:
            Q = S.advect(g, Q)
        if st & DIFFUSE:
            Q = S.diffuse(g, Q, self.NUT, nu)
        if st & DRAG:
            Q = S.drag(g, Q, self.C)
        if st & PROJECT:
            b = -(rho / g.dt) * S.divergence(g, Q)
            p, it = self.pressure.solve(b.ravel(), self.p.ravel())
            self.p = p.reshape(g.n)
            stats["cg_iters"] = it
            Q = S.project(g, Q, self.p, rho)
            stats["max_div"] = float(np.abs(S.divergence(g, Q)).max())
        if (st & TURB) and self.turb_on:
            self.K, self.W, self.NUT = S.turbulence(g, Q, self.K, self.W, cfg)
        self.Q = Q
        return stats
