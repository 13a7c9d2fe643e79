"""Discrete adjoint of the oracle's time step -- TEST INFRASTRUCTURE ONLY.

The oracle's step (advection, diffusion, drag, projection, k-omega; see
``step`` and ``solver``) restated operation by operation with float64 torch
tensors on the CPU, so that torch.autograd yields its exact discrete
adjoint: the vector-Jacobian product of one step with respect to the state
it starts from and to the cell porosity.  The arithmetic follows the NumPy
oracle one to one (same formulas, same order, same boundary rules, the same
ghost-padded arrays); the pressure solve is an autograd Function whose
backward is the same solve, since the Poisson matrix is symmetric.

Where the step takes a max, min or clamp, autograd follows the branch the
forward took (a MacCormack value clamped to its sample range takes that
sample's derivative, a face the drag stops passes nothing, a floored k or
omega and a clipped nu_t pass nothing through the clipped argument); at an
exact tie torch splits or picks a side by its own rule, so comparisons use
states where ties do not occur.  The square roots of the strain-rate limiter
and of the face speed are given a zero derivative where their argument is
exactly zero (the value there is 0 either way).

Pins (tests/test_oracle_adjoint.py): the forward equals the NumPy oracle's
step to rounding; the products equal central differences of the NumPy
oracle's step, directionally and per element.
"""
import numpy as np
import torch

from .bc import (Geometry, INLET, OUTLET, WALL, C_MU, ALPHA, BETA, SIGMA, SIGMA_STAR, C_LIM)
from .pressure import PressureSolver
from .solver import ADVECT, DIFFUSE, DRAG, PROJECT, TURB

F64 = torch.float64


def win(Q, ext, off=(0, 0, 0)):
    return Q[1 + off[0]:1 + off[0] + ext[0],
             1 + off[1]:1 + off[1] + ext[1],
             1 + off[2]:1 + off[2] + ext[2]]


def unit(d, s=1):
    o = [0, 0, 0]
    o[d] = s
    return tuple(o)


def _const(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def _sqrt0(x):
    """sqrt with a zero derivative at exactly 0."""
    pos = x > 0
    return torch.where(pos, torch.sqrt(torch.clamp(x, min=1e-300)), torch.zeros_like(x))


class _PressureSolve(torch.autograd.Function):
    """p = A^-1 b with the oracle's solver; the adjoint is A^-1 again (A = A^T)."""

    @staticmethod
    def forward(ctx, b, solver):
        ctx.solver = solver
        shape = b.shape
        x, _ = solver.solve(b.detach().numpy().ravel(), np.zeros(b.numel()))
        return torch.as_tensor(x.reshape(shape))

    @staticmethod
    def backward(ctx, gp):
        y, _ = ctx.solver.solve(gp.detach().numpy().ravel(), np.zeros(gp.numel()))
        return torch.as_tensor(y.reshape(gp.shape)), None


class TorchStep:
    """One oracle step on torch tensors.  ``cfg`` as for OracleGrid; the
    pressure solver is the oracle's ('direct' for small grids)."""

    def __init__(self, cfg, solver="auto"):
        self.cfg = dict(cfg)
        self.g = Geometry(self.cfg)
        self.pressure = PressureSolver(self.g, method=solver)
        self.turb_on = int(cfg["turb_model"]) != 0

    # --------------------------------------------------- boundary rules ----
    def face_bc(self, Q, c):
        """Boundary rules of face array Q (component c) as the oracle's
        Geometry.apply_face_bc: Dirichlet normal faces, then ghosts x, y, z."""
        g = self.g
        Q = Q.clone()
        ext = g.face_ext(c)
        for end, side in ((0, 2 * c), (1, 2 * c + 1)):
            kind = g.bc[side]
            if kind == OUTLET:
                continue
            idx = [slice(None)] * 3
            idx[c] = 1 if end == 0 else ext[c]
            if kind == INLET and c != 2:
                kp = np.arange(Q.shape[2]) - 1
                Q[tuple(idx)] = _const(g.inflow_component(c, kp))[None, :].expand_as(Q[tuple(idx)])
            else:
                Q[tuple(idx)] = 0.0
        for ax in range(3):
            for end in (0, 1):
                side = 2 * ax + end
                gs = [slice(None)] * 3
                a = [slice(None)] * 3
                gs[ax] = 0 if end == 0 else -1
                a[ax] = 1 if end == 0 else -2
                gs, a = tuple(gs), tuple(a)
                if ax == c:
                    Q[gs] = Q[a]
                    continue
                kind = g.bc[side]
                if kind == INLET:
                    if ax == 2:
                        kk = -1 if end == 0 else Q.shape[2] - 2
                        Q[gs] = float(g.inflow_component(c, np.array(kk)))
                    else:
                        kp = np.arange(Q.shape[2]) - 1
                        Q[gs] = _const(g.inflow_component(c, kp))[None, :].expand_as(Q[gs])
                elif kind == WALL:
                    Q[gs] = -Q[a]
                else:
                    Q[gs] = Q[a]
        return Q

    def scalar_bc(self, Q, inlet_value=None):
        """Ghosts of a cell array as Geometry.apply_scalar_bc."""
        g = self.g
        Q = Q.clone()
        for ax in range(3):
            for end in (0, 1):
                side = 2 * ax + end
                gs = [slice(None)] * 3
                a = [slice(None)] * 3
                gs[ax] = 0 if end == 0 else -1
                a[ax] = 1 if end == 0 else -2
                if inlet_value is not None and g.bc[side] == INLET:
                    Q[tuple(gs)] = float(inlet_value)
                else:
                    Q[tuple(gs)] = Q[tuple(a)]
        return Q

    def _pad_face(self, x, c):
        g = self.g
        Q = torch.zeros(g.face_pshape(c), dtype=F64)
        win(Q, g.face_ext(c))[...] = x
        return self.face_bc(Q, c)

    def _pad_cell(self, x, inlet_value=None):
        g = self.g
        Q = torch.zeros(g.cell_pshape(), dtype=F64)
        win(Q, g.n)[...] = x
        return self.scalar_bc(Q, inlet_value)

    # ----------------------------------------------------------- stages ----
    def face_velocity(self, Q, c):
        g = self.g
        ext = g.face_ext(c)
        out = [None, None, None]
        out[c] = win(Q[c], ext)
        for cp in range(3):
            if cp == c:
                continue
            acc = torch.zeros(ext, dtype=F64)
            for a in (-1, 0):
                for b in (0, 1):
                    off = [0, 0, 0]
                    off[c] = a
                    off[cp] = b
                    acc = acc + win(Q[cp], ext, off)
            out[cp] = 0.25 * acc
        return out

    @staticmethod
    def trilinear(Qp, fi, fj, fk):
        corner = []
        for f, n in zip((fi, fj, fk), Qp.shape):
            f = torch.clamp(f, -1.0, n - 2.0)
            i0 = torch.clamp(torch.floor(f), max=n - 3.0).detach()
            corner.append((i0.long() + 1, f - i0))
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
        allv = torch.stack(list(s.values()))
        return val, allv.min(dim=0).values, allv.max(dim=0).values

    def advect(self, Q):
        g = self.g
        out = []
        for c in range(3):
            ext = g.face_ext(c)
            V = self.face_velocity(Q, c)
            I, J, K = torch.meshgrid(torch.arange(ext[0], dtype=F64), torch.arange(ext[1], dtype=F64),
                                     torch.arange(ext[2], dtype=F64), indexing="ij")
            d = [V[a] * g.dt / g.h[a] for a in range(3)]
            qhat, qmin, qmax = self.trilinear(Q[c], I - d[0], J - d[1], K - d[2])
            Qhat = Q[c].clone()
            win(Qhat, ext)[...] = qhat
            Qhat = self.face_bc(Qhat, c)
            qchk, _, _ = self.trilinear(Qhat, I + d[0], J + d[1], K + d[2])
            q = win(Q[c], ext)
            qt = torch.clamp(qhat + 0.5 * (q - qchk), min=qmin, max=qmax)
            Qt = Q[c].clone()
            win(Qt, ext)[...] = qt
            out.append(self.face_bc(Qt, c))
        return out

    @staticmethod
    def laplacian(Qp, ext, h):
        q = win(Qp, ext)
        lap = torch.zeros(ext, dtype=F64)
        for a in range(3):
            lap = lap + (win(Qp, ext, unit(a, 1)) - 2.0 * q + win(Qp, ext, unit(a, -1))) / h[a] ** 2
        return lap

    def face_mean_of_cells(self, Cp, c):
        ext = self.g.face_ext(c)
        return 0.5 * (win(Cp, ext, unit(c, -1)) + win(Cp, ext))

    def diffuse(self, Q, NUTp, nu):
        g = self.g
        out = []
        for c in range(3):
            ext = g.face_ext(c)
            nuf = nu + self.face_mean_of_cells(NUTp, c)
            new = Q[c].clone()
            win(new, ext)[...] = win(Q[c], ext) + g.dt * nuf * self.laplacian(Q[c], ext, g.h)
            out.append(self.face_bc(new, c))
        return out

    def drag_coefficient(self, phi):
        cfg = self.cfg
        return cfg["Cd"] * cfg["a"] * ((1.0 - phi) / (phi + cfg["e"])) ** cfg["b"]

    def drag(self, Q, Cp):
        g = self.g
        out = []
        for c in range(3):
            ext = g.face_ext(c)
            V = self.face_velocity(Q, c)
            speed = _sqrt0(V[0] ** 2 + V[1] ** 2 + V[2] ** 2)
            cf = self.face_mean_of_cells(Cp, c)
            fac = torch.clamp(1.0 - g.dt * cf * speed, min=0.0)
            new = Q[c].clone()
            win(new, ext)[...] = fac * win(Q[c], ext)
            out.append(self.face_bc(new, c))
        return out

    def divergence(self, Q):
        g = self.g
        div = torch.zeros(g.n, dtype=F64)
        for c in range(3):
            div = div + (win(Q[c], g.n, unit(c, 1)) - win(Q[c], g.n)) / g.h[c]
        return div

    def project(self, Q, p, rho):
        g = self.g
        Pp = torch.zeros(g.cell_pshape(), dtype=F64)
        win(Pp, g.n)[...] = p
        out = []
        for c in range(3):
            ext = g.face_ext(c)
            grad = (win(Pp, ext) - win(Pp, ext, unit(c, -1))) / g.h[c]
            new = Q[c].clone()
            win(new, ext)[...] = win(Q[c], ext) - g.dt / rho * grad
            out.append(self.face_bc(new, c))
        return out

    def strain_rate(self, Q):
        g = self.g
        n = g.n
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
            cen.append(0.5 * (a + b))
        G = [[None] * 3 for _ in range(3)]
        for c in range(3):
            G[c][c] = (win(Q[c], n, unit(c, 1)) - win(Q[c], n)) / g.h[c]
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
                G[c][d] = (cen[c][tuple(sl_p)] - cen[c][tuple(sl_m)]) / (2.0 * g.h[d])
        S2 = torch.zeros(n, dtype=F64)
        for c in range(3):
            for d in range(3):
                S2 = S2 + (0.5 * (G[c][d] + G[d][c])) ** 2
        ucell = []
        for c in range(3):
            sl = [slice(1, 1 + n[a]) for a in range(3)]
            sl[c] = slice(None)
            ucell.append(cen[c][tuple(sl)])
        return S2, ucell

    @staticmethod
    def omega_limit(S2):
        return C_LIM * _sqrt0(S2) / np.sqrt(C_MU / 2.0)

    def upwind_advection(self, ucell, Qp):
        g = self.g
        n = g.n
        q = win(Qp, n)
        adv = torch.zeros(n, dtype=F64)
        for d in range(3):
            qm = win(Qp, n, unit(d, -1))
            qp = win(Qp, n, unit(d, 1))
            ud = ucell[d]
            adv = adv + (torch.clamp(ud, min=0.0) * (q - qm) + torch.clamp(ud, max=0.0) * (qp - q)) / g.h[d]
        return adv

    def turbulence(self, Q, Kp, Wp):
        g, cfg = self.g, self.cfg
        n = g.n
        nu = float(cfg["nu"])
        cap = g.nu_max() - nu
        S2, ucell = self.strain_rate(Q)
        lim = self.omega_limit(S2)
        k = win(Kp, n)
        w = win(Wp, n)
        nut = torch.clamp(k / torch.maximum(w, lim), min=0.0, max=cap)
        adv_k = self.upwind_advection(ucell, Kp)
        adv_w = self.upwind_advection(ucell, Wp)
        lap_k = self.laplacian(Kp, n, g.h)
        lap_w = self.laplacian(Wp, n, g.h)
        k_new = k + g.dt * (-adv_k + 2.0 * nut * S2 - C_MU * k * w + (nu + SIGMA_STAR * nut) * lap_k)
        w_new = w + g.dt * (-adv_w + 2.0 * ALPHA * S2 - BETA * w * w + (nu + SIGMA * nut) * lap_w)
        k_new = torch.clamp(k_new, min=float(cfg["k_min"]))
        w_new = torch.clamp(w_new, min=float(cfg["omega_min"]))
        nut_new = torch.clamp(k_new / torch.maximum(w_new, lim), min=0.0, max=cap)
        k_in, w_in = g.turb_inlet()
        return self._pad_cell(k_new, k_in), self._pad_cell(w_new, w_in), self._pad_cell(nut_new)

    # ------------------------------------------------------------- step ----
    def step(self, state, phi):
        """One step from ``state`` (dict of compact tensors: u, v, w, p, k,
        omega, nut) with cell porosity ``phi``; returns the new compact
        state.  Mirrors OracleGrid._one_step."""
        g, cfg = self.g, self.cfg
        stg = int(cfg["stages"])
        rho, nu = float(cfg["rho"]), float(cfg["nu"])
        Q = [self._pad_face(state[f], c) for c, f in enumerate("uvw")]
        Cp = self._pad_cell(self.drag_coefficient(phi))
        k_in, w_in = g.turb_inlet()
        Kp = self._pad_cell(state["k"], k_in)
        Wp = self._pad_cell(state["omega"], w_in)
        NUTp = self._pad_cell(state["nut"])
        p = state["p"]
        if stg & ADVECT:
            Q = self.advect(Q)
        if stg & DIFFUSE:
            Q = self.diffuse(Q, NUTp, nu)
        if stg & DRAG:
            Q = self.drag(Q, Cp)
        if stg & PROJECT:
            b = -(rho / g.dt) * self.divergence(Q)
            p = _PressureSolve.apply(b, self.pressure)
            Q = self.project(Q, p, rho)
        if (stg & TURB) and self.turb_on:
            Kp, Wp, NUTp = self.turbulence(Q, Kp, Wp)
        out = {f: win(Q[c], g.face_ext(c)) for c, f in enumerate("uvw")}
        out.update(p=p, k=win(Kp, g.n), omega=win(Wp, g.n), nut=win(NUTp, g.n))
        return out


def state_fields(cfg):
    """Fields the reverse step carries: (u, v, w), plus (k, omega, nut) when
    the k-omega update runs in the step."""
    turb = int(cfg["turb_model"]) != 0 and int(cfg["stages"]) & TURB
    return ("u", "v", "w", "k", "omega", "nut") if turb else ("u", "v", "w")


def adjoint_steps(cfg, state, phi, seed, nsteps=1, solver="auto"):
    """Vector-Jacobian product of ``nsteps`` oracle steps.

    state: dict of compact float64 arrays (u, v, w, p, k, omega, nut);
    phi: cell porosity; seed: dict of dJ/dx for the fields of
    state_fields(cfg) after the last step.  Returns (adj, phibar, final)
    with adj = dJ/dx for those fields at the first step's start, phibar =
    dJ/dphi summed over the steps, and the final state (NumPy)."""
    ts = TorchStep(cfg, solver)
    fields = state_fields(cfg)
    x0 = {f: torch.tensor(np.asarray(state[f], dtype=np.float64), requires_grad=f in fields)
          for f in ("u", "v", "w", "p", "k", "omega", "nut")}
    ph = torch.tensor(np.asarray(phi, dtype=np.float64), requires_grad=True)
    x = x0
    for _ in range(nsteps):
        x = ts.step(x, ph)
    J = sum((x[f] * torch.as_tensor(np.asarray(seed[f], dtype=np.float64))).sum() for f in fields)
    grads = torch.autograd.grad(J, [x0[f] for f in fields] + [ph], allow_unused=True)
    adj = {f: (gr.numpy() if gr is not None else np.zeros_like(np.asarray(state[f], dtype=np.float64)))
           for f, gr in zip(fields, grads[:-1])}
    return adj, grads[-1].numpy(), {f: v.detach().numpy() for f, v in x.items()}
