"""Pressure Poisson operator, its solution and the AI preconditioner (oracle).

The projection solves A p = b with A = -L_h, the 7-point negative Laplacian
on cell centres, and b = -(rho/dt) div u*.  Because obstacles enter only
through the porosity drag, A depends on the grid and the boundary kinds
alone and is built once (Sec. 3, "Porosity Model vs. Solid-wall Boundary
Conditions").  Boundary rows: a Neumann side (inlet, wall, slip) drops the
neighbour; an outlet side keeps it with ghost pressure zero.  Unknowns are
ordered z fastest: index (i ny + j) nz + k.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bc import OUTLET


def poisson_matrix(g):
    """Sparse CSR matrix A (float64)."""
    nx, ny, nz = g.n
    N = nx * ny * nz
    idx = np.arange(N).reshape(nx, ny, nz)
    diag = np.zeros((nx, ny, nz))
    rows, cols, vals = [], [], []
    for ax in range(3):
        w = 1.0 / g.h[ax] ** 2
        n = g.n[ax]
        for end, step in ((0, -1), (1, 1)):
            side = 2 * ax + end
            # cells having a neighbour inside the domain in this direction
            inner = [slice(None)] * 3
            nbr = [slice(None)] * 3
            if step < 0:
                inner[ax] = slice(1, n)
                nbr[ax] = slice(0, n - 1)
            else:
                inner[ax] = slice(0, n - 1)
                nbr[ax] = slice(1, n)
            diag[tuple(inner)] += w
            rows.append(idx[tuple(inner)].ravel())
            cols.append(idx[tuple(nbr)].ravel())
            vals.append(np.full(rows[-1].size, -w))
            # boundary cells: an outlet ghost (p = 0) still couples
            if g.bc[side] == OUTLET:
                bnd = [slice(None)] * 3
                bnd[ax] = 0 if step < 0 else n - 1
                diag[tuple(bnd)] += w
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sum_duplicates()
    return A


def ai_preconditioner(A, omega, order=1):
    """Approximate-inverse preconditioner M^-1 = K^T K (Sec. 3, "Approximate
    Inverse Preconditioner") with

        K = sqrt(2 - omega) Dbar^(-1/2) (I - L Dbar^-1 [+ (L Dbar^-1)^2])

    Dbar = D / omega, D and L the diagonal and strictly lower part of A.
    The full product K^T K is kept (no truncation to the pattern of A): the
    truncated first-order form is indefinite for omega above about 1.1 in
    3-D, while K^T K is positive definite for any 0 < omega < 2."""
    d = A.diagonal()
    Dbar_inv = sp.diags(omega / d)
    Dbar_mhalf = sp.diags(np.sqrt(omega / d))
    L = sp.tril(A, k=-1)
    LD = L @ Dbar_inv
    I = sp.identity(A.shape[0], format="csr")
    inner = I - LD
    if order == 2:
        inner = inner + LD @ LD
    K = math.sqrt(2.0 - omega) * (Dbar_mhalf @ inner)
    return (K.T @ K).tocsr(), K.tocsr()


class PressureSolver:
    """Solves A p = b.  ``method`` 'direct' factors A once (sparse LU);
    'cg' runs preconditioned CG from the warm start to ||r|| <= tol ||b||;
    'none' only builds A (for checks that never solve)."""

    def __init__(self, g, method="auto", tol=1e-12, maxit=20000, precond="ai1", ai_omega=1.6):
        self.A = poisson_matrix(g)
        N = self.A.shape[0]
        if method == "auto":
            method = "direct" if N <= 150_000 else "cg"
        self.method = method
        self.tol, self.maxit = tol, maxit
        self.M = None
        if method == "direct":
            self.lu = spla.splu(self.A.tocsc())
        elif method == "none":
            pass
        elif precond == "ai1":
            self.M, _ = ai_preconditioner(self.A, ai_omega)

    def solve(self, b, x0):
        if self.method == "none":
            raise RuntimeError("this oracle grid was built without a pressure solver")
        if self.method == "direct":
            x = self.lu.solve(b)
            return x, 0
        return pcg(self.A, b, x0, self.M, self.tol, self.maxit)


def pcg(A, b, x0, M=None, tol=1e-12, maxit=20000, criterion=0):
    """Preconditioned conjugate gradients (Saad, Alg. 9.1) from x0.

    criterion 0 stops at ||r||_2 <= tol ||b||_2; criterion 1 is the paper's
    test (M^-1 r . r) / ||b||^2 < tol (appendix, "Efficiency of the AI
    Preconditioner").  Returns (x, iterations)."""
    x = x0.copy()
    r = b - A @ x
    bb = float(b @ b)
    z = M @ r if M is not None else r.copy()
    rz = float(r @ z)

    def done(rr, rz_):
        if criterion == 0:
            return rr <= tol * tol * bb
        return rz_ < tol * bb

    if done(float(r @ r), rz):
        return x, 0
    d = z.copy()
    for it in range(1, maxit + 1):
        q = A @ d
        alpha = rz / float(d @ q)
        x += alpha * d
        r -= alpha * q
        z = M @ r if M is not None else r.copy()
        rz_new = float(r @ z)
        if done(float(r @ r), rz_new):
            return x, it
        d = z + (rz_new / rz) * d
        rz = rz_new
    return x, maxit
