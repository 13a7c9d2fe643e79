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


def axis_operator(g, ax):
    """The 1-D factor of A along axis ``ax``: (1/h^2) tridiag(-1, d, -1) over
    the n cells of that axis, where d counts the neighbours inside the axis
    plus an outlet ghost at an end whose side is an outlet (a Neumann end
    drops its neighbour).  A is the Kronecker sum of the three factors
    (z fastest): A = T_x (x) I (x) I + I (x) T_y (x) I + I (x) I (x) T_z,
    because each axis adds its own terms to a row and its diagonal depends
    only on the position along that axis."""
    n, w = g.n[ax], 1.0 / g.h[ax] ** 2
    T = np.zeros((n, n))
    for i in range(n):
        d = 0.0
        for nb, side in ((i - 1, 2 * ax), (i + 1, 2 * ax + 1)):
            if 0 <= nb < n:
                T[i, nb] = -w
                d += w
            elif g.bc[side] == OUTLET:
                d += w
        T[i, i] = d
    return T


class FastDiagonalSolver:
    """Exact solve of A p = b by diagonalising the separable operator
    (Lynch, Rice and Thomas's fast diagonalisation): with T_a = V_a diag(l_a)
    V_a^T (symmetric eigendecomposition of each 1-D factor),

        p = (V_x (x) V_y (x) V_z) [ (V_x (x) V_y (x) V_z)^T b / (l_x + l_y + l_z) ].

    The transforms are three dense products along the axes, O(N (nx+ny+nz))
    flops; the denominators are positive because at least one side is an
    outlet (that axis's factor is positive definite, the others semidefinite).
    A direct solve to rounding for grids too large for sparse LU."""

    def __init__(self, g):
        self.n = g.n
        self.V, lam = [], []
        for ax in range(3):
            l_a, V_a = np.linalg.eigh(axis_operator(g, ax))
            self.V.append(V_a)
            lam.append(l_a)
        self.den = lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :]
        if not np.all(self.den > 0):
            raise ValueError("singular pressure operator (no outlet side)")

    def _transform(self, x, transpose):
        for ax in range(3):
            V = self.V[ax].T if transpose else self.V[ax]
            x = np.moveaxis(np.tensordot(V, x, axes=([1], [ax])), 0, ax)
        return x

    def solve(self, b):
        bt = self._transform(np.asarray(b, dtype=np.float64).reshape(self.n), transpose=True)
        return self._transform(bt / self.den, transpose=False).ravel()


class PressureSolver:
    """Solves A p = b.  ``method`` 'direct' factors A once (sparse LU);
    'fastdiag' diagonalises the separable A (exact, for large grids); 'cg'
    runs preconditioned CG from the warm start to ||r|| <= tol ||b||; 'none'
    only builds A (for checks that never solve).  'auto' takes 'direct' up to
    150,000 cells and 'fastdiag' above."""

    def __init__(self, g, method="auto", tol=1e-12, maxit=20000, precond="ai1", ai_omega=1.6):
        self.g = g
        self._A = None
        N = g.ncell
        if method == "auto":
            method = "direct" if N <= 150_000 else "fastdiag"
        self.method = method
        self.tol, self.maxit = tol, maxit
        self.M = None
        if method == "direct":
            self.lu = spla.splu(self.A.tocsc())
        elif method == "fastdiag":
            self.fd = FastDiagonalSolver(g)
        elif method == "none":
            pass
        elif precond == "ai1":
            self.M, _ = ai_preconditioner(self.A, ai_omega)

    @property
    def A(self):
        """The sparse matrix, built on first use."""
        if self._A is None:
            self._A = poisson_matrix(self.g)
        return self._A

    def solve(self, b, x0):
        if self.method == "none":
            raise RuntimeError("this oracle grid was built without a pressure solver")
        if self.method == "direct":
            x = self.lu.solve(b)
            return x, 0
        if self.method == "fastdiag":
            return self.fd.solve(b), 0
        return pcg(self.A, b, x0, self.M, self.tol, self.maxit)


def pcg(A, b, x0, M=None, tol=1e-12, maxit=20000, criterion=0):
    """Preconditioned conjugate gradients (Saad, Alg. 9.1) from x0.

    criterion 0 stops at ||r||_2 <= tol ||b||_2; criterion 1 is the paper's
    test (M^-1 r . r) / ||b||^2 < tol (appendix, "Efficiency of the AI
    Preconditioner").  An initial guess whose residual is longer than b
    (a worse start than zero) is replaced by zero.  Returns (x, iterations)."""
    x = x0.copy()
    r = b - A @ x
    bb = float(b @ b)
    if float(r @ r) > bb:
        x = np.zeros_like(x)
        r = b.copy()
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
