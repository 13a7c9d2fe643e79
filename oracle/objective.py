"""Design objective of the optimisation routine -- TEST INFRASTRUCTURE ONLY.

Sec. 4 (the Nurnberg study) scores a design by the mean wind speed over N
target regions: L = sum_i (s_i - u_t)^2, where s_i averages the wind speed
over region i and u_t is the ideal speed (0.55 m/s there).  The speed of a
cell is the norm of its cell-centre velocity, each component the mean of the
cell's two faces on the staggered grid (Sec. 3.1).  Regions are boxes of
cell indices, half-open on each axis.

A second objective scores pedestrian comfort on a horizontal plane (see
``plane_objective``), and ``field_objective`` is the general form that
compares the flow with a desired one region by region.

Pinned by tests/test_oracle_objective.py (uniform-flow closed forms, linear
profiles with known means and plane values, brute force on a tiny grid).
"""
import numpy as np


def cell_speed(u, v, w):
    """Cell-centre speed |(u_c, v_c, w_c)| from face arrays of extents
    (nx+1, ny, nz), (nx, ny+1, nz), (nx, ny, nz+1)."""
    uc = 0.5 * (u[:-1, :, :] + u[1:, :, :])
    vc = 0.5 * (v[:, :-1, :] + v[:, 1:, :])
    wc = 0.5 * (w[:, :, :-1] + w[:, :, 1:])
    return np.sqrt(uc * uc + vc * vc + wc * wc)


def region_means(u, v, w, regions):
    """Mean cell speed over each box ((i0, i1), (j0, j1), (k0, k1))."""
    s = cell_speed(np.asarray(u, np.float64), np.asarray(v, np.float64), np.asarray(w, np.float64))
    out = []
    for (i0, i1), (j0, j1), (k0, k1) in regions:
        out.append(float(np.mean(s[i0:i1, j0:j1, k0:k1])))
    return np.array(out)


def region_objective(u, v, w, regions, u_target):
    """L = sum over regions of (mean speed - u_target)^2."""
    m = region_means(u, v, w, regions)
    return float(np.sum((m - u_target) ** 2))


def field_objective(u, v, w, u_target, regions):
    """The general form of Sec. 4: sum over regions of the Euclidean norm of
    F_i(u) - F_i(u_t), F_i being the cell-centre velocities (all three
    components) of the cells of region i; u_target is [3, nx, ny, nz]."""
    u, v, w = (np.asarray(a, np.float64) for a in (u, v, w))
    cc = np.stack([0.5 * (u[:-1, :, :] + u[1:, :, :]), 0.5 * (v[:, :-1, :] + v[:, 1:, :]),
                   0.5 * (w[:, :, :-1] + w[:, :, 1:])])
    d = cc - np.asarray(u_target, np.float64)
    total = 0.0
    for (i0, i1), (j0, j1), (k0, k1) in regions:
        total += float(np.sqrt(np.sum(d[:, i0:i1, j0:j1, k0:k1] ** 2)))
    return total


def plane_objective(u, v, w, phi, h, z_plane, s_target=2.0, s_min=0.3, w_penalty=10.0):
    """Pedestrian comfort on the plane z = z_plane: the cell-centre velocity
    and the porosity interpolated linearly in z between the two cell centres
    around the plane, s = sqrt(|u|^2 + 1e-12), and
    dx dy sum over columns of phi [(s - s_target)^2 + w_penalty max(0, s_min - s)^2]."""
    u, v, w, phi = (np.asarray(a, np.float64) for a in (u, v, w, phi))
    nz = phi.shape[2]
    zc = z_plane / h[2] - 0.5
    k0 = min(max(int(np.floor(zc)), 0), nz - 2)
    t = zc - k0
    uc = 0.5 * (u[:-1, :, :] + u[1:, :, :])
    vc = 0.5 * (v[:, :-1, :] + v[:, 1:, :])
    wc = 0.5 * (w[:, :, :-1] + w[:, :, 1:])
    lerp = lambda a: (1.0 - t) * a[:, :, k0] + t * a[:, :, k0 + 1]
    up, vp, wp, pp = lerp(uc), lerp(vc), lerp(wc), lerp(phi)
    s = np.sqrt(up * up + vp * vp + wp * wp + 1e-12)
    lo = np.maximum(0.0, s_min - s)
    return float(np.sum(pp * ((s - s_target) ** 2 + w_penalty * lo * lo)) * h[0] * h[1])


def fd_gradient(J, theta, eps):
    """Forward-difference gradient of J at theta (Sec. 4: one extra
    simulation per parameter, step eps)."""
    theta = np.asarray(theta, np.float64)
    j0 = J(theta)
    g = np.zeros_like(theta)
    for n in range(theta.size):
        t = theta.copy()
        t[n] += eps
        g[n] = (J(t) - j0) / eps
    return j0, g
