"""Pins of the oracle's design objective (Sec. 4, target-region objective)
and of its forward-difference gradient, against closed forms and brute force."""
import math

import numpy as np

from oracle import cell_speed, region_means, region_objective, plane_objective, field_objective, fd_gradient


def faces(nx, ny, nz, u=0.0, v=0.0, w=0.0):
    return (np.full((nx + 1, ny, nz), u), np.full((nx, ny + 1, nz), v), np.full((nx, ny, nz + 1), w))


def test_uniform_flow_closed_form():
    # every cell moves at |(3, 4, 0)| = 5, so each region mean is 5
    u, v, w = faces(6, 5, 4, u=3.0, v=4.0)
    regions = [((0, 6), (0, 5), (0, 4)), ((1, 3), (2, 4), (1, 2)), ((5, 6), (4, 5), (3, 4))]
    assert np.allclose(region_means(u, v, w, regions), 5.0, rtol=0, atol=1e-15)
    assert math.isclose(region_objective(u, v, w, regions, 0.55), 3 * (5.0 - 0.55) ** 2, rel_tol=1e-15)
    # the target itself scores zero
    assert region_objective(u, v, w, regions, 5.0) == 0.0


def test_linear_profiles_have_known_region_means():
    # face value a*i on the i-th x face: cell i holds a*(i + 1/2), so the mean
    # over cells i0..i1-1 is a*(i0 + i1)/2; likewise for w along k
    nx, ny, nz, a = 9, 4, 7, 0.25
    u, v, w = faces(nx, ny, nz)
    u[...] = a * np.arange(nx + 1)[:, None, None]
    m = region_means(u, v, w, [((2, 7), (0, 4), (0, 7)), ((0, 1), (1, 2), (3, 5))])
    assert np.allclose(m, [a * (2 + 7) / 2, a * 0.5], rtol=1e-15)
    u[...] = 0.0
    w[...] = -a * np.arange(nz + 1)[None, None, :]      # speed ignores the sign
    m = region_means(u, v, w, [((0, 9), (0, 4), (3, 6))])
    assert np.allclose(m, [a * (3 + 6) / 2], rtol=1e-15)


def test_axes_are_not_exchanged():
    # a y-face profile that grows along j leaves the x extent irrelevant
    nx, ny, nz = 5, 8, 3
    u, v, w = faces(nx, ny, nz)
    v[...] = np.arange(ny + 1)[None, :, None].astype(float)
    s = cell_speed(u, v, w)
    assert s.shape == (nx, ny, nz)
    assert np.allclose(s, (np.arange(ny) + 0.5)[None, :, None])


def test_brute_force_on_tiny_random_state():
    rng = np.random.default_rng(7)
    nx, ny, nz = 4, 3, 5
    u = rng.normal(size=(nx + 1, ny, nz))
    v = rng.normal(size=(nx, ny + 1, nz))
    w = rng.normal(size=(nx, ny, nz + 1))
    regions = [((0, 4), (0, 3), (0, 5)), ((1, 2), (0, 2), (2, 5)), ((3, 4), (2, 3), (4, 5))]
    J = 0.0
    for (i0, i1), (j0, j1), (k0, k1) in regions:
        tot, cnt = 0.0, 0
        for i in range(i0, i1):
            for j in range(j0, j1):
                for k in range(k0, k1):
                    cu = (u[i, j, k] + u[i + 1, j, k]) / 2
                    cv = (v[i, j, k] + v[i, j + 1, k]) / 2
                    cw = (w[i, j, k] + w[i, j, k + 1]) / 2
                    tot += math.sqrt(cu * cu + cv * cv + cw * cw)
                    cnt += 1
        J += (tot / cnt - 0.55) ** 2
    assert math.isclose(region_objective(u, v, w, regions, 0.55), J, rel_tol=1e-13)


def test_forward_difference_of_a_quadratic_is_exact_closed_form():
    # J = sum c_n (t_n - s_n)^2: (J(t + e e_n) - J(t))/e = 2 c_n (t_n - s_n) + c_n e
    c = np.array([1.0, 2.5, 0.5])
    s = np.array([0.3, -1.0, 2.0])
    J = lambda t: float(np.sum(c * (t - s) ** 2))
    t = np.array([1.0, 0.5, -0.25])
    j0, g = fd_gradient(J, t, 0.1)
    assert j0 == J(t)
    assert np.allclose(g, 2 * c * (t - s) + c * 0.1, rtol=1e-12)


def test_plane_objective_uniform_flow_closed_form():
    nx, ny, nz, h = 7, 5, 6, (2.0, 3.0, 2.0)
    for U, ph in ((3.5, 1.0), (0.1, 1.0), (3.5, 0.5)):
        u, v, w = faces(nx, ny, nz, u=U)
        phi = np.full((nx, ny, nz), ph)
        s = math.sqrt(U * U + 1e-12)
        ref = nx * ny * h[0] * h[1] * ph * ((s - 2.0) ** 2 + 10.0 * max(0.0, 0.3 - s) ** 2)
        assert math.isclose(plane_objective(u, v, w, phi, h, 1.5), ref, rel_tol=1e-14)


def test_plane_objective_interpolates_linear_profiles_exactly():
    # u faces sit at the cell-centre heights (k + 1/2) dz: a profile a z gives
    # a z_plane at the plane; the porosity is linear in z as well
    nx, ny, nz, h, a = 4, 3, 8, (1.0, 1.0, 2.0), 0.7
    zc = (np.arange(nz) + 0.5) * h[2]
    u, v, w = faces(nx, ny, nz)
    u[...] = a * zc[None, None, :]
    phi = np.broadcast_to(0.05 * zc[None, None, :], (nx, ny, nz)).copy()
    for zp in (1.0, 1.5, 4.2, 14.9, 15.0):
        s = math.sqrt((a * zp) ** 2 + 1e-12)
        ref = nx * ny * h[0] * h[1] * 0.05 * zp * ((s - 2.0) ** 2 + 10.0 * max(0.0, 0.3 - s) ** 2)
        assert math.isclose(plane_objective(u, v, w, phi, h, zp), ref, rel_tol=1e-12), zp


def test_plane_objective_brute_force():
    rng = np.random.default_rng(11)
    nx, ny, nz, h = 3, 4, 5, (1.5, 2.0, 1.2)
    u = rng.normal(size=(nx + 1, ny, nz))
    v = rng.normal(size=(nx, ny + 1, nz)) * 0.2
    w = rng.normal(size=(nx, ny, nz + 1)) * 0.2
    phi = rng.uniform(0, 1, size=(nx, ny, nz))
    zp = 2.3   # between the centres of k = 1 (1.8) and k = 2 (3.0)
    t = (zp - 1.8) / 1.2
    J = 0.0
    for i in range(nx):
        for j in range(ny):
            vec = []
            for k in (1, 2):
                vec.append(((u[i, j, k] + u[i + 1, j, k]) / 2, (v[i, j, k] + v[i, j + 1, k]) / 2,
                            (w[i, j, k] + w[i, j, k + 1]) / 2))
            p = [(1 - t) * vec[0][c] + t * vec[1][c] for c in range(3)]
            s = math.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2 + 1e-12)
            f = (1 - t) * phi[i, j, 1] + t * phi[i, j, 2]
            J += f * ((s - 2.0) ** 2 + 10.0 * max(0.0, 0.3 - s) ** 2) * h[0] * h[1]
    assert math.isclose(plane_objective(u, v, w, phi, h, zp), J, rel_tol=1e-12)


def test_field_objective_closed_forms():
    nx, ny, nz = 6, 5, 4
    rng = np.random.default_rng(2)
    u = rng.normal(size=(nx + 1, ny, nz))
    v = rng.normal(size=(nx, ny + 1, nz))
    w = rng.normal(size=(nx, ny, nz + 1))
    cc = np.stack([(u[:-1] + u[1:]) / 2, (v[:, :-1] + v[:, 1:]) / 2, (w[:, :, :-1] + w[:, :, 1:]) / 2])
    regions = [((0, 6), (0, 5), (0, 4)), ((1, 3), (2, 5), (1, 2)), ((5, 6), (4, 5), (3, 4))]
    # the desired flow itself scores 0
    assert field_objective(u, v, w, cc, regions) == 0.0
    # a uniform offset delta: each region contributes sqrt(cells) |delta|
    delta = np.array([0.3, -1.2, 0.4])
    ref = sum(math.sqrt((b[0][1] - b[0][0]) * (b[1][1] - b[1][0]) * (b[2][1] - b[2][0])) for b in regions)
    got = field_objective(u, v, w, cc - delta[:, None, None, None], regions)
    assert math.isclose(got, ref * 1.3, rel_tol=1e-13)   # |delta| = 1.3


def test_field_objective_brute_force():
    nx, ny, nz = 3, 4, 2
    rng = np.random.default_rng(5)
    u = rng.normal(size=(nx + 1, ny, nz))
    v = rng.normal(size=(nx, ny + 1, nz))
    w = rng.normal(size=(nx, ny, nz + 1))
    ut = rng.normal(size=(3, nx, ny, nz))
    regions = [((0, 2), (1, 4), (0, 2)), ((2, 3), (0, 1), (1, 2))]
    J = 0.0
    for (i0, i1), (j0, j1), (k0, k1) in regions:
        ss = 0.0
        for i in range(i0, i1):
            for j in range(j0, j1):
                for k in range(k0, k1):
                    c = ((u[i, j, k] + u[i + 1, j, k]) / 2, (v[i, j, k] + v[i, j + 1, k]) / 2,
                         (w[i, j, k] + w[i, j, k + 1]) / 2)
                    ss += sum((c[q] - ut[q, i, j, k]) ** 2 for q in range(3))
        J += math.sqrt(ss)
    assert math.isclose(field_objective(u, v, w, ut, regions), J, rel_tol=1e-13)
