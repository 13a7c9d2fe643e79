"""Pins of the oracle's smoothed object indicator (closed forms and limits)."""
import math

import numpy as np

from oracle.smooth import smooth_porosity, sig

N, H = (20, 16, 12), (2.0, 2.0, 2.0)


def test_deep_inside_and_far_outside():
    box = (10.0, 30.0, 8.0, 24.0, 0.0, 16.0, 0.0)
    phi = smooth_porosity(N, H, [box], [], 0.05)
    # a cell centre 1 m inside every face: the steps are 1 - sig(-20) each
    assert abs(phi[7, 7, 3]) < 1e-7
    # 5 m outside: sig(-100)
    assert phi[2, 7, 3] == 1.0 or phi[2, 7, 3] > 1 - 1e-40
    tree = (20.0, 16.0, 6.0, 0.0, 12.0, 0.4)
    phi = smooth_porosity(N, H, [], [tree], 0.05)
    assert abs(phi[9, 7, 2] - 0.4) < 1e-12


def test_half_value_on_a_face_and_ground_rule():
    # the face x = 11 passes through the centre of cell 5 (11 = 5.5 * 2)
    box = (11.0, 31.0, -100.0, 100.0, 0.0, 100.0, 0.0)
    s = 0.7
    phi = smooth_porosity(N, H, [box], [], s)
    # cell (5, 3, 0): centre (11, 7, 1); y steps at -100 and 100, top at 100
    ref = 1.0 - 0.5 * sig(20.0 / s) * sig(107 / s) * sig(93 / s) * sig(99 / s)
    assert math.isclose(phi[5, 3, 0], ref, rel_tol=1e-12)
    # standing on the ground: the first layer is as solid as the second
    assert phi[10, 3, 0] == phi[10, 3, 1]
    # a lifted box has a lower step at z0
    lifted = (11.0, 31.0, -100.0, 100.0, 5.0, 100.0, 0.0)
    phi2 = smooth_porosity(N, H, [lifted], [], s)
    ref = 1.0 - 0.5 * sig(95 / s) * sig(10 / s) ** 2 * sig(107 / s) * sig(93 / s)
    assert math.isclose(phi2[10, 3, 2], ref, rel_tol=1e-12)


def test_symmetry_and_monotone_height():
    box = (12.0, 28.0, 10.0, 22.0, 0.0, 9.3, 0.0)
    phi = smooth_porosity(N, H, [box], [], 1.0)
    assert np.allclose(phi, phi[::-1, :, :])      # symmetric about x = 20
    assert np.allclose(phi, phi[:, ::-1, :])      # and y = 16
    taller = smooth_porosity(N, H, [box[:5] + (10.3, 0.0)], [], 1.0)
    assert (taller <= phi + 1e-15).all() and (taller < phi - 1e-6).any()


def test_sharp_limit_is_the_cell_centre_box():
    box = (7.3, 29.1, 5.2, 21.7, 0.0, 13.1, 0.25)
    phi = smooth_porosity(N, H, [box], [], 1e-4)
    c = [(np.arange(N[a]) + 0.5) * H[a] for a in range(3)]
    inside = ((c[0][:, None, None] > 7.3) & (c[0][:, None, None] < 29.1) & (c[1][None, :, None] > 5.2) &
              (c[1][None, :, None] < 21.7) & (c[2][None, None, :] < 13.1))
    assert np.allclose(phi, np.where(inside, 0.25, 1.0), atol=1e-12)
