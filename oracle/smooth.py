"""Smoothed object indicator for design optimisation -- TEST INFRASTRUCTURE ONLY.

Moving a building by a fraction of a cell must change the porosity
continuously for a gradient to exist (Sec. 3, the cut-cell volume ratio
lets the boundary slide within a cell).  Here each object's indicator is a
product of logistic steps of width s across its faces, evaluated at cell
centres:

    box:       I(p) = prod over axes  sig((p_a - lo_a)/s) sig((hi_a - p_a)/s)
    cylinder:  I(p) = sig((R - rho)/s) sig((z - z0)/s) sig((z1 - z)/s)

with sig(t) = 1 / (1 + exp(-t)) and rho the distance from the axis; an
object standing on the ground (z0 <= 0) has no lower step.  A cell's
porosity is min(1, min over objects of 1 - I (1 - phi_o)).

Pinned by tests/test_oracle_smooth.py (limits far inside and outside, the
half value on a face, the ground rule, symmetry, the sharp-step limit
against the box porosity at cell centres).
"""
import numpy as np


def sig(t):
    """Logistic function, evaluated without overflow on either side."""
    t = np.asarray(t, np.float64)
    e = np.exp(-np.abs(t))
    return np.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def cell_centres(n, h):
    return [(np.arange(n[a]) + 0.5) * h[a] for a in range(3)]


def box_indicator(n, h, box, s):
    x0, x1, y0, y1, z0, z1 = box[:6]
    cx, cy, cz = cell_centres(n, h)
    fx = sig((cx - x0) / s) * sig((x1 - cx) / s)
    fy = sig((cy - y0) / s) * sig((y1 - cy) / s)
    fz = sig((z1 - cz) / s) * (sig((cz - z0) / s) if z0 > 0 else 1.0)
    return fx[:, None, None] * fy[None, :, None] * fz[None, None, :]


def cylinder_indicator(n, h, cyl, s):
    xc, yc, r, z0, z1 = cyl[:5]
    cx, cy, cz = cell_centres(n, h)
    rho = np.sqrt((cx[:, None] - xc) ** 2 + (cy[None, :] - yc) ** 2)
    fr = sig((r - rho) / s)
    fz = sig((z1 - cz) / s) * (sig((cz - z0) / s) if z0 > 0 else 1.0)
    return fr[:, :, None] * fz[None, None, :]


def smooth_porosity(n, h, boxes, cylinders, s):
    """boxes: rows (x0, x1, y0, y1, z0, z1, phi); cylinders: rows
    (cx, cy, R, z0, z1, phi); float64 porosity [nx, ny, nz]."""
    phi = np.ones(n)
    for b in boxes:
        np.minimum(phi, 1.0 - box_indicator(n, h, b, s) * (1.0 - b[6]), out=phi)
    for c in cylinders:
        np.minimum(phi, 1.0 - cylinder_indicator(n, h, c, s) * (1.0 - c[5]), out=phi)
    return phi
