"""Seeded urban layouts resolved into a per-cell porosity field.

Objects are axis-aligned boxes standing on the ground (buildings) and
vertical cylinders (trees), each with its own object porosity phi_o (0 for a
solid building).  A cell's porosity is the fraction of its volume outside the
objects (appendix, porosity validation: phi = 1 - V_s/V); cut cells are
resolved by uniform sub-division of the cell (Sec. 3, "Urban model
resolving") with ``sub`` sample points per axis.  Where several objects
overlap a cell, the smallest porosity wins:

    phi_cell = min over objects of  1 - f_in * (1 - phi_o)

with f_in the fraction of sub-samples inside the object.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Box:
    x: tuple
    y: tuple
    z: tuple
    phi: float = 0.0


@dataclass
class Cylinder:
    cx: float
    cy: float
    r: float
    z: tuple
    phi: float = 0.5


def _axis_fraction(n, h, lo, hi, sub):
    """Fraction of the ``sub`` sample points of each of ``n`` cells inside [lo, hi)."""
    s = (np.arange(sub) + 0.5) / sub
    pts = (np.arange(n)[:, None] + s[None, :]) * h
    return ((pts >= lo) & (pts < hi)).mean(axis=1)


def _index_range(n, h, lo, hi):
    i0 = max(int(np.floor(lo / h)), 0)
    i1 = min(int(np.ceil(hi / h)), n)
    return i0, i1


def porosity_field(nx, ny, nz, dx, dy, dz, boxes=(), cylinders=(), sub=4):
    """Return phi[nx, ny, nz] (float64, z fastest) for the given objects."""
    phi = np.ones((nx, ny, nz), dtype=np.float64)
    for b in boxes:
        i0, i1 = _index_range(nx, dx, *b.x)
        j0, j1 = _index_range(ny, dy, *b.y)
        k0, k1 = _index_range(nz, dz, *b.z)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        fx = _axis_fraction(nx, dx, *b.x, sub)[i0:i1]
        fy = _axis_fraction(ny, dy, *b.y, sub)[j0:j1]
        fz = _axis_fraction(nz, dz, *b.z, sub)[k0:k1]
        f = fx[:, None, None] * fy[None, :, None] * fz[None, None, :]
        blk = phi[i0:i1, j0:j1, k0:k1]
        np.minimum(blk, 1.0 - f * (1.0 - b.phi), out=blk)
    s = (np.arange(sub) + 0.5) / sub
    for c in cylinders:
        i0, i1 = _index_range(nx, dx, c.cx - c.r, c.cx + c.r)
        j0, j1 = _index_range(ny, dy, c.cy - c.r, c.cy + c.r)
        k0, k1 = _index_range(nz, dz, *c.z)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        xs = ((np.arange(i0, i1)[:, None] + s[None, :]) * dx).reshape(-1)
        ys = ((np.arange(j0, j1)[:, None] + s[None, :]) * dy).reshape(-1)
        inside = ((xs[:, None] - c.cx) ** 2 + (ys[None, :] - c.cy) ** 2) <= c.r ** 2
        fxy = inside.reshape(i1 - i0, sub, j1 - j0, sub).mean(axis=(1, 3))
        fz = _axis_fraction(nz, dz, *c.z, sub)[k0:k1]
        f = fxy[:, :, None] * fz[None, None, :]
        blk = phi[i0:i1, j0:j1, k0:k1]
        np.minimum(blk, 1.0 - f * (1.0 - c.phi), out=blk)
    return phi


def random_city(nx, ny, nz, dx, dy, dz, seed, n_boxes, n_trees,
                footprint=(10.0, 40.0), height=(10.0, 60.0),
                tree_r=(3.0, 6.0), tree_h=(8.0, 15.0), tree_phi=(0.3, 0.7),
                random_direction=False, margin=0.1):
    """Draw a seeded city; returns (boxes, cylinders, wind_dir_deg or None).

    Buildings: footprint width and depth uniform in ``footprint`` metres,
    height uniform in ``height`` capped at 0.8 of the domain height, porosity
    0.  Trees: radius uniform in ``tree_r``, height uniform in ``tree_h``,
    porosity uniform in ``tree_phi``.  Centres are uniform inside the domain
    minus a ``margin`` fraction on each side.  Overlaps are allowed.
    """
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = nx * dx, ny * dy, nz * dz
    wind = float(rng.uniform(0.0, 360.0)) if random_direction else None
    boxes, cyls = [], []
    for _ in range(n_boxes):
        cx = rng.uniform(margin * Lx, (1 - margin) * Lx)
        cy = rng.uniform(margin * Ly, (1 - margin) * Ly)
        w = rng.uniform(*footprint)
        d = rng.uniform(*footprint)
        h = min(rng.uniform(*height), 0.8 * Lz)
        boxes.append(Box((cx - w / 2, cx + w / 2), (cy - d / 2, cy + d / 2), (0.0, h), 0.0))
    for _ in range(n_trees):
        cx = rng.uniform(margin * Lx, (1 - margin) * Lx)
        cy = rng.uniform(margin * Ly, (1 - margin) * Ly)
        r = rng.uniform(*tree_r)
        h = min(rng.uniform(*tree_h), 0.8 * Lz)
        ph = rng.uniform(*tree_phi)
        cyls.append(Cylinder(cx, cy, r, (0.0, h), ph))
    return boxes, cyls, wind


def preset_porosity(p, case=None):
    """Return (phi, config) for preset dictionary ``p`` (see ``configs.preset``).

    For the batched preset pass ``case`` (an index) to get one case's grid,
    porosity and wind direction.  The returned config is a copy with the
    grid shape and wind direction filled in.
    """
    cfg = dict(p["config"])
    lay = p["layout"]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    dx, dy, dz = cfg["dx"], cfg["dy"], cfg["dz"]
    if lay["kind"] == "objects":
        boxes = [Box(b["x"], b["y"], b["z"], b["phi"]) for b in lay["boxes"]]
        cyls = [Cylinder(c["cx"], c["cy"], c["r"], c["z"], c["phi"]) for c in lay["cylinders"]]
        return porosity_field(nx, ny, nz, dx, dy, dz, boxes, cyls), cfg
    if lay["kind"] == "random":
        boxes, cyls, wind = random_city(
            nx, ny, nz, dx, dy, dz, lay["seed"], lay["n_boxes"], lay["n_trees"],
            height=lay.get("height", (10.0, 60.0)),
            random_direction=lay.get("random_direction", False))
        if wind is not None:
            cfg["wind_dir_deg"] = wind
        return porosity_field(nx, ny, nz, dx, dy, dz, boxes, cyls), cfg
    if lay["kind"] == "batched":
        if case is None:
            raise ValueError("batched preset needs a case index")
        c = lay["cases"][case]
        rng = np.random.default_rng(c["seed"])
        nx, ny, nz = c["shapes"][int(rng.integers(len(c["shapes"])))]
        nb = int(rng.integers(lay["n_range"][0], lay["n_range"][1] + 1))
        nt = int(rng.integers(lay["n_range"][0], lay["n_range"][1] + 1))
        cfg.update(nx=nx, ny=ny, nz=nz, wind_dir_deg=c["direction"])
        boxes, cyls, _ = random_city(nx, ny, nz, dx, dy, dz, int(rng.integers(1 << 30)), nb, nt)
        return porosity_field(nx, ny, nz, dx, dy, dz, boxes, cyls), cfg
    raise ValueError("unknown layout kind %r" % lay["kind"])
