"""Closed triangle meshes of the layout objects (input data only).

Buildings and trees become closed triangle meshes, the form in which the
paper's design tool hands objects to the simulator (Sec. 3, "Urban model
resolving").  Each generator returns (vertices [n, 3] float64, triangles
[m, 3] int32); the winding is outward, although the even-odd inside test
does not depend on it.  ``meshes_of`` concatenates objects into the flat
arrays of the voxelizer call: vertices, triangles, per-object triangle
offsets and per-object porosity.
"""
import numpy as np


def box_mesh(x, y, z):
    """Axis-aligned box [x0, x1] x [y0, y1] x [z0, z1]: 8 vertices, 12 triangles."""
    v = np.array([[x[a], y[b], z[c]] for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=np.float64)
    # vertex index = 4a + 2b + c
    quads = [(0, 1, 3, 2), (4, 6, 7, 5),      # x0, x1
             (0, 4, 5, 1), (2, 3, 7, 6),      # y0, y1
             (0, 2, 6, 4), (1, 5, 7, 3)]      # z0, z1
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return v, np.array(t, dtype=np.int32)


def prism_mesh(cx, cy, r, z, nsides=16, phase=0.0):
    """Vertical prism over a regular n-gon inscribed in the circle (cx, cy, r),
    z in [z0, z1] (a tree trunk-and-crown cylinder as a mesh): 4n triangles."""
    ang = phase + 2.0 * np.pi * np.arange(nsides) / nsides
    ring = np.stack([cx + r * np.cos(ang), cy + r * np.sin(ang)], axis=1)
    v = np.concatenate([np.column_stack([ring, np.full(nsides, z[0])]),
                        np.column_stack([ring, np.full(nsides, z[1])]),
                        [[cx, cy, z[0]], [cx, cy, z[1]]]])
    n = nsides
    t = []
    for i in range(n):
        j = (i + 1) % n
        t += [(i, j, n + j), (i, n + j, n + i)]       # side
        t += [(2 * n, j, i), (2 * n + 1, n + i, n + j)]  # bottom, top fans
    return v, np.array(t, dtype=np.int32)


def ring_mesh(x, y, hole_x, hole_y, z):
    """A block with a rectangular courtyard (non-convex): outer box
    x * y minus the open shaft hole_x * hole_y, z in [z0, z1]; 32 triangles."""
    xs = [x[0], hole_x[0], hole_x[1], x[1]]
    ys = [y[0], hole_y[0], hole_y[1], y[1]]
    verts, tris = [], []

    def vid(p):
        verts.append(p)
        return len(verts) - 1

    # top and bottom: the 8 cells of the 3 x 3 split of the footprint around
    # the hole, two triangles each
    for zz, up in ((z[0], False), (z[1], True)):
        for a in range(3):
            for b in range(3):
                if a == 1 and b == 1:
                    continue
                p = [vid((xs[a], ys[b], zz)), vid((xs[a + 1], ys[b], zz)),
                     vid((xs[a + 1], ys[b + 1], zz)), vid((xs[a], ys[b + 1], zz))]
                if up:
                    tris += [(p[0], p[1], p[2]), (p[0], p[2], p[3])]
                else:
                    tris += [(p[0], p[2], p[1]), (p[0], p[3], p[2])]
    # walls: outer (facing out) and inner (facing the hole)
    def wall(p0, p1, outward):
        a, b = vid((p0[0], p0[1], z[0])), vid((p1[0], p1[1], z[0]))
        c, d = vid((p1[0], p1[1], z[1])), vid((p0[0], p0[1], z[1]))
        tris.extend([(a, b, c), (a, c, d)] if outward else [(a, c, b), (a, d, c)])
    for (lx, ly, out) in ((x, y, True), (hole_x, hole_y, False)):
        c = [(lx[0], ly[0]), (lx[1], ly[0]), (lx[1], ly[1]), (lx[0], ly[1])]
        for i in range(4):
            wall(c[i], c[(i + 1) % 4], out)
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int32)


def uv_sphere_mesh(c, r, nlat=12, nlon=24):
    """Closed convex polyhedron inscribed in a sphere (latitude-longitude grid)."""
    verts = [(c[0], c[1], c[2] - r)]
    for a in range(1, nlat):
        th = np.pi * a / nlat - np.pi / 2
        for b in range(nlon):
            ph = 2 * np.pi * b / nlon
            verts.append((c[0] + r * np.cos(th) * np.cos(ph), c[1] + r * np.cos(th) * np.sin(ph),
                          c[2] + r * np.sin(th)))
    verts.append((c[0], c[1], c[2] + r))
    top = len(verts) - 1
    ring = lambda a, b: 1 + (a - 1) * nlon + (b % nlon)
    t = []
    for b in range(nlon):
        t.append((0, ring(1, b + 1), ring(1, b)))
        t.append((top, ring(nlat - 1, b), ring(nlat - 1, b + 1)))
    for a in range(1, nlat - 1):
        for b in range(nlon):
            p, q, s, u = ring(a, b), ring(a, b + 1), ring(a + 1, b + 1), ring(a + 1, b)
            t += [(p, q, s), (p, s, u)]
    return np.array(verts, dtype=np.float64), np.array(t, dtype=np.int32)


def meshes_of(objects):
    """Flatten [(vertices, triangles, phi_o), ...] into (vertices [V, 3],
    triangles [T, 3] with global vertex indices, tri_begin [n + 1], phi [n])."""
    vs, ts, begin, phis = [], [], [0], []
    nv = 0
    for v, t, ph in objects:
        vs.append(np.asarray(v, np.float64))
        ts.append(np.asarray(t, np.int32) + nv)
        nv += len(v)
        begin.append(begin[-1] + len(t))
        phis.append(float(ph))
    if not vs:
        return (np.zeros((0, 3)), np.zeros((0, 3), np.int32), np.array([0], np.int32), np.zeros(0))
    return (np.concatenate(vs), np.concatenate(ts).astype(np.int32), np.array(begin, np.int32),
            np.array(phis, np.float64))


def city_meshes(boxes, cylinders, nsides=16):
    """Meshes of a layout's boxes and cylinders (see ``porosity.random_city``)."""
    objs = [box_mesh(b.x, b.y, b.z) + (b.phi,) for b in boxes]
    objs += [prism_mesh(c.cx, c.cy, c.r, c.z, nsides) + (c.phi,) for c in cylinders]
    return meshes_of(objs)
