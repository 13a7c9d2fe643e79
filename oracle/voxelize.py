"""Cell porosity of triangle-mesh objects -- TEST INFRASTRUCTURE ONLY.

Sec. 3 ("Urban model resolving"): each object's surface is a closed triangle
mesh.  A first pass takes the object's axis-aligned bounding box; a second
pass decides for the points near it whether they lie inside by casting a
ray and counting surface crossings (odd = inside), each crossing found with
the Moller-Trumbore ray/triangle test.  Cut cells are resolved by uniform
sub-division: the porosity of a cell is the fraction of its sub-sample
points outside the object (phi = 1 - V_s/V).

Readings: the sample points of cell (i, j, k) are ((i + (s + 1/2)/sub) dx,
(j + ...) dy, (k + ...) dz) for s = 0..sub-1 per axis; the ray runs along
+x; a triangle parallel to the ray (zero determinant) is not crossed; the
bounding box selects every cell it overlaps (a cell whose centre lies
outside the box can still have samples inside the object); an object with
its own porosity phi_o (a tree) gives 1 - f_in (1 - phi_o), and overlapping
objects take the smallest value.

Pinned by tests/test_oracle_voxelize.py (box, prism, courtyard block and
sphere against closed forms; order and winding invariance; the bounding-box
pass against brute force over every cell).
"""
import numpy as np


def ray_crossings(points, verts, tris):
    """Number of triangles hit by the rays from each point along +x
    (Moller-Trumbore with direction (1, 0, 0); hits at t > 0)."""
    p = np.asarray(points, np.float64)
    v0 = verts[tris[:, 0]]
    e1 = verts[tris[:, 1]] - v0
    e2 = verts[tris[:, 2]] - v0
    # P = D x E2 with D = (1, 0, 0): (0, -e2z, e2y); det = E1 . P; the
    # published algorithm scales by the reciprocal of det
    det = -e1[:, 1] * e2[:, 2] + e1[:, 2] * e2[:, 1]
    ok = det != 0.0
    v0, e1, e2, det = v0[ok], e1[ok], e2[ok], det[ok]
    inv = 1.0 / det
    count = np.zeros(len(p), dtype=np.int64)
    for n in range(len(det)):
        T = p - v0[n]
        u = (-T[:, 1] * e2[n, 2] + T[:, 2] * e2[n, 1]) * inv[n]
        # Q = T x E1; v = D . Q; t = E2 . Q
        qx = T[:, 1] * e1[n, 2] - T[:, 2] * e1[n, 1]
        qy = T[:, 2] * e1[n, 0] - T[:, 0] * e1[n, 2]
        qz = T[:, 0] * e1[n, 1] - T[:, 1] * e1[n, 0]
        v = qx * inv[n]
        t = (e2[n, 0] * qx + e2[n, 1] * qy + e2[n, 2] * qz) * inv[n]
        hit = (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t > 0.0)
        count += hit
    return count


def inside(points, verts, tris):
    """Even-odd rule: a point is inside when its ray crosses the surface an
    odd number of times."""
    return (ray_crossings(points, verts, tris) % 2) == 1


def sample_offsets(sub):
    return (np.arange(sub) + 0.5) / sub


def cell_ranges(n, h, aabb):
    """Cells of each axis that the bounding box overlaps (first pass)."""
    out = []
    for a in range(3):
        lo, hi = aabb[0][a], aabb[1][a]
        i0 = max(int(np.floor(lo / h[a])), 0)
        i1 = min(int(np.ceil(hi / h[a])), n[a])
        out.append((i0, max(i0, i1)))
    return out


def object_inside_fraction(n, h, verts, tris, sub, use_aabb=True):
    """f_in per cell (float64 array of shape n): the fraction of each cell's
    sub^3 sample points inside the object."""
    f = np.zeros(n)
    if len(tris) == 0:
        return f
    used = verts[np.unique(tris)]
    aabb = (used.min(axis=0), used.max(axis=0))
    rng = cell_ranges(n, h, aabb) if use_aabb else [(0, n[0]), (0, n[1]), (0, n[2])]
    if any(a >= b for a, b in rng):
        return f
    s = sample_offsets(sub)
    axes = [((np.arange(a, b)[:, None] + s[None, :]) * h[ax]).reshape(-1) for ax, (a, b) in enumerate(rng)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    ins = inside(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1), verts, tris)
    m = [b - a for a, b in rng]
    ins = ins.reshape(m[0], sub, m[1], sub, m[2], sub)
    (i0, i1), (j0, j1), (k0, k1) = rng
    f[i0:i1, j0:j1, k0:k1] = ins.mean(axis=(1, 3, 5))
    return f


def voxelize(n, h, verts, tris, tri_begin, phi_obj, sub, use_aabb=True):
    """Cell porosity [nx, ny, nz] (float64) of the objects: per object
    1 - f_in (1 - phi_o), combined by the minimum; 1 where no object is."""
    phi = np.ones(n)
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    for o in range(len(phi_obj)):
        t = tris[tri_begin[o]:tri_begin[o + 1]]
        f = object_inside_fraction(n, h, verts, t, sub, use_aabb)
        cand = 1.0 - f * (1.0 - phi_obj[o])
        np.minimum(phi, np.where(f > 0, cand, 1.0), out=phi)
    return phi


def sampled_cells(n, h, verts, tris, tri_begin, phi_obj, sub, cells):
    """The porosity of a few cells only (a list of (i, j, k)), for checks at
    sizes where the full field is too slow."""
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    s = sample_offsets(sub)
    out = []
    for (i, j, k) in cells:
        pts = np.stack(np.meshgrid((i + s) * h[0], (j + s) * h[1], (k + s) * h[2], indexing="ij"), -1).reshape(-1, 3)
        val = 1.0
        for o in range(len(phi_obj)):
            t = tris[tri_begin[o]:tri_begin[o + 1]]
            if len(t) == 0:
                continue
            used = verts[np.unique(t)]
            lo, hi = used.min(axis=0), used.max(axis=0)
            cell_lo = np.array([i * h[0], j * h[1], k * h[2]])
            cell_hi = cell_lo + np.asarray(h)
            if np.any(cell_hi <= lo) or np.any(cell_lo >= hi):
                continue
            f = inside(pts, verts, t).mean()
            if f > 0:
                val = min(val, 1.0 - f * (1.0 - phi_obj[o]))
        out.append(val)
    return np.array(out)
