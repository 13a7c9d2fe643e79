"""Pins of the oracle's mesh voxelizer (Sec. 3, urban model resolving)
against closed forms: which sub-samples lie inside a box, a prism, a block
with a courtyard, a tetrahedron; the volume of a sphere mesh; invariances."""
import numpy as np

from uf_layouts import Box, porosity_field
from uf_layouts.meshes import box_mesh, prism_mesh, ring_mesh, uv_sphere_mesh, meshes_of
from oracle.voxelize import voxelize, inside, sample_offsets

N = (14, 12, 10)
H = (2.0, 1.5, 2.5)


def samples_of(n, h, sub):
    s = sample_offsets(sub)
    ax = [((np.arange(n[a])[:, None] + s[None, :]) * h[a]) for a in range(3)]
    return ax   # per axis: [cells, sub]


def fraction_from(mask_fn, n, h, sub):
    """f_in per cell from an explicit inside predicate on sample coordinates."""
    ax = samples_of(n, h, sub)
    X = ax[0][:, None, None, :, None, None]
    Y = ax[1][None, :, None, None, :, None]
    Z = ax[2][None, None, :, None, None, :]
    m = mask_fn(X, Y, Z)
    m = np.broadcast_to(m, (n[0], n[1], n[2], sub, sub, sub))
    return m.mean(axis=(3, 4, 5))


def test_box_mesh_equals_closed_form_box_porosity():
    x, y, z = (3.3, 17.1), (2.2, 9.7), (0.0, 13.3)
    v, t = box_mesh(x, y, z)
    for sub in (1, 2, 4):
        got = voxelize(N, H, v, t, [0, len(t)], [0.0], sub)
        ref = porosity_field(*N, *H, boxes=[Box(x, y, z, 0.0)], sub=sub)
        assert np.array_equal(got, ref), sub
    # an object porosity scales the solid fraction
    got = voxelize(N, H, v, t, [0, len(t)], [0.4], 4)
    ref = porosity_field(*N, *H, boxes=[Box(x, y, z, 0.4)], sub=4)
    assert np.array_equal(got, ref)


def test_prism_matches_point_in_polygon():
    cx, cy, r, z, n = 13.1, 8.3, 6.2, (1.1, 19.7), 7
    v, t = prism_mesh(cx, cy, r, z, nsides=n, phase=0.3)
    ang = 0.3 + 2 * np.pi * np.arange(n) / n
    px, py = cx + r * np.cos(ang), cy + r * np.sin(ang)

    def in_prism(X, Y, Z):
        ok = (Z > z[0]) & (Z < z[1])
        for a in range(n):
            b = (a + 1) % n
            # counter-clockwise polygon: inside is left of every edge
            ok = ok & ((px[b] - px[a]) * (Y - py[a]) - (py[b] - py[a]) * (X - px[a]) > 0)
        return ok
    got = voxelize(N, H, v, t, [0, len(t)], [0.0], 4)
    assert np.array_equal(got, 1.0 - fraction_from(in_prism, N, H, 4))
    assert got.min() == 0.0 and (got < 1).sum() > 20


def test_courtyard_block_is_not_convex():
    x, y, hx, hy, z = (2.3, 25.1), (1.2, 16.4), (9.1, 15.3), (5.3, 11.9), (0.0, 17.2)
    v, t = ring_mesh(x, y, hx, hy, z)

    def in_ring(X, Y, Z):
        outer = (X > x[0]) & (X < x[1]) & (Y > y[0]) & (Y < y[1]) & (Z > z[0]) & (Z < z[1])
        hole = (X > hx[0]) & (X < hx[1]) & (Y > hy[0]) & (Y < hy[1])
        return outer & ~hole
    got = voxelize(N, H, v, t, [0, len(t)], [0.0], 4)
    assert np.array_equal(got, 1.0 - fraction_from(in_ring, N, H, 4))
    # the courtyard itself stays open
    assert got[6, 5, 2] == 1.0


def test_tetrahedron_crossings_match_barycentric_inside():
    rng = np.random.default_rng(3)
    P = rng.normal(size=(4, 3)) * 3
    v = P
    t = np.array([(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)], dtype=np.int32)
    pts = rng.normal(size=(4000, 3)) * 2.5
    M = np.column_stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]])
    lam = np.linalg.solve(M, (pts - P[0]).T).T
    bary_in = (lam > 0).all(axis=1) & (lam.sum(axis=1) < 1)
    assert bary_in.sum() > 50
    assert np.array_equal(inside(pts, v, t), bary_in)


def test_sphere_volume_converges():
    c, r = (14.0, 10.2, 12.9), 8.3
    v, t = uv_sphere_mesh(c, r, 16, 32)
    # volume of the polyhedron by the divergence theorem
    a, b, d = v[t[:, 0]] - c, v[t[:, 1]] - c, v[t[:, 2]] - c
    vol = np.einsum("ij,ij->i", a, np.cross(b, d)).sum() / 6.0
    n, h = (16, 16, 12), (2.0, 1.5, 2.5)
    got = voxelize(n, h, v, t, [0, len(t)], [0.0], 4)
    est = (1.0 - got).sum() * np.prod(h)
    assert abs(est - vol) < 0.01 * vol, (est, vol)


def test_order_winding_and_bounding_box_pass_do_not_change_the_result():
    objs = [box_mesh((3.3, 17.1), (2.2, 9.7), (0.0, 13.3)) + (0.0,),
            prism_mesh(20.2, 11.3, 4.1, (0.0, 9.9), 9, 0.1) + (0.5,),
            ring_mesh((1.1, 12.2), (9.9, 17.5), (4.2, 8.8), (12.1, 15.2), (0.0, 7.7)) + (0.2,)]
    v, t, b, ph = meshes_of(objs)
    base = voxelize(N, H, v, t, b, ph, 2)
    assert np.array_equal(base, voxelize(N, H, v, t, b, ph, 2, use_aabb=False))
    t2 = t.copy()
    for o in range(len(ph)):
        seg = t2[b[o]:b[o + 1]]
        t2[b[o]:b[o + 1]] = seg[::-1][:, [0, 2, 1]]
    assert np.array_equal(base, voxelize(N, H, v, t2, b, ph, 2))
    # overlapping objects take the smallest porosity
    singles = [voxelize(N, H, *meshes_of([o])[:2], [0, len(o[1])], [o[2]], 2) for o in objs]
    assert np.array_equal(base, np.minimum.reduce(singles))
