"""Cell porosity of triangle-mesh objects on the GPU (``uf_voxelize``).

Argument marshalling only: the bounding-box pass, the ray casting and the
cut-cell sub-sampling all run in the library's HIP kernels.
"""
import ctypes

import numpy as np

from . import _lib as L


def voxelize(n, h, verts, tris, tri_begin, phi_obj, sub=4, dtype="f32", device="cuda:0", timing=None):
    """Porosity [nx, ny, nz] (a torch tensor on ``device``) of the objects.

    ``verts`` [V, 3] and ``tris`` [T, 3] (host arrays or device tensors),
    ``tri_begin`` [nobj + 1] and ``phi_obj`` [nobj] (host) as in
    ``uf_mesh_set``.  Runs on torch's current stream of ``device``.  Pass a
    dict as ``timing`` to receive the ray-casting kernel's milliseconds
    under "cast_ms"."""
    import torch
    dev = torch.device(device)
    tdt = torch.float32 if dtype in ("f32", 0) else torch.float64
    v = torch.as_tensor(np.asarray(verts, np.float64) if not torch.is_tensor(verts) else verts)
    v = v.to(device=dev, dtype=torch.float64).contiguous()
    t = torch.as_tensor(np.asarray(tris, np.int32) if not torch.is_tensor(tris) else tris)
    t = t.to(device=dev, dtype=torch.int32).contiguous()
    begin = (ctypes.c_int32 * len(tri_begin))(*[int(x) for x in tri_begin])
    pobj = (ctypes.c_double * max(len(phi_obj), 1))(*[float(x) for x in phi_obj])
    m = L.uf_mesh_set()
    m.nx, m.ny, m.nz = (int(x) for x in n)
    m.dx, m.dy, m.dz = (float(x) for x in h)
    m.sub = int(sub)
    m.nobj = len(phi_obj)
    m.tri_begin = ctypes.cast(begin, ctypes.POINTER(ctypes.c_int32))
    m.phi_obj = ctypes.cast(pobj, ctypes.POINTER(ctypes.c_double))
    m.nverts = int(v.shape[0]) if v.numel() else 0
    m.ntris = int(t.shape[0]) if t.numel() else 0
    m.verts_dev = v.data_ptr() if v.numel() else None
    m.tris_dev = t.data_ptr() if t.numel() else None
    out = torch.empty(tuple(int(x) for x in n), dtype=tdt, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    ms = ctypes.c_double()
    L.check(L.uf_voxelize(ctypes.byref(m), 0 if tdt == torch.float32 else 1, ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(stream), ctypes.byref(ms) if timing is not None else None))
    if timing is not None:
        timing["cast_ms"] = ms.value
    return out


def smooth_porosity(n, h, boxes, cylinders, width, dtype="f32", device="cuda:0"):
    """Porosity [nx, ny, nz] of objects with smoothed faces (uf_smooth_porosity):
    ``boxes`` rows (x0, x1, y0, y1, z0, z1, phi), ``cylinders`` rows
    (cx, cy, R, z0, z1, phi), logistic steps of ``width`` metres."""
    import torch
    dev = torch.device(device)
    tdt = torch.float32 if dtype in ("f32", 0) else torch.float64
    bx = [float(v) for row in boxes for v in row]
    cy = [float(v) for row in cylinders for v in row]
    bk = (ctypes.c_double * max(len(bx), 1))(*bx)
    ck = (ctypes.c_double * max(len(cy), 1))(*cy)
    o = L.uf_smooth_objects()
    o.nx, o.ny, o.nz = (int(x) for x in n)
    o.dx, o.dy, o.dz = (float(x) for x in h)
    o.width = float(width)
    o.nboxes, o.ncyls = len(boxes), len(cylinders)
    o.boxes = ctypes.cast(bk, ctypes.POINTER(ctypes.c_double))
    o.cylinders = ctypes.cast(ck, ctypes.POINTER(ctypes.c_double))
    out = torch.empty(tuple(int(x) for x in n), dtype=tdt, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    L.check(L.uf_smooth_porosity(ctypes.byref(o), 0 if tdt == torch.float32 else 1, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(stream)))
    return out
