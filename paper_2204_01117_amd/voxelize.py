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


def _smooth_objects(n, h, boxes, cylinders, width):
    """uf_smooth_objects and the host arrays it points to."""
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
    return o, (bk, ck)


def smooth_porosity(n, h, boxes, cylinders, width, dtype="f32", device="cuda:0"):
    """Porosity [nx, ny, nz] of objects with smoothed faces (uf_smooth_porosity):
    ``boxes`` rows (x0, x1, y0, y1, z0, z1, phi), ``cylinders`` rows
    (cx, cy, R, z0, z1, phi), logistic steps of ``width`` metres."""
    import torch
    dev = torch.device(device)
    tdt = torch.float32 if dtype in ("f32", 0) else torch.float64
    o, keep = _smooth_objects(n, h, boxes, cylinders, width)
    out = torch.empty(tuple(int(x) for x in n), dtype=tdt, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    L.check(L.uf_smooth_porosity(ctypes.byref(o), 0 if tdt == torch.float32 else 1, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(stream)))
    del keep
    return out


def smooth_porosity_grad(n, h, boxes, cylinders, width, phibar, noalloc=False):
    """Reverse of ``smooth_porosity`` (uf_smooth_porosity_grad): from
    phibar = dJ/dphi (float64 [nx, ny, nz] on the GPU) to dJ/d(box rows)
    and dJ/d(cylinder rows), numpy arrays shaped like ``boxes`` (7 columns)
    and ``cylinders`` (6 columns).  ``noalloc`` calls
    uf_smooth_porosity_grad_noalloc, which allocates no device memory."""
    import numpy as np
    import torch
    assert phibar.dtype == torch.float64 and phibar.is_cuda and phibar.is_contiguous()
    assert tuple(phibar.shape) == tuple(int(x) for x in n)
    o, keep = _smooth_objects(n, h, boxes, cylinders, width)
    nb, nc = len(boxes), len(cylinders)
    out = (ctypes.c_double * max(7 * nb + 6 * nc, 1))()
    stream = torch.cuda.current_stream(phibar.device).cuda_stream
    fn = L.uf_smooth_porosity_grad_noalloc if noalloc else L.uf_smooth_porosity_grad
    L.check(fn(ctypes.byref(o), ctypes.c_void_p(phibar.data_ptr()), out, ctypes.c_void_p(stream)))
    del keep
    g = np.array(out[:7 * nb + 6 * nc], dtype=np.float64)
    return g[:7 * nb].reshape(nb, 7), g[7 * nb:].reshape(nc, 6)
