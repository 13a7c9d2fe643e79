"""ctypes declarations of the C ABI (include/uf.h).  Argument marshalling only."""
import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_int64, c_void_p, c_char_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libuf.so")

STATUS = {0: "UF_OK", 1: "UF_EINVAL", 2: "UF_ENOMEM", 3: "UF_EDEVICE", 4: "UF_ENOCONV",
          5: "UF_ENONFINITE", 6: "UF_ESTATE", 7: "UF_ENOTIMPL"}
FIELDS = ("u", "v", "w", "p", "k", "omega", "nut", "phi")
FIELD_IDS = {name: i for i, name in enumerate(FIELDS)}


class uf_config(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("dx", c_double), ("dy", c_double), ("dz", c_double), ("dt", c_double),
        ("dtype", c_int32), ("bc", c_int32 * 6), ("inflow_kind", c_int32),
        ("u_ref", c_double), ("z_ref", c_double), ("z0", c_double), ("karman", c_double),
        ("wind_dir_deg", c_double), ("inflow_profile", POINTER(c_double)),
        ("nu", c_double), ("rho", c_double),
        ("turb_model", c_int32), ("turb_I", c_double), ("turb_L", c_double),
        ("k_min", c_double), ("omega_min", c_double),
        ("Cd", c_double), ("a", c_double), ("b", c_double), ("e", c_double),
        ("precond", c_int32), ("ai_omega", c_double), ("cg_tol", c_double),
        ("cg_maxit", c_int32), ("cg_criterion", c_int32), ("stages", c_int32),
        ("stream", c_void_p),
        ("alloc", c_void_p), ("free", c_void_p), ("alloc_ctx", c_void_p),
    ]


class uf_step_stats(ctypes.Structure):
    _fields_ = [("cg_iters", c_int32), ("cg_iters_total", c_int32), ("cg_rel_residual", c_double),
                ("converged", c_int32), ("nonfinite", c_int32), ("ms", c_float), ("cg_iters_max", c_int32),
                ("max_div", c_double), ("max_cfl", c_double), ("nut_clip_frac", c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class uf_batch_tuning(ctypes.Structure):
    _fields_ = [("band", c_int32 * 6), ("blocks", c_int32 * 6), ("ms", c_float * 6)]


OBJ_REGIONS, OBJ_PLANE, OBJ_FIELD = 0, 1, 2


class uf_objective_spec(ctypes.Structure):
    _fields_ = [("nregions", c_int32), ("boxes", POINTER(c_int32)), ("u_target", c_double),
                ("kind", c_int32), ("z_plane", c_double), ("s_target", c_double), ("s_min", c_double),
                ("w_penalty", c_double), ("u_target_dev", c_void_p), ("dJ_dphi_accum_dev", c_void_p)]


def make_objective_spec(regions, u_target):
    """uf_objective_spec from a list of boxes ((i0, i1), (j0, j1), (k0, k1)), half-open.
    Returns (struct, keepalive)."""
    flat = [int(v) for box in regions for lohi in box for v in lohi]
    keep = (c_int32 * max(len(flat), 1))(*flat)
    s = uf_objective_spec()
    s.kind = OBJ_REGIONS
    s.nregions = len(regions)
    s.boxes = ctypes.cast(keep, POINTER(c_int32))
    s.u_target = float(u_target)
    return s, keep


def make_plane_spec(z_plane, s_target=2.0, s_min=0.3, w_penalty=10.0):
    """uf_objective_spec of the pedestrian-plane objective."""
    s = uf_objective_spec()
    s.kind = OBJ_PLANE
    s.z_plane, s.s_target, s.s_min, s.w_penalty = float(z_plane), float(s_target), float(s_min), float(w_penalty)
    return s


class uf_mesh_set(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("dx", c_double), ("dy", c_double), ("dz", c_double),
                ("sub", c_int32), ("nobj", c_int32),
                ("tri_begin", POINTER(c_int32)), ("phi_obj", POINTER(c_double)),
                ("nverts", c_int32), ("ntris", c_int32),
                ("verts_dev", c_void_p), ("tris_dev", c_void_p)]


class uf_smooth_objects(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("dx", c_double), ("dy", c_double), ("dz", c_double), ("width", c_double),
                ("nboxes", c_int32), ("boxes", POINTER(c_double)),
                ("ncyls", c_int32), ("cylinders", POINTER(c_double))]


class UFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status
        self.name = STATUS.get(status, str(status))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libuf.so not found at %s; build it with "
                          "`python -m paper_2204_01117_amd.build`" % LIB_PATH)
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_SIGS = {
    "uf_create_grid": (c_int32, [POINTER(uf_config), POINTER(c_void_p)]),
    "uf_destroy_grid": (c_int32, [c_void_p]),
    "uf_set_porosity": (c_int32, [c_void_p, c_void_p]),
    "uf_set_field": (c_int32, [c_void_p, c_int32, c_void_p]),
    "uf_get_field": (c_int32, [c_void_p, c_int32, c_void_p]),
    "uf_field_extent": (c_int64, [POINTER(uf_config), c_int32, POINTER(c_int32)]),
    "uf_resolve_bc": (c_int32, [POINTER(uf_config), POINTER(c_int32)]),
    "uf_step": (c_int32, [c_void_p, c_int32, POINTER(uf_step_stats)]),
    "uf_pressure_solve": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(uf_step_stats)]),
    "uf_apply_operator": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "uf_objective": (c_int32, [c_void_p, c_void_p, POINTER(c_double), c_void_p]),
    "uf_adjoint_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "uf_adjoint_step_at": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "uf_set_stream": (c_int32, [c_void_p, c_void_p]),
    "uf_step_batch": (c_int32, [POINTER(c_void_p), c_int32, c_int32, c_void_p]),
    "uf_batch_create": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_void_p)]),
    "uf_batch_autotune": (c_int32, [c_void_p, POINTER(uf_batch_tuning)]),
    "uf_batch_step": (c_int32, [c_void_p, c_int32, c_void_p]),
    "uf_batch_destroy": (c_int32, [c_void_p]),
    "uf_smooth_porosity": (c_int32, [POINTER(uf_smooth_objects), c_int32, c_void_p, c_void_p]),
    "uf_smooth_porosity_grad": (c_int32, [POINTER(uf_smooth_objects), c_void_p, POINTER(c_double), c_void_p]),
    "uf_smooth_porosity_grad_noalloc": (c_int32, [POINTER(uf_smooth_objects), c_void_p, POINTER(c_double),
                                                  c_void_p]),
    "uf_voxelize": (c_int32, [POINTER(uf_mesh_set), c_int32, c_void_p, c_void_p, POINTER(c_double)]),
    "uf_kernel_timer_enable": (c_int32, [c_void_p, ctypes.c_uint32]),
    "uf_kernel_timer_read": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_int64)]),
    "uf_last_error": (c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

uf_create_grid = lib.uf_create_grid
uf_destroy_grid = lib.uf_destroy_grid
uf_set_porosity = lib.uf_set_porosity
uf_set_field = lib.uf_set_field
uf_get_field = lib.uf_get_field
uf_field_extent = lib.uf_field_extent
uf_resolve_bc = lib.uf_resolve_bc
uf_step = lib.uf_step
uf_pressure_solve = lib.uf_pressure_solve
uf_apply_operator = lib.uf_apply_operator
uf_objective = lib.uf_objective
uf_adjoint_step = lib.uf_adjoint_step
uf_adjoint_step_at = lib.uf_adjoint_step_at
uf_set_stream = lib.uf_set_stream
uf_step_batch = lib.uf_step_batch
uf_batch_create = lib.uf_batch_create
uf_batch_autotune = lib.uf_batch_autotune
uf_batch_step = lib.uf_batch_step
uf_batch_destroy = lib.uf_batch_destroy
uf_smooth_porosity = lib.uf_smooth_porosity
uf_smooth_porosity_grad = lib.uf_smooth_porosity_grad
uf_smooth_porosity_grad_noalloc = lib.uf_smooth_porosity_grad_noalloc
uf_voxelize = lib.uf_voxelize
uf_kernel_timer_enable = lib.uf_kernel_timer_enable
uf_kernel_timer_read = lib.uf_kernel_timer_read
TIMED_KERNELS = ("cg_Ad", "cg_axpy", "cg_precond", "mg_down0", "mg_up0", "mg_coarse", "cg_init",
                 "advect_fwd", "advect_corr", "diffuse", "drag", "project", "turbulence", "mg_update0",
                 "mg_rupd0")
uf_last_error = lib.uf_last_error


def check(status, allow=()):
    if status != 0 and status not in allow:
        msg = uf_last_error()
        raise UFError(status, msg.decode() if msg else "")
    return status


def make_config(cfg, stream=None):
    """Fill a uf_config from a configuration dictionary (keys as in uf.h).
    Returns (struct, keepalive) -- keep the second alive while the struct is used."""
    c = uf_config()
    for name, typ in uf_config._fields_:
        if name in ("bc", "inflow_profile", "stream", "dtype", "alloc", "free", "alloc_ctx"):
            continue
        setattr(c, name, cfg[name])
    dt = cfg["dtype"]
    c.dtype = {"f32": 0, "f64": 1}.get(dt, dt) if isinstance(dt, str) else int(dt)
    for s in range(6):
        c.bc[s] = int(cfg["bc"][s])
    keep = None
    if cfg.get("inflow_profile") is not None:
        keep = (c_double * len(cfg["inflow_profile"]))(*[float(x) for x in cfg["inflow_profile"]])
        c.inflow_profile = ctypes.cast(keep, POINTER(c_double))
    c.stream = stream
    return c, keep


# Device allocator callbacks of uf_config (alloc, free).
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


def torch_allocator(device, stream):
    """(alloc, free) callbacks that take the grid's memory from PyTorch's
    caching allocator on ``device`` for ``stream`` (a torch.cuda.Stream).
    Keep the returned pair alive as long as the grid."""
    import torch

    def _alloc(nbytes, ctx):
        return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(_alloc), FREE_FN(_free)
