"""Grid: a handle of the C ABI with torch CUDA tensors as device buffers."""
import ctypes
from ctypes import byref, c_int32, c_void_p

from . import _lib as L


class Grid:
    """One simulation grid on a GPU.  ``cfg`` is a configuration dictionary
    (see ``uf_layouts.default_config``).  All work is enqueued on torch's
    current stream of ``device``."""

    def __init__(self, cfg, device="cuda:0", stream=None, torch_memory=True, allocator=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.dtype = torch.float64 if str(cfg["dtype"]) in ("f64", "1") else torch.float32
        # ``stream``: a torch.cuda.Stream of its own (batched cases); by
        # default torch's current stream
        self.tstream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = self.tstream.cuda_stream
        c, keep = L.make_config(self.cfg, self.stream)
        # the grid's buffers come from ``allocator`` (an (alloc, free) pair of
        # uf_config callbacks, L.ALLOC_FN / L.FREE_FN) when given, else from
        # torch's caching allocator, unless torch_memory is False (hipMalloc)
        if allocator is not None:
            self._allocator = allocator
        else:
            self._allocator = L.torch_allocator(self.device, self.tstream) if torch_memory else None
        if self._allocator is not None:
            c.alloc = ctypes.cast(self._allocator[0], c_void_p)
            c.free = ctypes.cast(self._allocator[1], c_void_p)
        self._cstruct = c
        h = c_void_p()
        L.check(L.uf_create_grid(byref(c), byref(h)))
        del keep
        self.handle = h
        self.n = (int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"]))

    # ------------------------------------------------------------------ util
    def extent(self, name):
        d = (c_int32 * 3)()
        L.uf_field_extent(byref(self._cstruct), L.FIELD_IDS[name], d)
        return tuple(d)

    def _dev(self, t, shape):
        torch = self.torch
        t = torch.as_tensor(t).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    # ------------------------------------------------------------------- API
    def set_porosity(self, phi):
        t = self._dev(phi, self.n)
        self.torch.cuda.current_stream(self.device).synchronize()
        L.check(L.uf_set_porosity(self.handle, c_void_p(t.data_ptr())))
        self.tstream.synchronize()

    def set_field(self, name, arr):
        t = self._dev(arr, self.extent(name))
        self.torch.cuda.current_stream(self.device).synchronize()
        L.check(L.uf_set_field(self.handle, L.FIELD_IDS[name], c_void_p(t.data_ptr())))
        self.tstream.synchronize()

    def get_field(self, name):
        out = self.torch.empty(self.extent(name), dtype=self.dtype, device=self.device)
        L.check(L.uf_get_field(self.handle, L.FIELD_IDS[name], c_void_p(out.data_ptr())))
        if self.tstream != self.torch.cuda.current_stream(self.device):
            self.tstream.synchronize()
        return out

    def state(self):
        return {f: self.get_field(f) for f in ("u", "v", "w", "p", "k", "omega", "nut")}

    def set_state(self, st):
        for f, a in st.items():
            if f != "phi":
                self.set_field(f, a)

    def step(self, nsteps=1, stats=True, allow=()):
        s = L.uf_step_stats()
        rc = L.uf_step(self.handle, int(nsteps), byref(s) if stats else None)
        L.check(rc, allow)
        d = s.as_dict() if stats else {}
        d["status"] = L.STATUS[rc]
        return d

    def pressure_solve(self, b, x0=None, allow=()):
        b = self._dev(b, self.n)
        x = self._dev(x0 if x0 is not None else self.torch.zeros(self.n), self.n).clone()
        s = L.uf_step_stats()
        self.torch.cuda.current_stream(self.device).synchronize()
        rc = L.uf_pressure_solve(self.handle, c_void_p(b.data_ptr()), c_void_p(x.data_ptr()), byref(s))
        L.check(rc, allow)
        d = s.as_dict()
        d["status"] = L.STATUS[rc]
        return x, d

    def apply_operator(self, op, x):
        x = self._dev(x, self.n)
        y = self.torch.empty(self.n, dtype=self.dtype, device=self.device)
        own = self.tstream != self.torch.cuda.current_stream(self.device)
        if own:
            self.torch.cuda.current_stream(self.device).synchronize()
        L.check(L.uf_apply_operator(self.handle, int(op), c_void_p(x.data_ptr()), c_void_p(y.data_ptr())))
        if own:
            self.tstream.synchronize()
        return y

    def _seed_buffer(self):
        """Flat device buffer of the three face components (u, v, w blocks)
        and its per-component views."""
        ext = [self.extent(f) for f in ("u", "v", "w")]
        sizes = [e[0] * e[1] * e[2] for e in ext]
        buf = self.torch.empty(sum(sizes), dtype=self.dtype, device=self.device)
        views, o = [], 0
        for e, n in zip(ext, sizes):
            views.append(buf[o:o + n].view(e))
            o += n
        return buf, tuple(views)

    def _objective(self, spec, grad):
        J = ctypes.c_double()
        buf, views = self._seed_buffer() if grad else (None, None)
        self.torch.cuda.current_stream(self.device).synchronize()
        L.check(L.uf_objective(self.handle, byref(spec), byref(J),
                               c_void_p(buf.data_ptr()) if grad else None))
        return (J.value, views) if grad else J.value

    def objective(self, regions, u_target, grad=False):
        """Target-region objective sum_i (mean speed of region i - u_target)^2 of
        the current state; regions are boxes ((i0, i1), (j0, j1), (k0, k1)).
        With ``grad``, also its derivative with respect to the state's faces
        as (du, dv, dw) tensors (the seed of the adjoint)."""
        spec, keep = L.make_objective_spec(regions, u_target)
        out = self._objective(spec, grad)
        del keep
        return out

    def field_objective(self, regions, u_target, grad=False):
        """General objective sum_i ||F_i(u) - F_i(u_t)||_2 with F_i the
        cell-centre velocities of region i; ``u_target`` is [3, nx, ny, nz].
        ``grad`` as in ``objective``."""
        ut = self._dev(u_target, (3,) + self.n)
        spec, keep = L.make_objective_spec(regions, 0.0)
        spec.kind = L.OBJ_FIELD
        spec.u_target_dev = ut.data_ptr()
        out = self._objective(spec, grad)
        del keep, ut
        return out

    def adjoint_fields(self):
        """Fields of the state the reverse step takes: (u, v, w), plus (k,
        omega, nut) when the k-omega update runs in the step."""
        turb = int(self.cfg["turb_model"]) == 1 and int(self.cfg["stages"]) & 16
        return ("u", "v", "w", "k", "omega", "nut") if turb else ("u", "v", "w")

    def adjoint_step(self, state, adj, phibar=None, after=None):
        """Reverse of one step (uf_adjoint_step): ``state`` holds the fields
        of ``adjoint_fields()`` the step started from, ``adj`` the
        derivative of the objective with respect to the same fields after
        the step; returns the derivative with respect to ``state`` and adds
        the porosity derivative of this step into ``phibar`` (float64
        [nx, ny, nz]) when given.  ``after``: the (u, v, w, ...) the step
        produced, when the caller holds it (uf_adjoint_step_at: no
        recompute of the projection for the k-omega reverse)."""
        names = self.adjoint_fields()
        assert len(state) == len(names) and len(adj) == len(names)
        st = [self._dev(a, self.extent(f)) for a, f in zip(state, names)]
        nx = [self._dev(a, self.extent(f)) for a, f in zip(after[:3], names)] if after is not None else None
        ad = [self._dev(a, self.extent(f)) for a, f in zip(adj, names)]
        out = [self.torch.empty(self.extent(f), dtype=self.dtype, device=self.device) for f in names]
        if phibar is not None:
            assert phibar.dtype == self.torch.float64 and tuple(phibar.shape) == self.n and phibar.is_contiguous()
        ptrs = lambda ts: (c_void_p * len(ts))(*[t.data_ptr() for t in ts])
        own = self.tstream != self.torch.cuda.current_stream(self.device)
        if own:
            self.torch.cuda.current_stream(self.device).synchronize()
        pb = c_void_p(phibar.data_ptr()) if phibar is not None else None
        if nx is not None:
            L.check(L.uf_adjoint_step_at(self.handle, ptrs(st), ptrs(nx), ptrs(ad), ptrs(out), pb))
        else:
            L.check(L.uf_adjoint_step(self.handle, ptrs(st), ptrs(ad), ptrs(out), pb))
        if own:
            self.tstream.synchronize()
        return tuple(out)

    def plane_objective(self, z_plane, s_target=2.0, s_min=0.3, w_penalty=10.0, grad=False, phibar=None):
        """Pedestrian-comfort objective on the horizontal plane z = z_plane:
        dx dy sum phi [(s - s_target)^2 + w_penalty max(0, s_min - s)^2].
        With ``grad`` as in ``objective``; its direct porosity derivative is
        added into ``phibar`` (float64 [nx, ny, nz]) when given."""
        spec = L.make_plane_spec(z_plane, s_target, s_min, w_penalty)
        if phibar is not None:
            assert grad and phibar.dtype == self.torch.float64 and tuple(phibar.shape) == self.n
            spec.dJ_dphi_accum_dev = phibar.data_ptr()
        return self._objective(spec, grad)

    def timer_enable(self, kernels=()):
        """Time every launch of the named kernels (see TIMED_KERNELS)."""
        mask = 0
        for k in kernels:
            mask |= 1 << L.TIMED_KERNELS.index(k)
        L.check(L.uf_kernel_timer_enable(self.handle, mask))

    def timer_read(self, kernel):
        """(total milliseconds, launches) of one timed kernel."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        L.check(L.uf_kernel_timer_read(self.handle, L.TIMED_KERNELS.index(kernel), byref(ms), byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "handle", None):
            L.uf_destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(grids, nsteps=1, stats=True, allow=()):
    """Advance several grids by ``nsteps`` each through uf_step_batch (give
    each Grid its own ``stream`` for their kernels to overlap).  Returns one
    stats dictionary per grid."""
    n = len(grids)
    arr = (c_void_p * n)(*[g.handle for g in grids])
    st = (L.uf_step_stats * n)()
    rc = L.uf_step_batch(arr, n, int(nsteps), ctypes.cast(st, c_void_p) if stats else None)
    L.check(rc, allow)
    out = [st[i].as_dict() if stats else {} for i in range(n)]
    for d in out:
        d["status"] = L.STATUS[rc]
    return out


STAGE_NAMES = ("predictor", "corrector", "diffusion", "drag", "projection", "k-omega")


class Batch:
    """Several grids advanced together (uf_batch): one persistent launch per
    stage for all of them, each step replayed from two hipGraphs.  The grids
    stay usable on their own between calls."""

    def __init__(self, grids):
        n = len(grids)
        self.grids = list(grids)
        arr = (c_void_p * n)(*[g.handle for g in grids])
        h = c_void_p()
        L.check(L.uf_batch_create(arr, n, byref(h)))
        self.handle = h

    def autotune(self):
        """Time every stage's launch for each band width and grid size (on
        scratch sets) and keep the fastest; returns the choice per stage."""
        t = L.uf_batch_tuning()
        L.check(L.uf_batch_autotune(self.handle, byref(t)))
        return {name: {"band": t.band[i], "blocks": t.blocks[i], "ms": t.ms[i]}
                for i, name in enumerate(STAGE_NAMES)}

    def step(self, nsteps=1, stats=True, allow=()):
        n = len(self.grids)
        arr = (L.uf_step_stats * n)() if stats else None
        rc = L.uf_batch_step(self.handle, int(nsteps), arr)
        L.check(rc, allow)
        if not stats:
            return [{"status": L.STATUS[rc]} for _ in range(n)]
        out = []
        for s in arr:
            d = s.as_dict()
            d["status"] = L.STATUS[rc]
            out.append(d)
        return out

    def close(self):
        if self.handle:
            L.uf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
