"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/uf.h, and rejects bad configurations before any
device work (UF_EINVAL with a message)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_01117_amd", "libuf.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libuf.so not built")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "uf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(uf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_named_entry_points():
    names = declared_functions()
    for n in ("uf_create_grid", "uf_set_porosity", "uf_step", "uf_objective", "uf_adjoint_step",
              "uf_destroy_grid", "uf_get_field", "uf_set_field", "uf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_exposes_same_names():
    import paper_2204_01117_amd as U
    for n in declared_functions():
        assert hasattr(U, n), n


def _create(cfg):
    import paper_2204_01117_amd as U
    c, keep = U.make_config(cfg)
    h = ctypes.c_void_p()
    rc = U.uf_create_grid(ctypes.byref(c), ctypes.byref(h))
    return rc, U.uf_last_error().decode(), h


@pytest.mark.parametrize("override,needle", [
    (dict(nx=0), "grid sizes"),
    (dict(dt=0.0), "dt"),
    (dict(dt=float("nan")), "dt"),
    (dict(dx=-1.0), "dx"),
    (dict(dtype=7), "dtype"),
    (dict(bc=[0, 0, 0, 0, 2, 3]), "outlet"),
    (dict(bc=[9, 1, 1, 1, 2, 3]), "boundary kind"),
    (dict(nu=1e3), "stability"),
    (dict(precond=5), "preconditioner"),
    (dict(ai_omega=2.0), "ai_omega"),
    (dict(cg_tol=0.0), "cg_tol"),
    (dict(cg_maxit=0), "cg_maxit"),
    (dict(cg_criterion=2), "cg_criterion"),
    (dict(stages=64), "stage"),
    (dict(z0=20.0), "log-law"),
    (dict(turb_I=0.0), "k-omega"),
    (dict(e=0.0), "e must"),
    (dict(inflow_kind=2, inflow_profile=None), "inflow_profile"),
])
def test_invalid_configs_are_rejected_before_device_work(override, needle):
    from uf_layouts import default_config
    cfg = default_config(8, 6, 4, 2.0, dt=0.2)
    cfg.update(override)
    rc, msg, h = _create(cfg)
    assert rc == 1, (rc, msg)          # UF_EINVAL
    assert needle in msg, msg
    assert not h.value


def test_null_arguments():
    import paper_2204_01117_amd as U
    assert U.uf_create_grid(None, None) == 1
    assert U.uf_destroy_grid(None) == 1
    assert U.uf_step(None, 1, None) == 1
    assert U.uf_set_porosity(None, None) == 1


def test_field_extents():
    import paper_2204_01117_amd as U
    from uf_layouts import default_config
    c, _ = U.make_config(default_config(5, 4, 3, 1.0))
    d = (ctypes.c_int32 * 3)()
    assert U.uf_field_extent(ctypes.byref(c), 0, d) == 6 * 4 * 3 and tuple(d) == (6, 4, 3)
    assert U.uf_field_extent(ctypes.byref(c), 1, d) == 5 * 5 * 3 and tuple(d) == (5, 5, 3)
    assert U.uf_field_extent(ctypes.byref(c), 2, d) == 5 * 4 * 4 and tuple(d) == (5, 4, 4)
    for f in range(3, 8):
        assert U.uf_field_extent(ctypes.byref(c), f, d) == 60 and tuple(d) == (5, 4, 3)
    assert U.uf_field_extent(ctypes.byref(c), 8, d) == -1


def test_adjoint_and_objective_reject_null():
    import paper_2204_01117_amd as U
    assert U.uf_adjoint_step(None, None, None, None, None) == 1
    assert U.uf_objective(None, None, None, None) == 1


def _header_structs():
    import re
    src = open(os.path.join(ROOT, "include", "uf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", src, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            fn = re.search(r"\(\*(\w+)\)\s*\(", decl)
            if fn:                                   # a function pointer field
                fields.append((fn.group(1), "fnptr", True, 1))
                continue
            parts = decl.split(",")
            first = parts[0].split()
            typ = " ".join(first[:-1]).replace("const ", "")
            names = [first[-1]] + [p.strip() for p in parts[1:]]
            for n in names:
                ptr = n.startswith("*") or typ.endswith("*")
                arr = re.search(r"\[(\d+)\]", n)
                fields.append((n.strip("*").split("[")[0], typ.rstrip("*").strip(), ptr,
                               int(arr.group(1)) if arr else 1))
        out[name] = fields
    return out


def test_ctypes_structs_match_the_header():
    """Field names, order, scalar types and array lengths of the ctypes
    mirrors equal the C declarations (a layout mismatch would corrupt every
    call)."""
    import ctypes
    import paper_2204_01117_amd as U
    ctype_of = {"int32_t": ctypes.c_int32, "double": ctypes.c_double, "float": ctypes.c_float}
    decl = _header_structs()
    for cname, cls in (("uf_config", U.uf_config), ("uf_step_stats", U.uf_step_stats),
                       ("uf_objective_spec", U.uf_objective_spec), ("uf_mesh_set", U.uf_mesh_set),
                       ("uf_smooth_objects", U.uf_smooth_objects), ("uf_batch_tuning", U.uf_batch_tuning)):
        hdr = decl[cname]
        assert [f[0] for f in hdr] == [f[0] for f in cls._fields_], cname
        for (name, typ, ptr, count), (_, ct) in zip(hdr, cls._fields_):
            if ptr:
                assert ct is ctypes.c_void_p or hasattr(ct, "contents") or issubclass(ct, ctypes._Pointer), name
            elif count > 1:
                assert ct._length_ == count and ct._type_ is ctype_of[typ], name
            else:
                assert ct is ctype_of[typ], (cname, name, typ, ct)


@pytest.mark.parametrize("deg,expect", [
    (0.0, [0, 1, 1, 1, 2, 3]),          # wind +x enters through -x
    (90.0, [1, 1, 0, 1, 2, 3]),         # cos 90 deg ~ 6e-17: tangential to the x sides
    (180.0, [1, 0, 1, 1, 2, 3]),
    (225.0, [1, 0, 1, 0, 2, 3]),        # through +x and +y
    (270.0, [1, 1, 1, 0, 2, 3]),
    (30.0, [0, 1, 0, 1, 2, 3]),
])
def test_library_resolves_auto_sides_like_the_hand_table(deg, expect):
    """The library's side-kind rule against the same hand table the oracle's
    rule is pinned to (inlet where the wind enters, ground wall, sky slip)."""
    import ctypes
    import paper_2204_01117_amd as U
    from uf_layouts import default_config
    c, keep = U.make_config(default_config(8, 6, 4, 1.0, wind_dir_deg=deg))
    out = (ctypes.c_int32 * 6)()
    assert U.uf_resolve_bc(ctypes.byref(c), out) == 0
    assert list(out) == expect


def test_library_resolve_bc_explicit_and_errors():
    import ctypes
    import math
    import paper_2204_01117_amd as U
    from uf_layouts import default_config
    out = (ctypes.c_int32 * 6)()
    c, _ = U.make_config(default_config(8, 6, 4, 1.0, wind_dir_deg=45.0, bc=[1, -1, 2, -1, 3, -1]))
    assert U.uf_resolve_bc(ctypes.byref(c), out) == 0 and list(out) == [1, 1, 2, 1, 3, 3]
    c, _ = U.make_config(default_config(8, 6, 4, 1.0, wind_dir_deg=math.degrees(math.acos(1e-9))))
    assert U.uf_resolve_bc(ctypes.byref(c), out) == 0 and out[0] == 0
    c, _ = U.make_config(default_config(8, 6, 4, 1.0, wind_dir_deg=math.degrees(math.acos(1e-13))))
    assert U.uf_resolve_bc(ctypes.byref(c), out) == 0 and out[0] == 1
    c, _ = U.make_config(default_config(8, 6, 4, 1.0, wind_dir_deg=float("nan")))
    assert U.uf_resolve_bc(ctypes.byref(c), out) == 1
    assert U.uf_resolve_bc(None, out) == 1


def test_allocator_hook_needs_both_functions():
    import paper_2204_01117_amd as U
    from uf_layouts import default_config
    c, _ = U.make_config(default_config(8, 6, 4, 2.0, dt=0.2))
    fn = U._lib.ALLOC_FN(lambda n, ctx: 0)
    c.alloc = ctypes.cast(fn, ctypes.c_void_p)
    h = ctypes.c_void_p()
    assert U.uf_create_grid(ctypes.byref(c), ctypes.byref(h)) == 1
    assert "alloc" in U.uf_last_error().decode() and not h.value


def test_batch_calls_reject_bad_arguments_without_a_device():
    """uf_batch_create checks its list before touching the device: NULL
    list or handle, no grids, more than UF_BATCH_MAX_GRIDS, a NULL entry;
    the other batch calls reject a NULL batch."""
    import ctypes
    import paper_2204_01117_amd as U
    h = ctypes.c_void_p()
    assert U.uf_batch_create(None, 1, ctypes.byref(h)) == 1
    arr = (ctypes.c_void_p * 65)()
    assert U.uf_batch_create(arr, 1, None) == 1
    assert U.uf_batch_create(arr, 0, ctypes.byref(h)) == 1
    assert U.uf_batch_create(arr, 65, ctypes.byref(h)) == 1
    assert b"at most 64" in U.uf_last_error()
    assert U.uf_batch_create(arr, 2, ctypes.byref(h)) == 1
    assert b"NULL grid" in U.uf_last_error()
    assert not h.value
    assert U.uf_batch_step(None, 1, None) == 1
    assert U.uf_batch_autotune(None, None) == 1
    assert U.uf_batch_destroy(None) == 1
