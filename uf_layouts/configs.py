"""Configuration dictionaries shared by the HIP path and the oracle.

The keys mirror the fields of ``uf_config`` in ``include/uf.h``.  The values
of the physical constants follow the paper: drag law constants a = 0.62,
b = 2.5, e = 1e-10 (Sec. 3, momentum equation with drag and its footnote),
C_d = 1.0 (appendix, porosity validation), k-omega coefficients from Table 1,
log-law inflow with kappa = 0.41 and z0 = 0.5 m (Sec. 5.1).  Values the
paper leaves open (nu, rho, turbulence intensity and length scale, time step
per workload) are readings documented with the design notes.

Workload presets describe synthetic stand-ins for the paper's urban models
(Bielefeld square, Nuernberg quarter), which are not available; see
``porosity.random_city`` for the layout recipe.
"""
import copy
import math

# Boundary kinds per domain side, sides ordered -x, +x, -y, +y, -z, +z.
BC_AUTO, BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP = -1, 0, 1, 2, 3
INFLOW_UNIFORM, INFLOW_LOGLAW, INFLOW_PROFILE = 0, 1, 2
TURB_OFF, TURB_KOMEGA = 0, 1
PC_NONE, PC_JACOBI, PC_AI1, PC_AI2, PC_MG = 0, 1, 2, 3, 4
STAGE_ADVECT, STAGE_DIFFUSE, STAGE_DRAG, STAGE_PROJECT, STAGE_TURB = 1, 2, 4, 8, 16
STAGE_ALL = 31


def default_config(nx=64, ny=32, nz=16, dx=4.0, dy=None, dz=None, **over):
    """Return a fresh configuration dictionary with every field set."""
    cfg = dict(
        nx=nx, ny=ny, nz=nz, dx=float(dx),
        dy=float(dx if dy is None else dy), dz=float(dx if dz is None else dz),
        dt=0.25, dtype="f32",
        bc=[BC_AUTO] * 6,
        inflow_kind=INFLOW_LOGLAW, u_ref=5.0, z_ref=10.0, z0=0.5, karman=0.41,
        wind_dir_deg=0.0, inflow_profile=None,
        nu=1.5e-5, rho=1.225,
        turb_model=TURB_KOMEGA, turb_I=0.1, turb_L=0.0,  # 0 -> 0.1 * domain height
        k_min=1e-10, omega_min=1e-10,
        Cd=1.0, a=0.62, b=2.5, e=1e-10,
        precond=PC_MG, ai_omega=1.6, cg_tol=1e-6, cg_maxit=500, cg_criterion=0,
        stages=STAGE_ALL,
    )
    for k, v in over.items():
        if k not in cfg:
            raise KeyError("unknown config key %r" % k)
        cfg[k] = v
    return cfg


def _c0():
    cfg = default_config(64, 32, 16, 4.0, dt=0.25, dtype="f64", u_ref=5.0, z_ref=10.0,
                         cg_tol=1e-8)
    # one solid box (12x8x10 cells) and one tree block (6x6x4 cells, phi 0.5),
    # both centred in y so that the layout is mirror-symmetric about y = L_y/2
    layout = dict(kind="objects",
                  boxes=[dict(x=(64.0, 112.0), y=(48.0, 80.0), z=(0.0, 40.0), phi=0.0),
                         dict(x=(160.0, 184.0), y=(52.0, 76.0), z=(4.0, 20.0), phi=0.5)],
                  cylinders=[])
    return dict(name="C0", config=cfg, steps=100, layout=layout,
                workload="64x32x16 dx=4m, 1 solid box + 1 tree block, log-law 5 m/s @10 m")


def _c1():
    cfg = default_config(256, 256, 64, 2.0, dt=0.09, dtype="f32", u_ref=6.0, z_ref=10.0)
    layout = dict(kind="random", seed=1, n_boxes=40, n_trees=60)
    return dict(name="C1", config=cfg, steps=500, layout=layout,
                workload="256x256x64 dx=2m, 40 buildings + 60 trees, log-law 6 m/s @10 m")


def _c2():
    cfg = default_config(512, 512, 128, 1.0, dt=0.045, dtype="f32", u_ref=6.0, z_ref=10.0)
    layout = dict(kind="random", seed=2, n_boxes=200, n_trees=400, random_direction=True)
    return dict(name="C2", config=cfg, steps=300, layout=layout,
                workload="512x512x128 dx=1m, 200 buildings + 400 trees, random direction")


def _c3():
    shapes = [(128, 128, 48), (192, 160, 48), (256, 256, 64)]
    cases = []
    for c in range(16):
        d, v = divmod(c, 2)
        cases.append(dict(seed=3000 + c, direction=45.0 * d, variant=v, shapes=shapes))
    cfg = default_config(128, 128, 48, 2.0, dt=0.09, dtype="f32", u_ref=6.0, z_ref=10.0)
    layout = dict(kind="batched", cases=cases, n_range=(20, 60))
    return dict(name="C3", config=cfg, steps=200, layout=layout,
                workload="16 cases, 8 directions x 2 variants, uneven grids")


def _c4():
    cfg = default_config(256, 256, 64, 2.0, dt=0.09, dtype="f32", u_ref=6.0, z_ref=10.0)
    layout = dict(kind="random", seed=4, n_boxes=21, n_trees=40)
    return dict(name="C4", config=cfg, steps=200, layout=layout,
                workload="256x256x64 dx=2m, 21 parametrised buildings + 40 trees")


def _cp():
    # paper-shaped context workload: 450x300x40 cells of 1 m, dt = 0.2 s;
    # friction speed 0.40 m/s with z0 = 0.5 m, i.e. U(10 m) = 0.40/0.41*ln(20)
    u_ref = 0.40 / 0.41 * math.log(20.0)
    cfg = default_config(450, 300, 40, 1.0, dt=0.2, dtype="f32", u_ref=u_ref, z_ref=10.0)
    layout = dict(kind="random", seed=5, n_boxes=60, n_trees=80, height=(10.0, 30.0))
    return dict(name="CP", config=cfg, steps=200, layout=layout,
                workload="450x300x40 dx=1m dt=0.2s (paper case-study shape)")


PRESETS = dict(C0=_c0, C1=_c1, C2=_c2, C3=_c3, C4=_c4, CP=_cp)


def preset(name, **over):
    """Return a deep copy of preset ``name`` with config fields overridden."""
    p = copy.deepcopy(PRESETS[name]())
    for k, v in over.items():
        if k not in p["config"]:
            raise KeyError("unknown config key %r" % k)
        p["config"][k] = v
    return p
