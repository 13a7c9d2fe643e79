"""Shared helpers of the test-suite (comparison metrics, seeded inputs)."""
import numpy as np

from uf_layouts import default_config
from uf_layouts.configs import BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP

STATE_FIELDS = ("u", "v", "w", "p", "k", "omega", "nut")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_np(x):
    if hasattr(x, "detach"):
        return x.detach().double().cpu().numpy()
    return np.asarray(x, dtype=np.float64)


def state_errors(sg, so):
    """Relative L2 error per group: velocity (u, v, w stacked), p, k, omega, nut."""
    sg = {f: to_np(v) for f, v in sg.items()}
    so = {f: to_np(v) for f, v in so.items()}
    out = {"vel": rel(np.concatenate([sg[f].ravel() for f in "uvw"]),
                      np.concatenate([so[f].ravel() for f in "uvw"]))}
    for f in ("p", "k", "omega", "nut"):
        out[f] = rel(sg[f], so[f])
    return out


def random_small_config(seed, dtype="f64", **over):
    """A seeded small grid with random side kinds (at least one outlet),
    random wind direction and random cell sizes; ragged sizes on purpose."""
    rng = np.random.default_rng(seed)
    n = [int(x) for x in rng.integers(3, 14, size=3)]
    kinds = [int(x) for x in rng.choice([BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP], size=6)]
    if BC_OUTLET not in kinds:
        kinds[int(rng.integers(6))] = BC_OUTLET
    h = float(rng.uniform(0.8, 2.5))
    cfg = default_config(*n, h, dy=h * float(rng.uniform(0.7, 1.3)), dz=h * float(rng.uniform(0.7, 1.3)),
                         dtype=dtype, dt=float(0.25 * h / 6.0), u_ref=4.0, z_ref=3.0 * h,
                         wind_dir_deg=float(rng.uniform(0, 360)), bc=kinds)
    cfg.update(over)
    return cfg


def random_porosity(seed, n):
    """Porosity with exact 0 (solid), exact 1 (air) and porous cells."""
    rng = np.random.default_rng(seed + 1000)
    phi = rng.uniform(0.3, 1.0, size=n)
    phi[rng.random(n) < 0.15] = 0.0
    phi[rng.random(n) < 0.3] = 1.0
    return phi
