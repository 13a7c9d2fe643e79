"""Seeded smooth perturbations of a state (test and benchmark inputs).

Parity tests at full size start both sides from the same state: the
oracle's initial state plus a smooth random perturbation drawn here.  The
perturbation is a sum of a few Fourier modes with seeded wave numbers,
phases and amplitudes; it holds none of the solver's arithmetic.
"""
import numpy as np


def smooth_noise(shape, seed, amplitude=1.0, modes=6, max_wave=4):
    """Array of ``shape`` (float64): sum of ``modes`` products of cosines
    cos(2 pi k_a x_a / n_a + phase_a) over the three axes, x_a the index,
    with integer wave numbers 0 .. max_wave, scaled so that the largest
    magnitude is ``amplitude``."""
    rng = np.random.default_rng(seed)
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    out = np.zeros(shape)
    for _ in range(modes):
        term = np.ones(shape)
        amp = rng.uniform(0.5, 1.0) * rng.choice([-1.0, 1.0])
        for a, x in enumerate(axes):
            k = int(rng.integers(0, max_wave + 1))
            ph = rng.uniform(0.0, 2.0 * np.pi)
            sh = [1, 1, 1]
            sh[a] = shape[a]
            term = term * np.cos(2.0 * np.pi * k * x / max(shape[a], 1) + ph).reshape(sh)
        out += amp * term
    m = np.abs(out).max()
    return out * (amplitude / m) if m > 0 else out


def perturbed_state(state, seed, rel_velocity=0.15, rel_turb=0.3):
    """A copy of ``state`` (dict of arrays: u, v, w, p, k, omega, nut) with
    smooth seeded perturbations: each velocity component gets noise of
    rel_velocity times the largest speed in the state; k and omega are
    multiplied by (1 + noise of rel_turb), so they stay positive for
    rel_turb < 1; p and nut are kept."""
    out = {f: np.array(v, dtype=np.float64, copy=True) for f, v in state.items()}
    vmax = max(float(np.abs(out[f]).max()) for f in ("u", "v", "w"))
    for q, f in enumerate(("u", "v", "w")):
        out[f] = out[f] + smooth_noise(out[f].shape, seed * 16 + q, rel_velocity * vmax)
    for q, f in enumerate(("k", "omega")):
        if f in out:
            out[f] = out[f] * (1.0 + smooth_noise(out[f].shape, seed * 16 + 3 + q, rel_turb))
    return out
