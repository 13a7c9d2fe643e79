"""Pins of the oracle's discrete adjoint (oracle/adjoint.py): its forward is
the NumPy oracle's step, and its vector-Jacobian products are the
derivatives of that step -- checked against central differences of the NumPy
oracle, along random directions and entry by entry."""
import numpy as np
import pytest

from uf_layouts import perturbed_state
from oracle import OracleGrid
from oracle.adjoint import TorchStep, adjoint_steps, state_fields
from helpers import rel, random_small_config, random_porosity

import torch

FIELDS = ("u", "v", "w", "p", "k", "omega", "nut")


def _case(seed, **over):
    cfg = random_small_config(seed, dtype="f64", **over)
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    phi = random_porosity(seed, n)
    phi = np.where((phi > 0) & (phi < 1), phi, np.clip(phi, 0.05, 0.95))   # no exact 0/1: smooth drag
    og = OracleGrid(cfg)
    og.set_porosity(phi)
    st = perturbed_state(og.state(), seed=seed)
    return cfg, phi, st


def _oracle_run(cfg, phi, st, nsteps=1):
    og = OracleGrid(cfg)
    og.set_porosity(phi)
    for f, v in st.items():
        og.set_field(f, v)
    og.step(nsteps)
    return og.state()


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("stages", [1, 2, 4, 8, 16, 31])
def test_forward_equals_numpy_oracle(seed, stages):
    cfg, phi, st = _case(seed, stages=stages)
    ref = _oracle_run(cfg, phi, st)
    ts = TorchStep(cfg)
    out = ts.step({f: torch.tensor(st[f]) for f in FIELDS}, torch.tensor(phi))
    for f in FIELDS:
        assert rel(out[f].detach().numpy(), ref[f]) <= 1e-13, (f, rel(out[f].detach().numpy(), ref[f]))


def _J(cfg, phi, st, seed, fields, nsteps=1):
    out = _oracle_run(cfg, phi, st, nsteps)
    return sum(float((out[f] * seed[f]).sum()) for f in fields)


@pytest.mark.parametrize("seed,turb", [(0, 1), (1, 1), (2, 0), (3, 1), (5, 0)])
def test_vjp_matches_central_differences_directionally(seed, turb):
    cfg, phi, st = _case(seed, turb_model=turb)
    fields = state_fields(cfg)
    rng = np.random.default_rng(100 + seed)
    a = {f: rng.normal(size=st[f].shape) for f in fields}
    adj, phibar, _ = adjoint_steps(cfg, st, phi, a)
    d = {f: rng.normal(size=st[f].shape) * (np.abs(st[f]).mean() + 1e-3) for f in fields}
    dphi = rng.normal(size=phi.shape) * 0.01
    h = 1e-6
    plus = dict(st, **{f: st[f] + h * d[f] for f in fields})
    minus = dict(st, **{f: st[f] - h * d[f] for f in fields})
    fd = (_J(cfg, phi + h * dphi, plus, a, fields) - _J(cfg, phi - h * dphi, minus, a, fields)) / (2 * h)
    ad = sum(float((adj[f] * d[f]).sum()) for f in fields) + float((phibar * dphi).sum())
    assert abs(ad - fd) <= 1e-6 * abs(fd), (ad, fd)


def test_vjp_entries_match_central_differences():
    """Single entries of the porosity gradient and of the state adjoint
    against central differences of the NumPy oracle, k-omega on."""
    cfg, phi, st = _case(7)
    fields = state_fields(cfg)
    rng = np.random.default_rng(7)
    a = {f: rng.normal(size=st[f].shape) for f in fields}
    adj, phibar, _ = adjoint_steps(cfg, st, phi, a)
    h = 1e-6
    scale_phi = np.abs(phibar).max()
    for _ in range(5):
        c = tuple(int(rng.integers(s)) for s in phi.shape)
        e = np.zeros_like(phi)
        e[c] = 1.0
        fd = (_J(cfg, phi + h * e, st, a, fields) - _J(cfg, phi - h * e, st, a, fields)) / (2 * h)
        assert abs(phibar[c] - fd) <= 1e-6 * scale_phi, (c, phibar[c], fd)
    for f in ("u", "k"):
        scale = np.abs(adj[f]).max()
        for _ in range(4):
            c = tuple(int(rng.integers(s)) for s in st[f].shape)
            e = np.zeros_like(st[f])
            e[c] = 1.0
            fd = (_J(cfg, phi, dict(st, **{f: st[f] + h * e}), a, fields)
                  - _J(cfg, phi, dict(st, **{f: st[f] - h * e}), a, fields)) / (2 * h)
            assert abs(adj[f][c] - fd) <= 1e-6 * scale, (f, c, adj[f][c], fd)


def test_three_step_vjp_matches_central_differences():
    cfg, phi, st = _case(11)
    fields = state_fields(cfg)
    rng = np.random.default_rng(11)
    a = {f: rng.normal(size=st[f].shape) for f in fields}
    adj, phibar, _ = adjoint_steps(cfg, st, phi, a, nsteps=3)
    dphi = rng.normal(size=phi.shape) * 0.01
    h = 1e-6
    fd = (_J(cfg, phi + h * dphi, st, a, fields, 3) - _J(cfg, phi - h * dphi, st, a, fields, 3)) / (2 * h)
    assert abs(float((phibar * dphi).sum()) - fd) <= 1e-6 * abs(fd)
