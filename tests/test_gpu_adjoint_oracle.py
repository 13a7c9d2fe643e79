"""The GPU's reverse step (uf_adjoint_step, FP64) against the oracle's own
discrete adjoint (oracle/adjoint.py: torch autograd through an FP64
transcription of the oracle's step, pinned to the NumPy oracle and to its
central differences), element by element: the state adjoint of every field
the reverse carries and the porosity gradient, for one step and for a chain
of four, on ragged random grids with random side kinds, with and without
the k-omega update.  Inputs: the oracle's initial state plus a seeded smooth
perturbation, and seeded normal adjoint seeds."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from uf_layouts import perturbed_state
from uf_layouts.configs import PC_MG, TURB_OFF, TURB_KOMEGA
from oracle import OracleGrid
from oracle.adjoint import adjoint_steps, state_fields
from helpers import rel, to_np, random_small_config, random_porosity

import paper_2204_01117_amd as U


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(seed, turb):
    cfg = random_small_config(seed, dtype="f64", precond=PC_MG, cg_tol=1e-13, cg_maxit=5000,
                              turb_model=TURB_KOMEGA if turb else TURB_OFF)
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    phi = random_porosity(seed, n)
    og = OracleGrid(cfg)
    st = perturbed_state(og.state(), seed=seed)
    rng = np.random.default_rng(500 + seed)
    seed_adj = {f: rng.normal(size=st[f].shape) for f in state_fields(cfg)}
    return cfg, phi, st, seed_adj


def _grid(cfg, phi, st):
    g = U.Grid(cfg)
    g.set_porosity(torch.as_tensor(phi))
    g.set_state({f: torch.as_tensor(v) for f, v in st.items()})
    return g


def _compare(what, gpu, ref, tol):
    errs = {f: rel(to_np(gpu[f]), ref[f]) for f in ref}
    log(what, {f: "%.1e" % e for f, e in errs.items()})
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, (what, bad)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("turb", [0, 1])
def test_one_reverse_step_equals_oracle_adjoint(seed, turb):
    cfg, phi, st, a = _case(seed, turb)
    fields = state_fields(cfg)
    adj, phibar, _ = adjoint_steps(cfg, st, phi, a)
    g = _grid(cfg, phi, st)
    pb = torch.zeros(phi.shape, dtype=torch.float64, device="cuda:0")
    out = g.adjoint_step([torch.as_tensor(st[f]) for f in fields], [torch.as_tensor(a[f]) for f in fields], pb)
    got = dict(zip(fields, out))
    got["phi"] = pb
    ref = dict(adj, phi=phibar)
    _compare("seed %d turb %d one step" % (seed, turb), got, ref, 1e-9)
    g.close()


@pytest.mark.parametrize("seed,turb", [(4, 1), (5, 0)])
def test_four_step_reverse_chain_equals_oracle_adjoint(seed, turb):
    cfg, phi, st, a = _case(seed, turb)
    fields = state_fields(cfg)
    adj, phibar, _ = adjoint_steps(cfg, st, phi, a, nsteps=4)
    g = _grid(cfg, phi, st)
    states = [{f: torch.as_tensor(v).cuda() for f, v in st.items()}]
    for _ in range(4):
        g.step(1)
        states.append({f: v.clone() for f, v in g.state().items()})
    pb = torch.zeros(phi.shape, dtype=torch.float64, device="cuda:0")
    lam = [torch.as_tensor(a[f]).cuda() for f in fields]
    for n in range(3, -1, -1):
        lam = list(g.adjoint_step([states[n][f] for f in fields], lam, pb,
                                  after=[states[n + 1][f] for f in fields]))
    got = dict(zip(fields, lam))
    got["phi"] = pb
    _compare("seed %d turb %d four steps" % (seed, turb), got, dict(adj, phi=phibar), 1e-8)
    g.close()
