"""Host logic of the forward-difference optimiser (Sec. 4) on a closed form:
no GPU work is involved, the objective is a Python callable."""
import numpy as np

from oracle import fd_gradient
import paper_2204_01117_amd.optimize as O


def quad():
    c = np.array([1.0, 0.5, 2.0])
    s = np.array([0.2, 0.9, 0.4])
    return (lambda t: float(np.sum(c * (np.asarray(t) - s) ** 2))), c, s


def test_gradient_agrees_with_oracle_forward_differences():
    J, c, s = quad()
    t = np.array([0.7, 0.1, 0.35])
    for eps in (0.1, 1e-3):
        v, g = O.forward_difference_gradient(J, t, eps)
        v0, g0 = fd_gradient(J, t, eps)
        assert v == v0
        assert np.array_equal(g, g0)


def test_descent_converges_to_the_forward_difference_fixed_point():
    # the forward-difference gradient of the quadratic is 2c(t - s) + c eps,
    # zero at t = s - eps/2: the descent (minus sign) converges there
    J, c, s = quad()
    eps, lam = 0.1, 0.2
    theta, hist = O.gradient_descent(J, [1.0, -1.0, 0.0], eps=eps, lam=lam, iters=60)
    assert np.allclose(theta, s - eps / 2, atol=1e-8)
    values = [h[1] for h in hist]
    assert all(b < a for a, b in zip(values, values[1:]))
    assert len(hist) == 60


def test_descent_clips_to_bounds():
    J, c, s = quad()
    theta, hist = O.gradient_descent(J, [0.5, 0.5, 0.5], eps=0.1, lam=5.0, iters=1, lower=0.0, upper=1.0)
    step = 0.5 - 5.0 * hist[0][2]
    assert np.array_equal(theta, np.clip(step, 0.0, 1.0))
    assert ((theta >= 0) & (theta <= 1)).all()


class _ToyGrid:
    """A stand-in for Grid with a state-dependent map u <- u + dt (phi - u^3)
    on the u field (v, w, p carried along), J = sum(u^2) / 2, and the exact
    reverse of that map: checks the checkpoint-and-recompute schedule of
    AdjointObjective on the CPU (the reverse steps must see the states of
    their own forward steps, in reverse order)."""

    def __init__(self, m, dt):
        import torch
        self.torch, self.n, self.device, self.dt = torch, (m,), torch.device("cpu"), dt
        self.f = {k: torch.zeros(m, dtype=torch.float64) for k in ("u", "v", "w", "p", "k", "omega", "nut")}
        self.phi = torch.zeros(m, dtype=torch.float64)
        self.steps = 0
        self.reverse_inputs = []

    def state(self):
        return {k: v.clone() for k, v in self.f.items()}

    def set_state(self, st):
        for k, v in st.items():
            self.f[k] = self.torch.as_tensor(v, dtype=self.torch.float64).clone()

    def set_porosity(self, phi):
        self.phi = self.torch.as_tensor(phi, dtype=self.torch.float64).clone()

    def get_field(self, name):
        return self.f[name].clone()

    def adjoint_fields(self):
        return ("u", "v", "w")

    def extent(self, name):
        return (self.n[0], 1, 1)

    @property
    def dtype(self):
        return self.torch.float64

    def step(self, n=1, stats=False):
        for _ in range(n):
            u = self.f["u"]
            self.f["u"] = u + self.dt * (self.phi - u ** 3)
            self.f["p"] = self.f["p"] + 1.0
            self.steps += 1

    def objective(self, regions, u_target, grad=False):
        u = self.f["u"]
        J = float(0.5 * (u * u).sum())
        z = self.torch.zeros_like(u)
        return (J, (u.clone(), z, z)) if grad else J

    def adjoint_step(self, st, lam, phibar, after=None):
        u = st[0]
        self.reverse_inputs.append(float(u[0]))
        # the state handed over as the step's result is the step's result
        assert after is not None and self.torch.equal(after[0], u + self.dt * (self.phi - u ** 3))
        phibar += self.dt * lam[0]
        return (lam[0] * (1.0 - 3.0 * self.dt * u ** 2), lam[1], lam[2])


class _ToyDesign:
    def porosity(self, theta):
        return np.asarray(theta, dtype=np.float64)

    def gradient(self, theta, phibar):
        return phibar.numpy().copy()


def _toy_reference(theta, u0, dt, nsteps):
    us = [np.array(u0, dtype=np.float64)]
    for _ in range(nsteps):
        us.append(us[-1] + dt * (theta - us[-1] ** 3))
    lam, g = us[-1].copy(), np.zeros_like(theta)
    for u in reversed(us[:-1]):
        g += dt * lam
        lam = lam * (1.0 - 3.0 * dt * u ** 2)
    return 0.5 * float(np.sum(us[-1] ** 2)), g, [float(u[0]) for u in reversed(us[:-1])]


def test_adjoint_objective_checkpoint_schedule():
    import torch
    m, dt = 5, 0.1
    theta = np.linspace(0.2, 1.4, m)
    u0 = np.linspace(-0.5, 0.7, m)
    for nsteps, K in ((7, 3), (6, 3), (6, 20), (1, 1), (9, 1), (0, 4)):
        g = _ToyGrid(m, dt)
        g.f["u"] = torch.as_tensor(u0)
        A = O.AdjointObjective(g, _ToyDesign(), [], 0.0, nsteps=nsteps, checkpoint=K)
        J, grad = A.value_and_grad(theta)
        J0, g0, order = _toy_reference(theta, u0, dt, nsteps)
        assert abs(J - J0) <= 1e-14 * max(1.0, abs(J0))
        assert np.allclose(grad, g0, rtol=1e-13, atol=1e-15)
        assert g.reverse_inputs == order            # each reverse step saw its own state
        last = ((nsteps - 1) // K) * K if nsteps else 0
        assert g.steps == nsteps + last            # only the segments before the last are recomputed


def test_design_objective_is_a_torch_function():
    """design_objective wraps AdjointObjective for torch.autograd: the value
    and the gradient equal value_and_grad's."""
    import torch
    m, dt = 4, 0.1
    theta = torch.linspace(0.3, 1.1, m, dtype=torch.float64, requires_grad=True)
    g = _ToyGrid(m, dt)
    g.f["u"] = torch.linspace(-0.2, 0.5, m, dtype=torch.float64)
    A = O.AdjointObjective(g, _ToyDesign(), [], 0.0, nsteps=5, checkpoint=2)
    J = O.design_objective(theta, A)
    (gt,) = torch.autograd.grad(3.0 * J, theta)
    J0, g0, _ = _toy_reference(theta.detach().numpy(), np.linspace(-0.2, 0.5, m), dt, 5)
    assert abs(float(J.detach()) - J0) <= 1e-14 * max(1.0, abs(J0))
    assert np.allclose(gt.numpy(), 3.0 * g0, rtol=1e-13, atol=1e-15)


def test_adjoint_objective_keeps_every_state_when_it_fits():
    """checkpoint=None: the states fit (a host 'device' has no limit), so the
    sweep keeps them all and recomputes nothing; same gradient."""
    import torch
    m, dt, N = 5, 0.1, 7
    theta = np.linspace(0.2, 1.4, m)
    u0 = np.linspace(-0.5, 0.7, m)
    g = _ToyGrid(m, dt)
    g.f["u"] = torch.as_tensor(u0)
    A = O.AdjointObjective(g, _ToyDesign(), [], 0.0, nsteps=N)
    J, grad = A.value_and_grad(theta)
    J0, g0, order = _toy_reference(theta, u0, dt, N)
    assert A.segment == N and g.steps == N
    assert np.allclose(grad, g0, rtol=1e-13, atol=1e-15)
