"""Forward-difference gradient descent over design parameters (Sec. 4).

The paper's optimisation routine evaluates the objective by simulating the
flow for a design, estimates each partial derivative from one more
simulation with that parameter moved by eps (forward differences, so N + 1
simulations per iteration for N parameters), and moves the parameters by
lam times that gradient.  Printed with a plus sign, the update only
decreases the objective with a minus sign; ``gradient_descent`` takes the
descent form.  Defaults are the paper's eps = 0.1 and lam = 1.0.

``AdjointObjective`` gives the same gradient from one forward and one
reverse run (the discrete adjoint, uf_adjoint_step), whatever the number of
parameters -- an extension: the paper differences the simulator.

Every simulation runs on the GPU through :class:`Grid`; this module is host
control flow only.
"""
import numpy as np


class SimulationObjective:
    """theta -> objective of the flow after ``nsteps`` steps.

    Each call restores the state the grid held at construction (or
    ``initial_state``), sets the porosity ``porosity_of(theta)`` (an
    (nx, ny, nz) array, host or device), runs the steps and evaluates the
    target-region objective on the GPU.
    """

    def __init__(self, grid, porosity_of, regions=None, u_target=None, nsteps=0, initial_state=None, score=None):
        """``score(grid) -> float`` replaces the target-region objective when
        given (e.g. ``lambda g: g.plane_objective(1.5)``)."""
        self.grid = grid
        self.porosity_of = porosity_of
        self.regions = [tuple(tuple(int(x) for x in lohi) for lohi in box) for box in (regions or [])]
        self.u_target = float(u_target) if u_target is not None else 0.0
        self.score = score
        self.nsteps = int(nsteps)
        st = initial_state if initial_state is not None else grid.state()
        self.initial = {f: a.clone() if hasattr(a, "clone") else np.array(a) for f, a in st.items()}
        self.calls = 0

    def __call__(self, theta):
        g = self.grid
        g.set_state(self.initial)
        g.set_porosity(self.porosity_of(np.asarray(theta, dtype=np.float64)))
        if self.nsteps:
            g.step(self.nsteps, stats=False)
        self.calls += 1
        return self._score(g)

    def close(self):
        """Release the grids made for batched evaluations."""
        for g in getattr(self, "_pool", []):
            g.close()
        self._pool = []

    def _score(self, g):
        return self.score(g) if self.score is not None else g.objective(self.regions, self.u_target)

    def many(self, thetas):
        """The objective of several designs, simulated together
        (uf_step_batch, one grid and stream per design); each value equals
        what ``__call__`` returns for that design."""
        import torch
        from .grid import Grid, step_batch
        pool = getattr(self, "_pool", [])
        while len(pool) < len(thetas):
            pool.append(Grid(self.grid.cfg, device=self.grid.device, stream=torch.cuda.Stream(self.grid.device)))
        self._pool = pool
        grids = pool[:len(thetas)]
        for g, th in zip(grids, thetas):
            g.set_state(self.initial)
            g.set_porosity(self.porosity_of(np.asarray(th, dtype=np.float64)))
        if self.nsteps:
            step_batch(grids, self.nsteps, stats=False)
        self.calls += len(thetas)
        return [self._score(g) for g in grids]


class AdjointObjective:
    """theta -> (J, dJ/dtheta) of the flow after ``nsteps`` steps, the
    gradient by the discrete adjoint.

    ``design`` maps theta to porosity (``porosity(theta)``) and back
    (``gradient(theta, phibar)``), as :class:`BoxDesign` does.  The objective
    is the target-region one (``u_field`` None) or the field one
    (``u_field`` [3, nx, ny, nz]).  Checkpoint and recompute: the forward
    pass keeps the state every ``checkpoint`` steps and every state of the
    last segment; the reverse pass recomputes each earlier segment from its
    checkpoint (the forward is deterministic, so the recomputed states are
    the same bits) and runs the reverse steps over it, accumulating dJ/dphi.
    With the k-omega update in the step the reverse also carries k, omega
    and nu_t.
    """

    def __init__(self, grid, design, regions, u_target=0.55, nsteps=1, initial_state=None, checkpoint=None,
                 u_field=None, memory_fraction=0.25, plane=None):
        """``checkpoint``: steps per recomputed segment; None keeps every
        state of the horizon when they fit in ``memory_fraction`` of the
        GPU's free memory (no recompute at all), else checkpoints every 20
        steps.  ``plane``: keyword arguments of ``Grid.plane_objective``
        (z_plane, ...) to score the pedestrian plane instead of regions."""
        self.grid, self.design = grid, design
        self.regions = [tuple(tuple(int(x) for x in lohi) for lohi in box) for box in regions]
        self.u_target = float(u_target)
        self.u_field = u_field
        self.nsteps = int(nsteps)
        self.checkpoint = None if checkpoint is None else max(1, int(checkpoint))
        self.memory_fraction = float(memory_fraction)
        self.plane = dict(plane) if plane is not None else None
        st = initial_state if initial_state is not None else grid.state()
        self.initial = {f: a.clone() if hasattr(a, "clone") else np.array(a) for f, a in st.items()}
        self.calls = 0

    def _objective(self, grad, phibar=None):
        g = self.grid
        if self.plane is not None:
            return g.plane_objective(grad=grad, phibar=phibar, **self.plane)
        if self.u_field is not None:
            return g.field_objective(self.regions, self.u_field, grad=grad)
        return g.objective(self.regions, self.u_target, grad=grad)

    def _snapshot(self):
        return {f: self.grid.get_field(f) for f in ("u", "v", "w", "p", "k", "omega", "nut")}

    def __call__(self, theta):
        return self.value_and_grad(theta)[0]

    def _auto_checkpoint(self, fields):
        import torch
        g, N = self.grid, max(self.nsteps, 1)
        per_state = 0
        for f in fields:
            e = g.extent(f)
            per_state += e[0] * e[1] * e[2]
        per_state *= torch.finfo(g.dtype).bits // 8
        free = torch.cuda.mem_get_info(g.device)[0] if g.device.type == "cuda" else float("inf")
        return N if N * per_state <= self.memory_fraction * free else 20

    def value_and_grad(self, theta):
        import torch
        g, N = self.grid, self.nsteps
        theta = np.asarray(theta, dtype=np.float64)
        g.set_state(self.initial)
        g.set_porosity(self.design.porosity(theta))
        fields = g.adjoint_fields()
        K = self.checkpoint if self.checkpoint is not None else self._auto_checkpoint(fields)
        self.segment = K
        last = ((N - 1) // K) * K if N else 0
        ckpt, tail = {}, []
        for s in range(N):
            if s >= last:
                tail.append([g.get_field(f) for f in fields])
            elif s % K == 0:
                ckpt[s] = self._snapshot()
            g.step(1, stats=False)
        phibar = torch.zeros(g.n, dtype=torch.float64, device=g.device)
        J, lam = self._objective(grad=True, phibar=phibar)
        lam = tuple(lam) + tuple(torch.zeros_like(g.get_field(f)) for f in fields[3:])
        # each reverse step also gets the state its step produced: the one
        # the previous reverse step started from (the final state first)
        after = [g.get_field(f) for f in ("u", "v", "w")]
        for st in reversed(tail):
            lam = g.adjoint_step(st, lam, phibar, after=after)
            after = st
        for s0 in sorted(ckpt, reverse=True):
            g.set_state(ckpt[s0])
            states = []
            for _ in range(s0, min(s0 + K, N)):
                states.append([g.get_field(f) for f in fields])
                g.step(1, stats=False)
            for st in reversed(states):
                lam = g.adjoint_step(st, lam, phibar, after=after)
                after = st
        self.calls += 1
        self.phibar = phibar
        return J, self.design.gradient(theta, phibar)


def design_objective(theta, objective):
    """J(theta) as a differentiable torch scalar: the value and the adjoint
    gradient come from ``objective.value_and_grad`` (an AdjointObjective) in
    one call when the value is taken; backward multiplies the stored
    gradient by the incoming one.  ``theta``: a 1-D float64 tensor."""
    import torch

    class _Design(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            value, grad = objective.value_and_grad(t.detach().cpu().numpy())
            ctx.save_for_backward(torch.as_tensor(grad, dtype=t.dtype, device=t.device))
            return t.new_tensor(value)

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout * grad

    return _Design.apply(theta)


def forward_difference_gradient(J, theta, eps=0.1):
    """(J(theta), dJ/dtheta) by forward differences: N + 1 evaluations, all
    at once when J has a ``many`` method (the simulations are independent)."""
    theta = np.array(theta, dtype=np.float64)
    points = [theta]
    for n in range(theta.size):
        moved = theta.copy()
        moved.flat[n] += eps
        points.append(moved)
    if hasattr(J, "many"):
        values = [float(v) for v in J.many(points)]
    else:
        values = [float(J(p)) for p in points]
    base = values[0]
    grad = np.empty_like(theta)
    for n in range(theta.size):
        grad.flat[n] = (values[n + 1] - base) / eps
    return base, grad


def gradient_descent(J, theta0, eps=0.1, lam=1.0, iters=10, lower=None, upper=None, callback=None):
    """Descent theta <- theta - lam * grad, optionally clipped to
    [lower, upper] (porosity parameters live in [0, 1]).  The gradient comes
    from ``J.value_and_grad`` when J has one (the adjoint), else from
    forward differences of step eps.  Returns (final theta, history), the
    history a list of (theta, J(theta), grad) per iteration."""
    theta = np.array(theta0, dtype=np.float64)
    history = []
    for it in range(int(iters)):
        if hasattr(J, "value_and_grad"):
            value, grad = J.value_and_grad(theta)
        else:
            value, grad = forward_difference_gradient(J, theta, eps)
        history.append((theta.copy(), value, grad))
        if callback is not None:
            callback(it, theta, value, grad)
        theta = theta - lam * grad
        if lower is not None or upper is not None:
            theta = np.clip(theta, lower, upper)
    return theta, history
