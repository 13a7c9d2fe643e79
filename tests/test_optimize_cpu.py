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
