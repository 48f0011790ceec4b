"""Pins of the closure oracle (oracle/closure.py): a library routine for the
convolution, finite differences for every gradient, the algebraic properties
of the projection, the closed form of Adam's first step, and conservation of
the restriction."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import closure as cl


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_scipy_correlate_wrap():
    x = _rand((7, 9, 3), 0)
    w = _rand((3, 3, 3, 4), 1)
    b = _rand(4, 2)
    out = cl.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(ndimage.correlate(x[:, :, i], w[:, :, i, o], mode="wrap")
                         for i in range(3))
        assert np.abs(out[:, :, o] - ref).max() < 1e-12


def _num_grad(f, a, eps=1e-6):
    g = np.zeros_like(a)
    it = np.nditer(a, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = a[i]
        a[i] = old + eps
        fp = f()
        a[i] = old - eps
        fm = f()
        a[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


def test_conv_backward_matches_finite_differences():
    x = _rand((5, 6, 2), 3)
    w = _rand((3, 3, 2, 3), 4)
    b = _rand(3, 5)
    dout = _rand((5, 6, 3), 6)

    def f():
        return (cl.conv3x3(x, w, b) * dout).sum()

    dx, dw, db = cl.conv3x3_backward(x, w, dout)
    assert np.abs(dx - _num_grad(f, x)).max() < 1e-6
    assert np.abs(dw - _num_grad(f, w)).max() < 1e-6
    assert np.abs(db - _num_grad(f, b)).max() < 1e-6


def test_network_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    params = [(rng.standard_normal((3, 3, 2, 3)) * 0.5, rng.standard_normal(3) * 0.1),
              (rng.standard_normal((3, 3, 3, 3)) * 0.5, rng.standard_normal(3) * 0.1),
              (rng.standard_normal((3, 3, 3, 2)) * 0.5, rng.standard_normal(2) * 0.1)]
    x = rng.standard_normal((4, 5, 2))
    dy = rng.standard_normal((4, 5, 2))

    def f():
        return (cl.forward(params, x)[0] * dy).sum()

    y, cache = cl.forward(params, x)
    grads = cl.backward(params, cache, dy)
    for (w, b), (gw, gb) in zip(params, grads):
        assert np.abs(gw - _num_grad(f, w)).max() < 1e-5
        assert np.abs(gb - _num_grad(f, b)).max() < 1e-5


@pytest.mark.parametrize("scaled", [False, True])
def test_projection_properties(scaled):
    s = np.random.default_rng(3).uniform(1e-6, 1.0, 25) if scaled else np.ones(25)
    P = cl.projection(s)
    phi = cl.conserved_basis()
    assert np.abs(P @ P - P).max() < 1e-12
    assert np.abs(P - P.T).max() < 1e-12
    # the physical correction s * (P y) has zero mass, momentum and energy
    y = np.random.default_rng(4).standard_normal(25)
    assert np.abs(phi.T @ (s * (P @ y))).max() < 1e-12 * np.abs(s * y).max() * 100
    assert round(np.trace(P)) == 21
    # closest conserving vector in the metric sum (x/s)^2: P y - y is
    # orthogonal to every admissible direction
    q = np.random.default_rng(5).standard_normal(25)
    adm = s * (P @ q)
    assert abs(((P @ y - y) * (adm / s)).sum()) < 1e-10


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(9)
    y = rng.standard_normal((3, 4, 25))
    t = rng.standard_normal((3, 4, 25)) * 0.3
    s = rng.uniform(0.2, 2.0, 25)
    _, g = cl.loss_and_grad(y, t, s)
    num = _num_grad(lambda: cl.loss_and_grad(y, t, s)[0], y)
    assert np.abs(g - num).max() < 1e-6


def test_loss_ignores_what_no_admissible_correction_can_reach():
    """The loss compares with the closest admissible (moment-free) correction
    in the metric sum (x/s)^2; a target in the removed directions
    s^2 * (Phi a) has the zero correction as its closest point."""
    s = np.random.default_rng(2).uniform(0.01, 1.0, 25)
    t = (np.random.default_rng(1).standard_normal((2, 2, 4)) @ cl.conserved_basis().T) * s ** 2
    loss, _ = cl.loss_and_grad(np.zeros((2, 2, 25)), t, s)
    assert loss < 1e-22


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = cl.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    assert np.abs((p1 - p) + 0.01 * np.sign(g)).max() < 1e-9


def test_restriction_conserves_and_is_exact_for_uniform():
    rng = np.random.default_rng(2)
    rho = 1 + 0.1 * rng.standard_normal((8, 12))
    ux, uy = 0.05 * rng.standard_normal((2, 8, 12))
    th = 0.35 + 0.01 * rng.standard_normal((8, 12))
    e = rho * (2 * th + ux ** 2 + uy ** 2)
    r, u, w, t = cl.restrict(rho, rho * ux, rho * uy, e)
    assert abs(r.sum() * 16 - rho.sum()) < 1e-12
    assert abs((r * u).sum() * 16 - (rho * ux).sum()) < 1e-12
    E = r * (2 * t + u * u + w * w)
    assert abs(E.sum() * 16 - e.sum()) < 1e-11
    one = np.ones((8, 12))
    r, u, w, t = cl.restrict(one, 0.1 * one, -0.2 * one, one * (2 * 0.4 + 0.05))
    assert np.abs(u - 0.1).max() < 1e-15 and np.abs(t - 0.4).max() < 1e-15
