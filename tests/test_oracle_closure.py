"""Pins of the closure oracle (oracle/closure.py): a library routine for the
convolution, finite differences for every gradient, the algebraic properties
of the projection, streaming and the equilibrium's moments against the
lattice oracle, the invariants of the equilibrium shift, the closed form of
Adam's first step, and conservation of the restriction."""
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


def test_pull_is_the_oracle_step_without_collision():
    """With omega = 0 the collision is the identity, so one step of the
    lattice oracle (push form) is pure streaming: the same map as pull."""
    import oracle
    rng = np.random.default_rng(11)
    H, W = 7, 9
    P = rng.standard_normal((H, W, 25))
    lat = oracle.Lattice(2, W, H, omega=0.0)
    ref = lat.step(np.transpose(P, (2, 0, 1)))
    assert np.abs(cl.pull(P) - np.transpose(ref, (1, 2, 0))).max() == 0.0
    # and brute force on the definition f_k(y, x) = P_k(y - v_y, x - v_x)
    v = cl.velocities_2d().astype(int)
    f = cl.pull(P)
    for k in (0, 3, 8, 19, 24):
        for y in range(H):
            for x in range(W):
                assert f[y, x, k] == P[(y - v[k, 1]) % H, (x - v[k, 0]) % W, k]


def test_push_is_the_adjoint_of_pull():
    a = _rand((5, 8, 25), 12)
    b = _rand((5, 8, 25), 13)
    assert abs((cl.pull(a) * b).sum() - (a * cl.push(b)).sum()) < 1e-11


def test_conserved_matches_lattice_sums_of_the_equilibrium():
    """E = rho (2 theta + |u|^2) is what the D2Q25 equilibrium's populations
    carry (the moments of f_eq are exact to fourth order per direction)."""
    import oracle
    rho, ux, uy, th = 1.3, 0.07, -0.11, 0.41
    lat = oracle.Lattice(2, 4, 3, v=[0, 1, -1, 3, -3])
    ones = np.ones((3, 4))
    f = lat.init(rho * ones, ux * ones, uy * ones, th * ones)
    sums = lat.sums(f) / 12
    c = cl.conserved(np.array(rho), np.array(ux), np.array(uy), np.array(th))
    assert np.abs(sums - c).max() < 1e-14


def test_increment_error_special_cases():
    rng = np.random.default_rng(14)
    a = tuple(1 + 0.1 * rng.standard_normal((3, 4)) for _ in range(4))
    b = tuple(1 + 0.1 * rng.standard_normal((3, 4)) for _ in range(4))
    assert np.abs(cl.increment_error(a, b, a, b)).max() == 0.0     # model == truth
    assert np.abs(cl.increment_error(a, a, b, b)).max() == 0.0     # nothing changes
    d = cl.increment_error(a, b, a, a)                              # only the truth moves
    assert np.abs(d - (cl.conserved(*b) - cl.conserved(*a))).max() < 1e-15


def test_moment_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(9)
    y = rng.standard_normal((5, 7, 25))
    d = rng.standard_normal((5, 7, 4)) * 0.3
    s = rng.uniform(0.2, 2.0, 25)
    ms = rng.uniform(0.5, 2.0, 4)
    for reg in (0.0, 0.3):
        _, g, _, _ = cl.moment_loss_and_grad(y, d, s, ms, reg)
        num = _num_grad(lambda: cl.moment_loss_and_grad(y, d, s, ms, reg)[0], y)
        assert np.abs(g - num).max() < 1e-6 * max(1.0, np.abs(g).max())


def test_minimum_norm_term_is_the_projected_output_norm():
    """With d = 0 and unit loss weights the loss is the streamed moments'
    energy plus beta |Ph y|^2; the second term alone is beta * |y|^2 for y
    already moment-free in the scaled metric."""
    rng = np.random.default_rng(17)
    s = rng.uniform(0.1, 1.0, 25)
    y0 = rng.standard_normal((4, 5, 25)) @ cl.projection(s)          # Ph y0 = y0
    l0 = cl.moment_loss_and_grad(y0, np.zeros((4, 5, 4)), s, np.ones(4))[0]
    l1 = cl.moment_loss_and_grad(y0, np.zeros((4, 5, 4)), s, np.ones(4), 0.7)[0]
    assert abs((l1 - l0) - 0.7 * (y0 ** 2).sum() / 20) < 1e-12


def test_corrected_streaming_conserves_domain_totals():
    """A node-wise moment-free correction, streamed, leaves the totals of
    mass, momentum and energy unchanged; a spatially uniform residual
    therefore has no gradient."""
    rng = np.random.default_rng(15)
    s = rng.uniform(0.1, 1.0, 25)
    y = rng.standard_normal((6, 8, 25))
    _, _, c, _ = cl.moment_loss_and_grad(y, np.zeros((6, 8, 4)), s, np.ones(4))
    assert np.abs((cl.pull(c) @ cl.conserved_basis()).sum(axis=(0, 1))).max() < 1e-12
    # the flux form telescopes for any c, moment-free or not
    e = rng.standard_normal((6, 8, 25))
    assert np.abs(cl.streamed_moments(e).sum(axis=(0, 1))).max() < 1e-11
    d = np.broadcast_to(rng.standard_normal(4), (6, 8, 4))
    loss, g, _, _ = cl.moment_loss_and_grad(np.zeros((6, 8, 25)), d, s, np.ones(4))
    assert abs(loss - (d[0, 0] ** 2).sum()) < 1e-12
    assert np.abs(g).max() < 1e-13


def test_equilibrium_shift_moves_only_the_conserved_moments():
    """After the shift the pulled populations carry exactly the node moments
    m + g, their non-equilibrium part f - f_eq is unchanged, and the domain
    totals are conserved (the equilibrium reproduces its own mass, momentum
    and energy, checked through the lattice oracle's moments)."""
    import oracle
    rng = np.random.default_rng(16)
    H, W = 6, 7
    lat = oracle.Lattice(2, W, H, v=[0, 1, -1, 3, -3])
    fields = (1 + 0.01 * rng.standard_normal((H, W)), 0.05 * rng.standard_normal((H, W)),
              0.05 * rng.standard_normal((H, W)), 0.35 + 0.01 * rng.standard_normal((H, W)))
    nodes = lambda a: np.ascontiguousarray(np.transpose(a, (2, 0, 1)))
    back = lambda a: np.transpose(a, (1, 2, 0))
    P = cl.push(back(lat.init(*fields))) + 1e-4 * rng.standard_normal((H, W, 25))
    s = rng.uniform(1e-4, 1e-3, 25)
    c = s * (rng.standard_normal((H, W, 25)) @ cl.projection(s))
    P1 = cl.equilibrium_shift(P, c, lat)
    f0, f1 = cl.pull(P), cl.pull(P1)
    m0 = cl.conserved(*lat.moments(nodes(f0)))
    m1 = cl.conserved(*lat.moments(nodes(f1)))
    g = cl.streamed_moments(c)
    assert np.abs(g - cl.pull(c) @ cl.conserved_basis()).max() < 1e-15    # c is moment-free
    assert np.abs(m1 - (m0 + g)).max() < 1e-14
    neq0 = f0 - back(lat.init(*lat.moments(nodes(f0))))
    neq1 = f1 - back(lat.init(*lat.moments(nodes(f1))))
    assert np.abs(neq1 - neq0).max() < 1e-15
    assert np.abs(lat.sums(nodes(P1)) - lat.sums(nodes(P))).max() < 1e-13
    # no correction, no change
    assert np.abs(cl.equilibrium_shift(P, 0 * c, lat) - P).max() == 0.0


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
