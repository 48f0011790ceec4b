"""Pins of the adjoint oracle (oracle/adjoint.py): each vector-Jacobian
product against central finite differences of the oracle's own forward map
(the dot-product test <lam, J d> = <J^T lam, d> for random lam and d), and
the forward maps against the lattice and closure oracles they restate."""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from oracle import closure as ocl

H, W = 6, 7


def _state(seed, amp=0.03):
    rng = np.random.default_rng(seed)
    rho = 1 + amp * rng.standard_normal((H, W))
    ux, uy = amp * rng.standard_normal((H, W)), amp * rng.standard_normal((H, W))
    th = 0.35 + 0.2 * amp * rng.standard_normal((H, W))
    lat = oracle.Lattice(2, W, H, omega=1.8)
    f = lat.init(rho, ux, uy, th)                      # (25, H, W), pre-collision
    # a post-collision buffer whose pull is f, plus a non-equilibrium part
    S = np.transpose(f, (1, 2, 0)) + 1e-3 * rng.standard_normal((H, W, 25))
    return ocl.push(S), rng


def _dot_test(fwd, vjp_val, x, d, h):
    fd = (fwd(x + h * d) - fwd(x - h * d)) / (2 * h)
    return fd, vjp_val


def test_equilibrium_restates_the_lattice_oracle():
    P, _ = _state(0)
    S = ocl.pull(P)
    m = S @ ocl.conserved_basis()
    lat = oracle.Lattice(2, W, H)
    ref = np.transpose(lat.init(*adj.primitive(m)), (1, 2, 0))
    assert np.abs(adj.equilibrium(m) - ref).max() < 1e-15


def test_step_is_the_oracle_step():
    P, _ = _state(1)
    lat = oracle.Lattice(2, W, H, omega=1.8)
    want = lat.step(np.transpose(ocl.pull(P), (2, 0, 1)), 1)
    got = np.transpose(ocl.pull(adj.step(P, 1.8)), (2, 0, 1))
    # the lattice oracle takes theta from sum f |v - u|^2, this one from
    # E = sum f |v|^2: the same quantity, rounded in a different order
    assert np.abs(got - want).max() < 1e-14


def test_shift_is_the_closure_oracle_apply():
    P, rng = _state(2)
    cc = 1e-4 * rng.standard_normal((H, W, 25))
    cc = cc @ ocl.projection().T          # moment-free, as the network makes it
    lat = oracle.Lattice(2, W, H)
    assert np.abs(adj.shift(P, cc) - ocl.equilibrium_shift(P, cc, lat)).max() < 1e-15


@pytest.mark.parametrize("seed", [3, 4])
def test_equilibrium_vjp_dot_product(seed):
    P, rng = _state(seed)
    m = ocl.pull(P) @ ocl.conserved_basis()
    lam = rng.standard_normal((H, W, 25))
    d = rng.standard_normal((H, W, 4)) * np.array([1e-2, 1e-2, 1e-2, 1e-2])
    h = 1e-4
    fd = (adj.equilibrium(m + h * d) - adj.equilibrium(m - h * d)) / (2 * h)
    lhs = (lam * fd).sum()
    rhs = (adj.equilibrium_vjp(m, lam) * d).sum()
    assert abs(lhs - rhs) < 1e-7 * (abs(lhs) + 1e-12), (lhs, rhs)


@pytest.mark.parametrize("omega", [1.0, 1.8])
def test_step_vjp_dot_product(omega):
    P, rng = _state(5)
    lam = rng.standard_normal((H, W, 25))
    d = 1e-2 * rng.standard_normal((H, W, 25))
    h = 1e-4
    fd = (adj.step(P + h * d, omega) - adj.step(P - h * d, omega)) / (2 * h)
    lhs = (lam * fd).sum()
    rhs = (adj.step_vjp(P, lam, omega) * d).sum()
    assert abs(lhs - rhs) < 1e-7 * abs(lhs), (lhs, rhs)


def test_shift_vjp_dot_product():
    P, rng = _state(6)
    cc = 1e-3 * rng.standard_normal((H, W, 25))
    lam = rng.standard_normal((H, W, 25))
    dP, dc = adj.shift_vjp(P, cc, lam)
    h = 1e-5
    d = 1e-2 * rng.standard_normal((H, W, 25))
    fd = (adj.shift(P + h * d, cc) - adj.shift(P - h * d, cc)) / (2 * h)
    lhs, rhs = (lam * fd).sum(), (dP * d).sum()
    assert abs(lhs - rhs) < 1e-7 * abs(lhs), ("P", lhs, rhs)
    e = 1e-3 * rng.standard_normal((H, W, 25))
    fd = (adj.shift(P, cc + h * e) - adj.shift(P, cc - h * e)) / (2 * h)
    lhs, rhs = (lam * fd).sum(), (dc * e).sum()
    assert abs(lhs - rhs) < 1e-6 * abs(lhs), ("c", lhs, rhs)


def test_moment_loss_gradient_dot_product():
    P, rng = _state(7)
    tgt = ocl.pull(P) @ ocl.conserved_basis() + 1e-3 * rng.standard_normal((H, W, 4))
    w = np.array([1.0, 2.0, 3.0, 0.5])
    loss, g = adj.moment_loss(P, tgt, w)
    d = rng.standard_normal((H, W, 25))
    h = 1e-6
    fd = (adj.moment_loss(P + h * d, tgt, w)[0] - adj.moment_loss(P - h * d, tgt, w)[0]) / (2 * h)
    assert abs(fd - (g * d).sum()) < 1e-6 * abs(fd)
    assert loss > 0
