"""Pins of the oracle against the paper's accuracy table (the moments each
model's rule reproduces, Sec. 3.3) and its thermal conductivity
kappa = (d + 2) / 2 nu rho (Sec. 2.1)."""
import numpy as np
import pytest

import oracle


def _mu_hat(v, theta, u, n):
    c = oracle.lagrange_coeffs(v)
    r = oracle.weights_1d(c, u, theta)
    return float((r * np.asarray(v, dtype=float) ** n).sum())


@pytest.mark.parametrize("u", [-0.3, -0.07, 0.0, 0.05, 0.21])
def test_accuracy_table_rows(u):
    """The table's 2nd- to 4th-order moments of each model's rule, written
    in terms of theta0 (isothermal models) or theta (the thermal one):
      LBGK (zeta = 3):       theta0 + u^2,  3 theta0 u
      parametric zeta = 4:   theta0 + u^2,  4 theta0 u
      parametric 4-vel.:     theta0 + u^2,  3 theta0 u + u^3
      parametric 5-vel.:     theta + u^2,   3 theta u + u^3,
                             3 theta^2 + 6 theta u^2 + u^4"""
    th0 = 0.3
    for zeta, third in ((3.0, 3.0 * th0 * u), (4.0, 4.0 * th0 * u)):
        a = np.sqrt(zeta * th0)
        v = [0.0, a, -a]
        assert abs(_mu_hat(v, th0, u, 2) - (th0 + u * u)) < 1e-14
        assert abs(_mu_hat(v, th0, u, 3) - third) < 1e-14
    # four velocities +-a, +-3a with a = sqrt(3 theta0) / 2
    a = np.sqrt(3.0 * th0) / 2.0
    v4 = [a, -a, 3 * a, -3 * a]
    assert abs(_mu_hat(v4, th0, u, 2) - (th0 + u * u)) < 1e-14
    assert abs(_mu_hat(v4, th0, u, 3) - (3 * th0 * u + u ** 3)) < 1e-14
    # five velocities, thermal: the moments at the local temperature
    th = 0.45
    v5 = [0.0, 1.0, -1.0, 3.0, -3.0]
    assert abs(_mu_hat(v5, th, u, 2) - (th + u * u)) < 1e-14
    assert abs(_mu_hat(v5, th, u, 3) - (3 * th * u + u ** 3)) < 1e-14
    assert abs(_mu_hat(v5, th, u, 4) - (3 * th * th + 6 * th * u * u + u ** 4)) < 1e-13


def _entropy_wave_rate(dim, omega, L, steps, th0=0.5, eps=1e-4):
    """Decay rate / (nu k^2) of an isobaric temperature wave at rest.  The
    entropy perturbation s = theta'/theta0 - (gamma - 1) rho'/rho0, with
    gamma = (d + 2) / d, is zero in the acoustic modes, so it isolates the
    entropy mode, which decays as exp(-kappa / (rho c_p) k^2 t)."""
    x = np.arange(L)
    th = th0 * (1 + eps * np.sin(2 * np.pi * x / L))
    gm1 = 2.0 / dim
    if dim == 2:
        th2 = np.tile(th, (4, 1))
        rho = th0 / th2
        lat = oracle.Lattice(2, L, 4, omega=omega)
        f = lat.init(rho, 0 * rho, 0 * rho, th2)

        def amp(g):
            m = lat.moments(g)
            s = (m[3].mean(axis=0) - th0) / th0 - gm1 * (m[0].mean(axis=0) - 1)
            return s @ np.sin(2 * np.pi * x / L)
    else:
        rho = th0 / th
        lat = oracle.Lattice(1, L, omega=omega, bc=0)
        f = lat.init(rho, 0 * rho, None, th)

        def amp(g):
            m = lat.moments(g)
            return ((m[3] - th0) / th0 - gm1 * (m[0] - 1)) @ np.sin(2 * np.pi * x / L)
    a0, a1 = amp(f), amp(lat.step(f, steps))
    k = 2 * np.pi / L
    nu = (1 / omega - 0.5) * th0
    return -np.log(a1 / a0) / (k * k * steps) / nu


@pytest.mark.parametrize("dim", [1, 2])
def test_thermal_conductivity_gives_unit_prandtl_number(dim):
    """kappa = (d + 2) / 2 nu rho with c_p = (d + 2) / 2 gives a thermal
    diffusivity equal to nu: the entropy mode decays at nu k^2 (to 3e-3 at
    omega = 1, L = 64; second-order convergence at omega = 1.6)."""
    assert abs(_entropy_wave_rate(dim, 1.0, 64, 300) - 1) < 5e-3
    e64 = abs(_entropy_wave_rate(dim, 1.6, 64, 300) - 1)
    e128 = abs(_entropy_wave_rate(dim, 1.6, 128, 1200) - 1)
    assert e128 < 5e-3 and 3.0 < e64 / e128 < 5.0
