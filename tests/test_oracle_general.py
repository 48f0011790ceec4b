"""Pins of the oracle's step for general on-lattice velocity sets (Sec. 2.2:
any q distinct velocities give, through Eq. rdr, a rule matching the Maxwell
moments up to order q - 1).  Sets with q <= 4 are isothermal (the moments at
the fixed theta0, as for the three-velocity family), q >= 5 thermal."""
import numpy as np
import pytest

import oracle
from paper_1402_5487_amd import inputs

# name: (velocities, temperature, isothermal)
SETS = {
    # the paper's four-velocity on-lattice set: +-a, +-b with b = 3a and
    # a = sqrt(3 theta0) / 2, i.e. theta0 = 4/3 for a = 1
    "d1q4": ([1, -1, 3, -3], 4.0 / 3.0, True),
    # the asymmetric three-velocity example of Table 3vel, (0, 2, -4) sqrt(theta0),
    # on the lattice with sqrt(theta0) = 1/2
    "q3_asym": ([0, 1, -2], 0.25, True),
    "q5_asym": ([0, 1, -1, 2, -3], 0.7, False),
    "q6": ([0, 1, -1, 2, -2, 3], 0.5, False),
    "q7": ([0, 1, -1, 2, -2, 3, -3], 1.0, False),
}


def _lattice(name, n, omega, ny=None):
    v, th, iso = SETS[name]
    return oracle.Lattice(2, n, n if ny is None else ny, v=v, omega=omega,
                          theta0=th if iso else None)


def _gauss_moment(n, u, theta):
    """E[(u + sqrt(theta) z)^n], z standard normal, by 30-point Gauss-Hermite
    quadrature (exact for these polynomial degrees)."""
    z, w = np.polynomial.hermite_e.hermegauss(30)
    return float((w * (u + np.sqrt(theta) * z) ** n).sum() / w.sum())


@pytest.mark.parametrize("name", sorted(SETS))
def test_moment_identity_against_quadrature(name):
    """mu_hat_n = sum_i r_i v_i^n equals the Maxwell moment for n <= q - 1 and
    (for some state) not for n = q: the order the set buys (Sec. 2.2)."""
    v, th, _ = SETS[name]
    v = np.array(v, dtype=float)
    q = v.size
    c = oracle.lagrange_coeffs(v)
    miss = 0.0
    for u in (-0.2, -0.03, 0.0, 0.11, 0.25):
        for t in (0.6 * th, th, 1.4 * th):
            r = oracle.weights_1d(c, u, t)
            for n in range(q):
                want = _gauss_moment(n, u, t)
                assert abs((r * v ** n).sum() - want) < 1e-12 * max(1.0, abs(want)), (n, u, t)
            miss = max(miss, abs((r * v ** q).sum() - _gauss_moment(q, u, t)))
    assert miss > 1e-6


@pytest.mark.parametrize("name", sorted(SETS))
def test_step_conserves(name):
    """Periodic boundaries: mass and momentum for every set, the energy sum as
    well for the thermal ones (q >= 5 match mu_2 at the local temperature)."""
    v, th, iso = SETS[name]
    n = 10
    lat = _lattice(name, n, 1.3)
    rng = np.random.default_rng(len(v))
    f = lat.init(1 + 0.02 * rng.uniform(-1, 1, (n, n)), 0.03 * rng.uniform(-1, 1, (n, n)),
                 0.03 * rng.uniform(-1, 1, (n, n)), th * (1 + 0.02 * rng.uniform(-1, 1, (n, n))))
    s0 = lat.sums(f)
    s1 = lat.sums(lat.step(f, 20))
    assert abs(s1[0] - s0[0]) < 1e-12 * s0[0]
    assert np.abs(s1[1:3] - s0[1:3]).max() < 1e-12 * s0[0]
    if not iso:
        assert abs(s1[3] - s0[3]) < 1e-12 * s0[3]


@pytest.mark.parametrize("name", sorted(SETS))
def test_uniform_flow_is_a_fixed_point(name):
    _, th, _ = SETS[name]
    lat = _lattice(name, 6, 1.4)
    ones = np.ones((6, 6))
    f = lat.init(ones, 0.04 * ones, -0.02 * ones, th * ones)
    assert np.abs(lat.step(f, 5) - f).max() < 2e-14 * np.abs(f).max()


@pytest.mark.parametrize("name,tol", [("d1q4", 2e-3), ("q3_asym", 3e-3), ("q6", 1e-6),
                                      ("q7", 1e-6)])
def test_shear_wave_viscosity(name, tol):
    """u_x = U sin(2 pi y / L) decays as exp(-nu k^2 t), nu = (1/omega - 1/2) theta
    (theta0 for the isothermal sets), at omega = 1 and L = 64."""
    _, th, _ = SETS[name]
    L, U, steps = 64, 1e-4, 200
    lat = _lattice(name, L, 1.0)
    f = lat.init(*inputs.shear_wave(L, L, amp=U, theta=th))
    s = np.sin(2 * np.pi * np.arange(L) / L)

    def amp(g):
        return (lat.moments(g)[1].mean(axis=1) * s).sum() / (s * s).sum()

    a0, a1 = amp(f), amp(lat.step(f, steps))
    k = 2 * np.pi / L
    nu = -np.log(a1 / a0) / (k * k * steps)
    assert abs(nu / (0.5 * th) - 1) < tol
