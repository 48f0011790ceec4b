"""Pins of the oracle's isothermal three-velocity family (Sec. 2.3, Eq. 1d3v,
Table 3vel) and of its two-dimensional tensor product D2Q9 (Sec. 3.2)."""
import numpy as np
import pytest

import oracle
from paper_1402_5487_amd import inputs


@pytest.mark.parametrize("zeta", [3.0, 4.0, 5.0, 2.5])
def test_rule_is_eq_1d3v(zeta):
    """The Lagrange rule of {0, +-sqrt(zeta theta0)} with the isothermal
    Maxwell moments (mu_2 = theta0 + u^2) is the closed form the paper prints:
    r_i = w_i [1 + v_i u / theta0 + u^2 (v_i^2 - theta0) / ((zeta - 1) theta0^2)],
    w_1 = 1 - 1/zeta, w_2,3 = 1/(2 zeta)."""
    th0 = 0.3
    a = np.sqrt(zeta * th0)
    v = np.array([0.0, a, -a])
    c = oracle.lagrange_coeffs(v)
    w = np.array([1 - 1 / zeta, 1 / (2 * zeta), 1 / (2 * zeta)])
    for u in (-0.2, -0.05, 0.0, 0.1, 0.3):
        r = oracle.weights_1d(c, u, th0)
        closed = w * (1 + v * u / th0 + u * u * (v * v - th0) / ((zeta - 1) * th0 * th0))
        assert np.abs(r - closed).max() < 1e-14


def test_zeta3_rest_weights_are_lbgk_d2q9():
    """Table 3vel: zeta = 3 is the LBGK model; at rest its tensor product
    has the D2Q9 weights 4/9, 1/9, 1/36."""
    r = oracle.weights_1d(oracle.lagrange_coeffs([0, 1, -1]), 0.0, 1.0 / 3.0)
    w2 = np.outer(r, r)
    assert abs(w2[0, 0] - 4 / 9) < 1e-15
    assert abs(w2[0, 1] - 1 / 9) < 1e-15 and abs(w2[1, 0] - 1 / 9) < 1e-15
    assert abs(w2[1, 1] - 1 / 36) < 1e-15 and abs(w2[1, 2] - 1 / 36) < 1e-15


def _iso_lattice(n, zeta, omega, ny=None):
    return oracle.Lattice(2, n, n if ny is None else ny, v=[0, 1, -1], omega=omega,
                          theta0=1.0 / zeta)


@pytest.mark.parametrize("zeta", [3.0, 4.0])
def test_isothermal_step_conserves_mass_and_momentum(zeta):
    rng = np.random.default_rng(5)
    n = 12
    lat = _iso_lattice(n, zeta, 1.7)
    f = lat.init(1 + 0.05 * rng.standard_normal((n, n)), 0.05 * rng.standard_normal((n, n)),
                 0.05 * rng.standard_normal((n, n)), np.full((n, n), 1.0 / zeta))
    s0 = lat.sums(f)
    s1 = lat.sums(lat.step(f, 50))
    assert abs(s1[0] - s0[0]) < 1e-12 * s0[0]
    assert np.abs(s1[1:3] - s0[1:3]).max() < 1e-12 * s0[0]


def test_isothermal_equilibrium_is_a_fixed_point_of_uniform_flow():
    lat = _iso_lattice(6, 4.0, 1.3)
    ones = np.ones((6, 6))
    f = lat.init(ones, 0.07 * ones, -0.03 * ones, ones / 4.0)
    assert np.abs(lat.step(f, 7) - f).max() < 1e-15


@pytest.mark.parametrize("zeta,omega", [(3.0, 1.0), (4.0, 1.0), (3.0, 1.6), (4.0, 1.6)])
def test_viscosity_of_the_family(zeta, omega):
    """Shear wave u_x = U sin(2 pi y / L): amplitude decays as exp(-nu k^2 t)
    with nu = (1/omega - 1/2) theta0 in lattice units, which is the paper's
    (1/omega - 1/2) sqrt(theta0) dx / sqrt(zeta) for a = sqrt(zeta theta0) = 1."""
    L, U, steps = 64, 1e-4, 200
    lat = _iso_lattice(L, zeta, omega, ny=L)
    f = lat.init(*inputs.shear_wave(L, L, amp=U, theta=1.0 / zeta))
    y = np.arange(L)
    s = np.sin(2 * np.pi * y / L)

    def amp(g):
        return (lat.moments(g)[1].mean(axis=1) * s).sum() / (s * s).sum()

    a0 = amp(f)
    a1 = amp(lat.step(f, steps))
    k = 2 * np.pi / L
    nu = -np.log(a1 / a0) / (k * k * steps)
    nu_closed = (1 / omega - 0.5) / zeta
    assert abs(nu / nu_closed - 1) < (2e-3 if omega == 1.0 else 2e-2)


def test_viscosity_matched_omega_of_the_shear_layer_runs():
    """Sec. 3.2: equal viscosity (1/omega - 1/2) sqrt(theta0) dx / sqrt(zeta)
    for the LBGK at omega = 1.99880 and zeta = 4 gives the paper's 1.99862 to
    its printed precision (the exact value is 1.998614)."""
    w3 = 1.99880
    w4 = 1.0 / (0.5 + (1 / w3 - 0.5) * np.sqrt(4.0) / np.sqrt(3.0))
    assert abs(w4 - 1.99862) < 1e-5
    # and the step counts of equal physical time: dt scales as 1/sqrt(zeta)
    assert round(500 * np.sqrt(4.0 / 3.0)) == 577 and round(1500 * np.sqrt(4.0 / 3.0)) == 1732


def _shear_layer(zeta, omega, steps, n=128, l0=80.0):
    """The paper's shear layer (Sec. 3.2): l0 = 80, eps = 0.05, u0 = 0.069,
    the perturbation's phase x + 1/4, on an n x n periodic grid.  u0 is read
    in the paper's velocity unit sqrt(theta0) (it writes every velocity as
    v / sqrt(theta0)), so in this model's lattice units u0 / sqrt(zeta);
    returns |u| in units of sqrt(theta0) and (ux, uy) at each requested
    step."""
    th0 = 1.0 / zeta
    u0 = 0.069 * np.sqrt(th0)
    lat = _iso_lattice(n, zeta, omega)
    f = lat.init(*inputs.kelvin_helmholtz(n, n, u0=u0, delta=n / l0, theta=th0,
                                          uy_amp=0.05 * u0, phase=np.pi / 2))
    out, t = {}, 0
    for st in steps:
        f = lat.step(f, st - t)
        t = st
        _, ux, uy, _ = lat.moments(f)
        out[st] = (ux / np.sqrt(th0), uy / np.sqrt(th0))
    return out


def _high_k_share(ux, uy):
    n = ux.shape[0]
    spec = np.abs(np.fft.fft2(ux)) ** 2 + np.abs(np.fft.fft2(uy)) ** 2
    k = np.abs(np.fft.fftfreq(n))
    kk = np.maximum(k[:, None], k[None, :])
    return spec[kk >= 0.25].sum() / spec.sum()


def test_shear_layer_lbgk_and_zeta4_agree_and_zeta4_is_more_stable():
    """Sec. 3.2, Fig. LPViscosityMatch2d at all its step pairs (LBGK step n =
    zeta-4 step n sqrt(4/3)): at 500 / 577 the two models' velocity
    amplitudes agree; at 1500 / 1732 the LBGK run carries several times the
    zeta-4 run's share of energy at wavelengths below 4 nodes (the paper
    finds the first run far less stable than the second); at 1800 / 2078 the LBGK
    field is noise while the zeta-4 run still holds its vortices (finite,
    grid-scale share under 1 %, speeds of order u0)."""
    w3 = 1.99880
    w4 = 1.0 / (0.5 + (1 / w3 - 0.5) * 2.0 / np.sqrt(3.0))
    a = _shear_layer(3.0, w3, [500, 1500, 1800])
    b = _shear_layer(4.0, w4, [577, 1732, 2078])
    m3 = np.hypot(*a[500])
    m4 = np.hypot(*b[577])
    assert np.linalg.norm(m3 - m4) / np.linalg.norm(m3) < 0.01
    assert _high_k_share(*a[500]) < 1e-4 and _high_k_share(*b[577]) < 1e-4
    h3, h4 = _high_k_share(*a[1500]), _high_k_share(*b[1732])
    assert h3 > 5e-3 and h4 < 3e-3 and h3 > 4 * h4, (h3, h4)
    noise, kept = a[1800], b[2078]
    assert _high_k_share(*noise) > 0.3
    assert np.isfinite(kept[0]).all() and _high_k_share(*kept) < 0.01
    assert np.hypot(*kept).max() < 3 * 0.069


def _grid_errors(zeta, l0, sizes=(16, 32, 64, 128)):
    """Errors of |u| on n x n grids against the 128 x 128 grid at the same
    physical time, at the nodes the grids share (node i of an n grid sits at
    x = i / n).  Acoustic scaling: one lattice velocity for every grid (the
    paper's u0), the physical viscosity of the 128 grid's LBGK at
    omega = 1.99880 (lattice viscosity proportional to n), and the physical
    time of LBGK step 500 on the 128 grid (steps proportional to n)."""
    th0 = 1.0 / zeta
    nu128 = (1 / 1.99880 - 0.5) / 3.0 * np.sqrt(3.0 / zeta)    # same physical viscosity
    out = {}
    for n in sizes:
        omega = 1.0 / (0.5 + nu128 * n / 128 / th0)
        steps = int(round(500 * n / 128 * np.sqrt(zeta / 3.0)))
        ux, uy = _shear_layer(zeta, omega, [steps], n=n, l0=l0)[steps]
        out[n] = np.hypot(ux, uy)
    ref = out[128]
    return [np.linalg.norm(out[n] - ref[::128 // n, ::128 // n]) /
            np.linalg.norm(ref[::128 // n, ::128 // n]) for n in sizes[:-1]]


@pytest.mark.parametrize("zeta", [3.0, 4.0])
def test_shear_layer_grid_convergence(zeta):
    """Fig. LPConvergence: errors of the velocity amplitude on 16^2, 32^2 and
    64^2 grids against 128^2, for the LBGK D2Q9 and the zeta = 4 model; the
    paper reports second order.  The paper gives neither the time nor the
    scaling of the study (readings: acoustic scaling, the physical time of
    LBGK step 500).  With its l0 = 80 the layers are 0.2-1.6 nodes thick on
    these grids: the errors fall with resolution, and the order reaches
    1.6-1.8 between 32^2 and 64^2.  With resolved layers (l0 = 20) the
    order is 1.8-3 at both pairs: second order or better."""
    lit = _grid_errors(zeta, 80.0)
    assert lit[0] > lit[1] > lit[2]
    assert np.log2(lit[1] / lit[2]) > 1.5, lit
    res = _grid_errors(zeta, 20.0)
    orders = [np.log2(res[i] / res[i + 1]) for i in range(2)]
    assert min(orders) > 1.7 and max(orders) < 3.2, (res, orders)


def _shock_tube_q3(zeta, omega, steps, n=1000, rho_l=6.0, rho_r=1.0):
    """Sec. 3.2 shock tube on D1Q3: left half rho_L, right half rho_R, at
    rest, theta = theta0 = 1/zeta; returns (rho, u / sqrt(theta0))."""
    th0 = 1.0 / zeta
    lat = oracle.Lattice(1, n, v=[0, 1, -1], omega=omega, bc=1, theta0=th0)
    rho, ux, _, _ = inputs.shock_tube(n, rho_l=rho_l, theta_l=th0, rho_r=rho_r, theta_r=th0)
    f = lat.step(lat.init(rho, ux, None, np.full(n, th0)), steps)
    r, u, _, _ = lat.moments(f)
    return r, u / np.sqrt(th0)


def test_d1q3_zeta4_shock_tube_matches_exact_and_paper():
    """Sec. 3.2: rho_L / rho_R = 6, zeta = 4 at omega = 4 sqrt 3 - 6 (viscosity
    of the LBGK at omega = 1), 418 iterations.  The isothermal exact Riemann
    solution (gamma = 1; p*/p_R = 2.41 as in Table Rankine) gives the plateau
    velocity and the shock position; the paper marks u = 0.91 and x = 826
    (nodes numbered from 1)."""
    from oracle import riemann
    steps = 418
    r, u = _shock_tube_q3(4.0, 4 * np.sqrt(3) - 6, steps)
    s = riemann.star_state(6.0, 0.0, 6.0, 1.0, 0.0, 1.0, 1.0)
    assert abs(s.p - 2.41) < 0.005
    plateau = u[700:760]
    assert abs(plateau.mean() / s.u - 1) < 2e-3 and plateau.std() < 1e-3
    assert abs(plateau.mean() - 0.91) < 0.005
    speed = s.u * s.rho_r / (s.rho_r - 1.0) * np.sqrt(0.25)      # nodes per step
    mid = 0.5 * (s.rho_r + 1.0)
    i = int(np.where(r[600:] < mid)[0][0]) + 600
    front = i - 1 + (r[i - 1] - mid) / (r[i - 1] - r[i])
    assert abs(front - (499.5 + speed * steps)) < 1.5
    assert abs((front + 1) - 826) < 3
    # monotone profile: total variation of the exact solution is 2 u*
    assert np.abs(np.diff(u)).sum() < 1.02 * 2 * s.u


def test_d1q3_weak_shock_tube_nu_and_nu_hat():
    """Sec. 3.2, rho_L / rho_R = 1.1 (the figures of the weak shock tube and of
    the viscosity match): at the viscosity-matched omega = 4 sqrt 3 - 6 the
    zeta = 4 model differs from the LBGK (omega = 1) by about 0.3 % in density
    and about 0.003 in u / sqrt(theta0); matching instead with
    nu_hat = nu (zeta - 1) / 2, which accounts for mu_hat_3 = zeta theta0 u,
    makes the difference much smaller.  Same step counts as the ratio-6 tube
    (362 LBGK, 418 zeta = 4)."""
    r3, u3 = _shock_tube_q3(3.0, 1.0, 362, rho_l=1.1)
    r4, u4 = _shock_tube_q3(4.0, 4 * np.sqrt(3) - 6, 418, rho_l=1.1)
    # nu_hat of zeta = 4 equal to nu of the LBGK at omega = 1
    w_hat = 1.0 / (0.5 + 0.5 * (2.0 / np.sqrt(3.0)) * (2.0 / 3.0))
    r4h, u4h = _shock_tube_q3(4.0, w_hat, 418, rho_l=1.1)
    d_rho = np.abs((r4 - r3) / r3).max()
    d_u = np.abs(u4 - u3).max()
    assert 0.002 < d_rho < 0.004 and 0.002 < d_u < 0.004, (d_rho, d_u)
    d_rho_h = np.abs((r4h - r3) / r3).max()
    d_u_h = np.abs(u4h - u3).max()
    assert d_rho_h < d_rho / 10 and d_u_h < d_u / 10, (d_rho_h, d_u_h)


def test_d1q3_lbgk_shock_tube_oscillates():
    """Sec. 3.2: the LBGK model (zeta = 3, omega = 1, 362 iterations, the same
    physical time) gives an oscillating profile for the same shock tube."""
    _, u = _shock_tube_q3(3.0, 1.0, 362)
    assert np.abs(np.diff(u)).sum() > 10 * 2 * 0.9103
